"""Data collection, training and evaluation of the learned cost model.

The network, its training loop and its inference run in libtgemm.so
(tgemm_costmodel_*); this module only orders the steps:

  collect   exhaustive autotuning (tgemm_autotune) of every shape, appended to
            one tuning database (resumable: measured keys are skipped);
  split     a seeded split of the shapes into training and held-out sets;
  subset    the records of a set of shapes, as a database of their own;
  train     tgemm_costmodel_train on the training records;
  evaluate  for every held-out shape, the measured time of the schedule each
            selector picks, against the best measured schedule:
              model    the cost model's argmin,
              default  the built-in rule (the method without the model),
              nearest  the best schedule of the nearest training shape
                       (distance in log2 M, N, K);
            reported as the geometric mean of t_best / t_chosen, its 10th
            percentile and the share of shapes at >= 0.9.

Shapes of the study: im2col gemms of 3x3 convolutions, batch 32
(M = 32 H W, N = Cout, K = 9 Cin) plus log-uniform random shapes.

Command line:
  python -m paper_1804_10694_amd.costmodel {run|collect|fit} --out DIR
      [--random 2000] [--dtype f32] [--reps 5] [--held-out 200] [--epochs 60]
      [--budget SECONDS]
  collect stops after --budget seconds and resumes on the next call; fit trains
  and evaluates on what DIR holds; run does both, fitting only once every shape
  is collected.
"""
import argparse
import json
import math
import os
import time

import numpy as np

from . import inputs


def _tg():
    from . import tgemm
    return tgemm


def read_db(path):
    recs = []
    with open(path) as f:
        for line in f:
            try:
                r = json.loads(line)
            except json.JSONDecodeError:
                continue
            if r.get("valid"):
                recs.append(r)
    return recs


def by_shape(recs, dtype_code):
    out = {}
    for r in recs:
        if r["dtype"] != dtype_code:
            continue
        out.setdefault((r["M"], r["N"], r["K"]), {})[(r["sched"], r["group_m"], r["xcd"])] = r["ms"]
    return out


def shapes_done(db_path):
    """Shapes with at least one record in the database (appended whole, see collect)."""
    done = set()
    if not os.path.exists(db_path):
        return done
    with open(db_path) as f:
        for line in f:
            try:
                r = json.loads(line)
            except json.JSONDecodeError:
                continue
            done.add((r["dtype"], r["M"], r["N"], r["K"]))
    return done


def collect(shapes, dtype, db_path, reps=5, progress=None, budget_s=None):
    """Exhaustive autotuning of every shape not yet in db_path.

    Each shape is tuned into a temporary file which is appended to db_path only
    when the shape is complete, so the database holds whole shapes and a killed
    or budget-stopped run resumes at the first missing one.  Returns the number
    of shapes still missing.
    """
    tg = _tg()
    code = tg.DTYPES[dtype]
    done = shapes_done(db_path)
    todo = [s for s in dict.fromkeys(tuple(int(x) for x in s) for s in shapes)
            if (code, *s) not in done]
    tmp = db_path + ".shape"
    t0 = time.time()
    for i, (m, n, k) in enumerate(todo):
        if budget_s is not None and time.time() - t0 > budget_s:
            print(f"collect {dtype}: budget reached, {len(todo) - i} shapes left", flush=True)
            return len(todo) - i
        if os.path.exists(tmp):
            os.remove(tmp)
        tg.autotune(m, n, k, dtype, reps, tmp)
        with open(tmp) as f, open(db_path, "a") as g:
            g.write(f.read())
        os.remove(tmp)
        if progress and (i + 1) % progress == 0:
            print(f"collect {dtype}: {i + 1}/{len(todo)} shapes, {time.time() - t0:.0f} s",
                  flush=True)
    return 0


def split(shapes, held_out, seed=5):
    shapes = [tuple(int(x) for x in s) for s in shapes]
    uniq = sorted(set(shapes))
    rng = np.random.default_rng(seed)
    idx = rng.permutation(len(uniq))
    held = [uniq[i] for i in idx[:held_out]]
    train = [uniq[i] for i in idx[held_out:]]
    return train, held


def subset(db_path, shapes, out_path):
    keep = set(tuple(s) for s in shapes)
    n = 0
    with open(db_path) as f, open(out_path, "w") as g:
        for line in f:
            try:
                r = json.loads(line)
            except json.JSONDecodeError:
                continue
            if (r["M"], r["N"], r["K"]) in keep:
                g.write(line if line.endswith("\n") else line + "\n")
                n += 1
    return n


def _summary(ratios):
    a = np.asarray(ratios, dtype=np.float64)
    return {"geomean": float(np.exp(np.mean(np.log(a)))), "p10": float(np.percentile(a, 10)),
            "share_ge_0.9": float(np.mean(a >= 0.9)), "count": int(len(a))}


def evaluate(db_path, held_shapes, train_shapes, dtype):
    """Ratios t_best / t_chosen on the held-out shapes for four selectors: the
    model, the built-in rule ("default"), the best candidate of the nearest
    training shape, and one candidate for every shape ("single": the one with
    the best geometric mean over the training shapes that it serves all of)."""
    tg = _tg()
    code = tg.DTYPES[dtype]
    table = by_shape(read_db(db_path), code)
    tg.set_policy("default")
    train_best = {}
    for s in train_shapes:
        if s in table:
            train_best[s] = min(table[s], key=table[s].get)
    single = None
    if train_best:
        common = set.intersection(*(set(table[s]) for s in train_best))
        score = {c: sum(math.log(min(table[s].values()) / table[s][c]) for s in train_best) for c in common}
        single = max(score, key=score.get) if score else None
    tlog = np.array([[math.log2(x) for x in s] for s in train_best]) if train_best else None
    tkeys = list(train_best)
    ratios = {"model": [], "default": [], "nearest": [], "single": []}
    picks = []
    t_select = []
    for s in held_shapes:
        if s not in table:
            continue
        meas = table[s]
        best = min(meas.values())
        t0 = time.perf_counter()
        pred = tg.costmodel_predict(*s, dtype)
        t_select.append(time.perf_counter() - t0)
        sid, gm, xcd = tg.select_schedule(*s, dtype)
        choices = {"default": (sid, gm, xcd)}
        if pred is not None:
            choices["model"] = pred[:3]
        if tlog is not None:
            q = np.array([math.log2(x) for x in s])
            near = tkeys[int(np.argmin(np.sum((tlog - q) ** 2, axis=1)))]
            choices["nearest"] = train_best[near]
        if single is not None:
            choices["single"] = single
        for name, c in choices.items():
            t = meas.get(tuple(c))
            if t is not None:
                ratios[name].append(best / t)
        picks.append({"shape": s, "best_ms": best, **{k: list(v) for k, v in choices.items()}})
    out = {name: _summary(r) for name, r in ratios.items() if r}
    out["select_us_median"] = float(np.median(t_select) * 1e6) if t_select else None
    return out, picks


def study_shapes(n_random, seed=5, lo=64, hi=8192):
    conv = [tuple(int(x) for x in s) for s in inputs.conv_shapes()]
    rand = [tuple(int(x) for x in s) for s in inputs.random_shapes(n_random, lo, hi, seed)]
    return conv + rand


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["run", "collect", "fit"])
    ap.add_argument("--out", required=True)
    ap.add_argument("--random", type=int, default=2000)
    ap.add_argument("--hi", type=int, default=8192)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--held-out", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--budget", type=float, default=None, help="collection time limit, seconds")
    args = ap.parse_args()
    tg = _tg()
    os.makedirs(args.out, exist_ok=True)
    db = os.path.join(args.out, f"tune_{args.dtype}.jsonl")
    shapes = study_shapes(args.random, hi=args.hi)
    if args.cmd in ("run", "collect"):
        left = collect(shapes, args.dtype, db, args.reps, progress=50, budget_s=args.budget)
        print(json.dumps({"dtype": args.dtype, "shapes": len(set(shapes)), "left": left}), flush=True)
        if args.cmd == "collect" or left:
            return
    train, held = split(shapes, args.held_out)
    tdb = os.path.join(args.out, f"train_{args.dtype}.jsonl")
    n_train = subset(db, train, tdb)
    weights = os.path.join(args.out, f"costmodel_{args.dtype}.bin")
    t0 = time.time()
    loss = tg.costmodel_train(tdb, weights, epochs=args.epochs)
    t_train = time.time() - t0
    tg.costmodel_load(weights)
    summary, picks = evaluate(db, held, train, args.dtype)
    summary.update({"dtype": args.dtype, "train_records": n_train, "train_shapes": len(train),
                    "held_out_shapes": len(held), "final_loss": loss, "train_seconds": t_train,
                    "epochs": args.epochs})
    with open(os.path.join(args.out, f"eval_{args.dtype}.json"), "w") as f:
        json.dump({"summary": summary, "picks": picks}, f)
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
