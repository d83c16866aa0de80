"""Summaries of rocprofv3 output for the benchmark's gemm calls.

A gemm call is one kernel (direct schedules) or three (packed schedules: A
packing, B packing, then the main kernel), launched back to back on one
stream.  Dispatches are grouped into calls by that pattern, and a call is
matched to a benchmark path by its main kernel's grid size, which the
benchmark prints per path ("grid_threads").

  stats    per path: kernels of a call and their average durations, from a
           --kernel-trace run;
  traffic  per path: HBM bytes read and written per call, from one
           --pmc FETCH_SIZE run and one --pmc WRITE_SIZE run of the same
           command, scaled by what the counters read for the benchmark's
           closing 1 GiB device copy (--copy-calibration): the copy reads
           and writes 2^30 bytes each.

Command line:
  python -m paper_1804_10694_amd.profsum stats --trace T.csv --bench B.json --out X.md
      --command "..."
  python -m paper_1804_10694_amd.profsum traffic --fetch F.csv --write W.csv --bench B.json
      --out X.md --table T.json --command-fetch "..." --command-write "..."
"""
import argparse
import csv
import json
from collections import OrderedDict, defaultdict

MAIN_KERNELS = ("gemm_kernel", "packed_kernel", "packed_sk_kernel", "scaled_kernel", "inplace_gemm_kernel")
PACK_KERNELS = ("pack_rows_kernel", "pack_cols_kernel")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def short_name(name):
    """'void tg::packed_kernel<tg::PCfg<0, 128, ...> >(tg::PackedArgs)' -> 'packed_kernel<PCfg<0,128,...>>'."""
    n = name.replace("void ", "").replace("tg::", "")
    n = n.split("(")[0].replace(" ", "")
    return n


def kind(name):
    for k in MAIN_KERNELS + PACK_KERNELS:
        if k in name:
            return k
    return None


def read_dispatches(path):
    """Dispatches in order: dicts with id, name, grid (total threads), start, end, counters."""
    rows = OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            did = int(r["Dispatch_Id"])
            d = rows.get(did)
            if d is None:
                if "Grid_Size_X" in r:
                    grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
                else:
                    grid = int(float(r["Grid_Size"]))
                d = {"id": did, "name": r["Kernel_Name"], "grid": grid,
                     "start": int(r["Start_Timestamp"]), "end": int(r["End_Timestamp"]),
                     "counters": defaultdict(float)}
                rows[did] = d
            if "Counter_Name" in r:
                d["counters"][r["Counter_Name"]] += float(r["Counter_Value"])
    return sorted(rows.values(), key=lambda d: d["id"])


def group_calls(dispatches):
    """[(main dispatch, [pack dispatches before it])] in dispatch order."""
    calls, pending = [], []
    for d in dispatches:
        k = kind(d["name"])
        if k in PACK_KERNELS:
            pending.append(d)
        elif k in MAIN_KERNELS:
            calls.append((d, pending))
            pending = []
        else:
            pending = []
    return calls


def read_bench(path):
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{"):
                return json.loads(line)
    raise ValueError(f"no JSON line in {path}")


def paths_by_grid(bench):
    """Paths by the main kernel's grid (threads); stream-K paths, which launch one
    resident wave, under the key "sk"."""
    out = {}
    for label, p in bench["paths"].items():
        shape = label.split("_", 1)[1]
        g = "sk" if p.get("stream_k") else p["grid_threads"]
        out.setdefault(g, []).append((label, p["schedule_key"] + "@" + shape, p))
    return out


def match(calls, bench):
    """{label: (key, [calls])} for the calls whose main kernel grid (or, for a
    stream-K form, kernel name and tile) names one path."""
    grids = paths_by_grid(bench)
    got = defaultdict(list)
    for main, packs in calls:
        if "packed_sk_kernel" in main["name"]:
            tile = lambda p: ",%d,%d," % tuple(int(x) for x in p["schedule_key"].split(":")[2].split("x")[:2])
            cands = [c for c in grids.get("sk", []) if tile(c[2]) in short_name(main["name"])]
        else:
            cands = grids.get(main["grid"], [])
        # paths sharing a grid are told apart by the main kernel's mode (template argument 0/1)
        for label, key, p in cands:
            mode = "1" if label.startswith("x3") else "0"
            if f"<{mode}," in short_name(main["name"]):
                got[label].append((main, packs))
                break
    return {label: ([k for lb, k, _ in sum(grids.values(), []) if lb == label][0], cs)
            for label, cs in got.items()}


def cmd_stats(args):
    bench = read_bench(args.bench)
    calls = group_calls(read_dispatches(args.trace))
    m = match(calls, bench)
    lines = [f"# Kernel durations per gemm call: {args.title}", "", "Command (on one MI355X, from the repository root):", "",
             "    " + args.command, "",
             "Dispatches are grouped into calls (packing kernels, then the main kernel); the first call",
             "of each path is a cold warm-up and is left out of the averages.", "",
             "| Path | Kernel | Calls | Average (ms) | Min (ms) | Max (ms) |", "|---|---|---|---|---|---|"]
    for label in bench["paths"]:
        if label not in m:
            continue
        key, cs = m[label]
        cs = cs[1:] if len(cs) > 1 else cs
        per = defaultdict(list)
        tot = []
        for main, packs in cs:
            t = 0.0
            for d in packs + [main]:
                dur = (d["end"] - d["start"]) / 1e6
                per[short_name(d["name"])].append(dur)
                t += dur
            tot.append(t)
        for name, ts in per.items():
            lines.append(f"| {label} | `{name}` | {len(ts)} | {sum(ts) / len(ts):.4f} | {min(ts):.4f} | "
                         f"{max(ts):.4f} |")
        lines.append(f"| {label} | **whole call** | {len(tot)} | **{sum(tot) / len(tot):.4f}** | "
                     f"{min(tot):.4f} | {max(tot):.4f} |")
    lines += ["", "The benchmark line (no profiler) measured with HIP events around each call:", ""]
    for label, p in bench["paths"].items():
        lines.append(f"- {label}: average {p['avg_ms']} ms, {p['tflops']} TFLOP/s, {p['frac_peak']} of "
                     f"{p['peak_tflops']} ({p['schedule_key']})")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def calibration(dispatches, counter):
    """Counter value (KiB) of the closing 1 GiB device copy: the last dispatch of the run,
    which must be a copy kernel after the last gemm (the smaller copies before it move
    results to the host through staging buffers)."""
    last = max(i for i, d in enumerate(dispatches) if kind(d["name"]) in MAIN_KERNELS)
    if last == len(dispatches) - 1 or COPY_KERNEL not in dispatches[-1]["name"]:
        raise ValueError("the run does not end with the calibration copy")
    return dispatches[-1]["counters"][counter], 1


def cmd_traffic(args):
    bench = read_bench(args.bench)
    out = {}
    lines = [f"# HBM traffic per gemm call: {args.title}", "", "Commands (on one MI355X, from the repository root):", "",
             "    " + args.command_fetch, "    " + args.command_write, "",
             "FETCH_SIZE and WRITE_SIZE are summed over the kernels of one call (packing kernels and",
             "main kernel) and scaled by the factor that maps the closing 1 GiB device copy onto",
             "2^30 bytes read and 2^30 bytes written.", ""]
    per = {}
    cal = {}
    for counter, path in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        disp = read_dispatches(path)
        kib, ncopy = calibration(disp, counter)
        factor = 2 ** 30 / (kib * 1024.0)
        cal[counter] = {"copy_kib": kib, "copy_dispatches": ncopy, "factor": factor}
        for label, (key, cs) in match(group_calls(disp), bench).items():
            vals = [sum(d["counters"][counter] for d in packs + [main]) * 1024.0 * factor
                    for main, packs in cs[1:] or cs]
            per.setdefault(label, {"key": key})[counter] = sum(vals) / len(vals)
    lines += [f"Calibration: FETCH_SIZE x {cal['FETCH_SIZE']['factor']:.4f}, "
              f"WRITE_SIZE x {cal['WRITE_SIZE']['factor']:.4f}.", "",
              "| Path | Read (bytes) | Written (bytes) | Total | Compulsory | Total / compulsory |",
              "|---|---|---|---|---|---|"]
    sha = bench["roofline"]["kernel_source_sha256"]
    for label, rec in per.items():
        if "FETCH_SIZE" not in rec or "WRITE_SIZE" not in rec:
            continue
        m, n, k = (int(x) for x in label.split("_", 1)[1].split("x"))
        comp = 4 * (m * k + k * n + 2 * m * n)
        tot = rec["FETCH_SIZE"] + rec["WRITE_SIZE"]
        lines.append(f"| {label} | {rec['FETCH_SIZE']:.4g} | {rec['WRITE_SIZE']:.4g} | {tot:.4g} | {comp:.4g} | "
                     f"{tot / comp:.3f} |")
        out[rec["key"]] = {"hbm_bytes_per_launch": tot, "read_bytes": rec["FETCH_SIZE"],
                           "written_bytes": rec["WRITE_SIZE"], "compulsory_bytes": comp,
                           "source_sha256": sha, "calibration": cal}
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(args.table, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--bench", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="benchmark workload")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--bench", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--table", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--title", default="benchmark workload")
    args = ap.parse_args()
    (cmd_stats if args.cmd == "stats" else cmd_traffic)(args)


if __name__ == "__main__":
    main()
