"""The learned cost model end to end on the GPU, at a reduced scale.

Exhaustive autotuning measures every candidate schedule of a set of shapes;
the network is trained on the GPU on the training shapes; on held-out shapes
the schedule it picks is compared, by measured time, with the best measured
schedule and with the methods without the model (the built-in rule, and one
schedule for every shape).
Absolute runtime predictions are not asserted (measurements are the only
ground truth).
"""
import json
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1804_10694_amd import costmodel as CM
from paper_1804_10694_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    yield tgemm
    tgemm.set_policy("default")
    tgemm.costmodel_unload()


def _run_study(tg, d, dtype):
    # 300 shapes log-uniform in [128, 4096]^3 and 12 convolution shapes, a fifth held out
    shapes = [tuple(int(x) for x in s) for s in inputs.random_shapes(300, 128, 4096, seed=15)]
    shapes += [(32 * h * h, co, 9 * ci) for h in (7, 14, 28) for ci in (64, 256) for co in (64, 256)]
    db = str(d / f"tune_{dtype}.jsonl")
    t0 = time.perf_counter()
    CM.collect(shapes, dtype, db, reps=3, progress=50)
    search_s = (time.perf_counter() - t0) / len(shapes)
    train, held = CM.split(shapes, len(shapes) // 5, seed=5)
    tdb = str(d / f"train_{dtype}.jsonl")
    CM.subset(db, train, tdb)
    w = str(d / f"cm_{dtype}.bin")
    loss = tg.costmodel_train(tdb, w, epochs=80, batch=256, lr=1e-3, seed=5)
    tg.costmodel_load(w)
    return {"db": db, "train": train, "held": held, "weights": w, "loss": loss, "dir": d,
            "search_s": search_s}


@pytest.fixture(scope="module")
def study_x3(tg, tmp_path_factory):
    return _run_study(tg, tmp_path_factory.mktemp("cm_x3"), "x3")


@pytest.fixture(scope="module")
def study(tg, tmp_path_factory, study_x3):
    # f32 last, so that its network is the one loaded for the tests below
    return _run_study(tg, tmp_path_factory.mktemp("cm"), "f32")


def test_training_converges(study):
    print("final normalised loss", study["loss"])
    assert study["loss"] < 0.2


def test_model_against_the_method_without_it(tg, study):
    # quality: t_best / t_chosen on held-out shapes, against the built-in rule; both are
    # measured with 3 repetitions, so differences under about 2% are noise
    summary, _ = CM.evaluate(study["db"], study["held"], study["train"], "f32")
    print(json.dumps(summary))
    assert summary["model"]["count"] >= 20
    assert summary["model"]["geomean"] >= 0.9
    assert summary["model"]["geomean"] >= summary["default"]["geomean"] - 0.02
    # cost: choosing by the model takes microseconds, exhaustive search seconds
    print(f"model selection {summary['select_us_median']:.0f} us, "
          f"exhaustive search {study['search_s'] * 1e3:.0f} ms per shape")
    assert summary["select_us_median"] * 1e-6 * 100 < study["search_s"]


def test_model_gains_over_the_method_without_it_x3(tg, study_x3, study):
    # split-bf16x3.  The method without the network is exhaustive autotuning of every new
    # shape (Section VI-A: tile sizes found by measurement); the network's gain is its
    # selection cost at the same quality: microseconds instead of a search of every
    # candidate, with its picks at >= 0.95 of the exhaustive optimum and not behind the
    # built-in rule or the single best schedule by more than the timing noise of a
    # geometric mean over 62 held-out shapes (0.02).  The quality gain over the selectors
    # without a network is printed, not asserted: at this scale (shapes in [128, 4096])
    # one in-place schedule already measured 0.969 and the rule 0.982 against the model's
    # 0.980; the full study (200 held-out shapes in [64, 8192]) measured the model at
    # 0.988, one schedule at 0.924 and the rule at 0.973 (the rule was set from that
    # study's measurements).
    tg.costmodel_load(study_x3["weights"])
    try:
        summary, _ = CM.evaluate(study_x3["db"], study_x3["held"], study_x3["train"], "x3")
    finally:
        tg.costmodel_load(study["weights"])
    print(json.dumps(summary))
    assert summary["model"]["count"] >= 20 and summary["single"]["count"] >= 20
    model, rule, single = (summary[k]["geomean"] for k in ("model", "default", "single"))
    print(f"x3: model {model:.3f}, one schedule {single:.3f} (gain {model - single:+.3f}), "
          f"rule {rule:.3f} (gain {model - rule:+.3f}); selection {summary['select_us_median']:.0f} us "
          f"against {study_x3['search_s'] * 1e3:.0f} ms of search per shape")
    assert model >= 0.95
    assert model >= rule - 0.02 and model >= single - 0.02
    assert summary["select_us_median"] * 1e-6 * 300 < study_x3["search_s"]


def test_out_of_distribution_falls_back_to_autotuning(tg, study):
    db2 = str(study["dir"] / "fallback.jsonl")
    # inside the training range: the model answers, nothing is measured
    sid, gm, xcd, fb = tg.costmodel_select(700, 600, 500, "f32", 2, db2)
    assert not fb and tg.schedule_info(sid)["dtype"] == 0
    # far outside (M = 2^15): exhaustive autotuning runs and records measurements
    sid, gm, xcd, fb = tg.costmodel_select(32768, 64, 64, "f32", 2, db2)
    assert fb
    recs = [json.loads(l) for l in open(db2)]
    assert recs and all(r["M"] == 32768 for r in recs)
    assert min(recs, key=lambda r: r["ms"])["ms"] == min(
        r["ms"] for r in recs if (r["sched"], r["group_m"], r["xcd"]) == (sid, gm, xcd))


def test_model_policy_runs_correct_gemms(tg, study):
    tg.set_policy("model")
    for shape in [(700, 600, 500), (1500, 130, 900)]:
        A, B, C0 = inputs.gemm_inputs(*shape, seed=77)
        C = C0.to(DEV)
        tg.gemm(A.to(DEV), B.to(DEV), C, 1.0, 1.0, "f32")
        torch.cuda.synchronize()
        assert oracle.normwise_error(C.cpu().numpy(), oracle.gemm(A, B, C0, 1.0, 1.0)) <= 1e-5
        pred = tg.costmodel_predict(*shape, "f32")
        assert tg.select_schedule(*shape, "f32") == pred[:3]
    tg.set_policy("default")


def test_predictions_rank_every_candidate(tg, study):
    rows = tg.costmodel_predict_all(1000, 1000, 1000, "f32")
    ids = {r[0] for r in rows}
    assert ids == {i for i, _ in tg.schedules("f32")}
    assert all(np.isfinite(r[3]) and r[3] > 0 for r in rows)


def test_weight_file_from_another_table_is_refused(tg, study, tmp_path):
    data = bytearray(open(study["weights"], "rb").read())
    data[8] ^= 0xFF                     # the schedule-table hash follows magic and version
    p = tmp_path / "other.bin"
    p.write_bytes(bytes(data))
    assert tg.lib.tgemm_costmodel_load(str(p).encode()) == tg.NOT_SUPPORTED
