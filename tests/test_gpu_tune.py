"""Autotuner on the GPU (Tiramisu paper, Section VI-A: tile sizes by measurement).

Every compiled schedule x tile-order variant passes the exact-integer gate,
the database is resumable, and the "tuned" policy then runs the winner with
results within tolerance of the oracle.
"""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_1804_10694_amd import inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    yield tgemm
    tgemm.set_policy("default")


def _records(path):
    return [json.loads(l) for l in open(path) if l.strip()]


@pytest.mark.parametrize("dtype,shape", [("f32", (300, 200, 100)), ("x3", (260, 390, 130)),
                                         ("bf16", (256, 320, 272)), ("fp8", (200, 256, 384))])
def test_autotune_gate_and_resume(tg, tmp_path, dtype, shape):
    db = str(tmp_path / "tune.jsonl")
    best = tg.autotune(*shape, dtype, 3, db)
    recs = _records(db)
    serving = tg.schedules(dtype)
    M, N, K = shape
    es = {"f32": 4, "x3": 4, "bf16": 2, "fp8": 1}[dtype]
    aligned = (K * es) % 16 == 0 and (N * es) % 16 == 0
    expect = sum(1 for _, info in serving if info["vec"] <= 1 or aligned) * 8   # 0: packed; 8 tile orders
    assert len(recs) == expect
    assert all(r["valid"] for r in recs), [r for r in recs if not r["valid"]]
    fastest = min(r["ms"] for r in recs)
    assert any(r["sched"] == best and r["ms"] == fastest for r in recs)
    # a second run measures nothing new
    assert tg.autotune(*shape, dtype, 3, db) == best
    assert len(_records(db)) == expect


def test_tuned_policy_runs_the_winner(tg, tmp_path):
    db = str(tmp_path / "tune.jsonl")
    M, N, K = 700, 500, 300
    best = tg.autotune(M, N, K, "x3", 3, db)
    tg.set_policy("tuned")
    assert tg.select_schedule(M, N, K, "x3")[0] == best
    A, B, C0 = inputs.gemm_inputs(M, N, K, seed=41)
    C = C0.to(DEV)
    tg.gemm(A.to(DEV), B.to(DEV), C, 1.0, 1.0, "x3")
    torch.cuda.synchronize()
    tg.set_policy("default")
    assert oracle.normwise_error(C.cpu().numpy(), oracle.gemm(A, B, C0, 1.0, 1.0)) <= 1e-5


def test_interrupted_run_resumes(tg, tmp_path):
    # keep only the first third of a finished run, plus a torn last line
    db = tmp_path / "tune.jsonl"
    M, N, K = 256, 256, 128
    tg.autotune(M, N, K, "f32", 2, str(db))
    lines = db.read_text().splitlines()
    keep = lines[: len(lines) // 3]
    db.write_text("\n".join(keep) + "\n" + lines[-1][:30])
    tg.autotune(M, N, K, "f32", 2, str(db))
    recs = []
    for l in db.read_text().splitlines():
        try:
            recs.append(json.loads(l))
        except json.JSONDecodeError:
            pass
    keys = {(r["sched"], r["group_m"], r["xcd"]) for r in recs}
    assert len(keys) == len(lines)     # every key measured exactly once overall
    assert len(recs) == len(lines)
