"""Cost-model host logic (no GPU): features, weight-file faults, policy strings."""
import math
import struct

import pytest


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    yield tgemm
    tgemm.set_policy("default")


def test_features_are_finite_and_follow_the_problem(tg):
    sid = [i for i, info in tg.schedules("f32") if info["BM"] == 128 and info["vec"] == 4][0]
    f = tg.costmodel_features(4096, 2048, 1024, "f32", sid, 8, 1)
    assert len(f) == 22 and all(math.isfinite(x) for x in f)
    assert f[0:3] == [12.0, 11.0, 10.0]                       # log2 M, N, K
    assert f[3:6] == [0.0, 0.0, 0.0]                          # dtype one-hot (f32)
    assert f[6:9] == [7.0, 7.0, math.log2(tg.schedule_info(sid)["BK"])]
    assert f[10] == 3.0 and f[11] == 1.0                      # log2 group_m, xcd
    assert f[12] == math.log2(32 * 16)                        # tiles
    assert f[14] == 0.0                                       # no partial tiles
    ragged = tg.costmodel_features(4097, 2048, 1024, "f32", sid, 8, 1)
    assert ragged[14] > 0.0                                   # the last tile row is padding
    x3 = [i for i, info in tg.schedules("x3")][0]
    assert tg.costmodel_features(64, 64, 64, "x3", x3, 1, 0)[3] == 1.0
    assert f[20] == 0.0                                       # one workgroup per tile
    sk = [i for i, info in tg.schedules("f32") if info["split"] == 1][0]
    assert tg.costmodel_features(4097, 2048, 1024, "f32", sk, 8, 1)[20] == 1.0   # stream-K
    assert f[21] == 0.0                                       # 32 x 32 MFMA blocks
    m16 = [i for i, info in tg.schedules("f32") if info["mfma"] == 16][0]
    assert tg.costmodel_features(4097, 2048, 1024, "f32", m16, 8, 1)[21] == 1.0


def test_weight_file_faults_are_refused(tg, tmp_path):
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a weight file at all")
    assert tg.lib.tgemm_costmodel_load(str(bad).encode()) == tg.INVALID_VALUE
    trunc = tmp_path / "trunc.bin"
    trunc.write_bytes(struct.pack("<II", 0x4D434754, 1) + b"\x00" * 10)   # right magic, cut short
    assert tg.lib.tgemm_costmodel_load(str(trunc).encode()) == tg.INVALID_VALUE
    assert tg.lib.tgemm_costmodel_load(str(tmp_path / "absent.bin").encode()) == tg.INVALID_VALUE


def test_model_policy_without_model_falls_back(tg):
    tg.costmodel_unload()
    tg.set_policy("default")
    dflt = tg.select_schedule(3000, 2000, 1000, "f32")
    tg.set_policy("model")
    assert tg.select_schedule(3000, 2000, 1000, "f32") == dflt
    assert tg.costmodel_predict(3000, 2000, 1000, "f32") is None
    tg.set_policy("default")


def test_train_rejects_bad_arguments(tg, tmp_path):
    db = str(tmp_path / "none.jsonl").encode()
    w = str(tmp_path / "w.bin").encode()
    assert tg.lib.tgemm_costmodel_train(db, w, 0, 64, 1e-3, 1, None) == tg.INVALID_VALUE
    assert tg.lib.tgemm_costmodel_train(db, w, 5, 64, -1.0, 1, None) == tg.INVALID_VALUE
    assert tg.lib.tgemm_costmodel_train(db, w, 5, 64, 1e-3, 1, None) == tg.INVALID_VALUE  # no file


def test_collection_appends_whole_shapes_and_resumes(tmp_path, monkeypatch):
    """collect() writes a shape to the database only once it is tuned whole, stops at its
    time budget and resumes at the first missing shape (autotuning replaced by a stub)."""
    import json
    from paper_1804_10694_amd import costmodel as CM

    calls = []

    class Stub:
        DTYPES = {"f32": 0}

        @staticmethod
        def autotune(m, n, k, dtype, reps, db):
            calls.append((m, n, k))
            with open(db, "a") as f:
                for sid in range(3):
                    f.write(json.dumps({"dtype": 0, "M": m, "N": n, "K": k, "sched": sid,
                                        "group_m": 1, "xcd": 0, "ms": 1.0 + sid,
                                        "valid": True}) + "\n")

    monkeypatch.setattr(CM, "_tg", lambda: Stub)
    db = str(tmp_path / "db.jsonl")
    shapes = [(64, 64, 64), (128, 64, 64), (64, 64, 64), (256, 128, 64)]
    assert CM.collect(shapes, "f32", db, budget_s=-1.0) == 3      # budget spent before the first
    assert calls == []
    assert CM.collect(shapes[:2], "f32", db) == 0
    assert CM.collect(shapes, "f32", db) == 0                     # only the missing shape is tuned
    assert calls == [(64, 64, 64), (128, 64, 64), (256, 128, 64)]
    recs = CM.read_db(db)
    assert len(recs) == 9 and CM.shapes_done(db) == {(0, 64, 64, 64), (0, 128, 64, 64),
                                                     (0, 256, 128, 64)}
    assert not (tmp_path / "db.jsonl.shape").exists()
