"""Tuning database reader and the "tuned" policy (host only, no GPU).

Fault injection on the file the autotuner appends to: corrupt, truncated,
invalid and foreign-table records are skipped; the fastest valid record wins.
"""
import json

import pytest


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    yield tgemm
    tgemm.set_policy("default")


def _rec(tg, sid, ms, M=1000, N=900, K=700, dtype=0, gm=4, xcd=1, valid=True, space=None):
    info = tg.schedule_info(sid)
    return json.dumps({"arch": "gfx950", "space": space or format(tg.schedule_space_hash(), "x"),
                       "dtype": dtype, "M": M, "N": N, "K": K, "sched": sid, "BM": info["BM"],
                       "BN": info["BN"], "BK": info["BK"], "WGM": info["WGM"], "WGN": info["WGN"],
                       "vec": info["vec"], "group_m": gm, "xcd": xcd, "reps": 5, "ms": ms,
                       "tflops": 1.0, "valid": valid})


def test_fastest_valid_record_wins_and_faults_are_skipped(tg, tmp_path):
    f32 = [i for i, info in tg.schedules("f32") if info["vec"] == 4]
    a, b, c = f32[0], f32[1], f32[2]
    lines = [
        _rec(tg, a, 2.0),
        _rec(tg, b, 0.5, valid=False),                 # faster but failed the gate
        _rec(tg, c, 1.0, gm=16, xcd=0),                # the winner
        _rec(tg, a, 0.1, space="deadbeef"),            # another schedule table
        "{\"dtype\": 0, \"M\": 1000, garbage",           # corrupt line
        _rec(tg, b, 0.2, dtype=1),                     # schedule does not serve x3
        _rec(tg, c, 0.9)[:40],                         # truncated last line (no newline)
    ]
    db = tmp_path / "db.jsonl"
    db.write_text("\n".join(lines))
    used = tg.load_tuning_db(str(db))
    assert used == 2
    tg.set_policy("tuned")
    assert tg.select_schedule(1000, 900, 700, "f32") == (c, 16, 0)
    # shapes without a record fall back to the built-in rule
    tg.set_policy("default")
    dflt = tg.select_schedule(1234, 900, 700, "f32")
    tg.set_policy("tuned")
    assert tg.select_schedule(1234, 900, 700, "f32") == dflt
    tg.set_policy("default")


def test_missing_db_is_an_error(tg, tmp_path):
    with pytest.raises(tg.TgemmError):
        tg.load_tuning_db(str(tmp_path / "absent.jsonl"))


def test_force_policy(tg):
    x3 = [i for i, info in tg.schedules("x3") if info["vec"] == 4][1]
    tg.set_policy(f"force:{x3}")
    assert tg.select_schedule(4096, 4096, 4096, "x3")[0] == x3
    # a forced id that does not serve the dtype falls back to the rule
    sid = tg.select_schedule(4096, 4096, 4096, "f32")[0]
    assert tg.schedule_info(sid)["dtype"] == 0
    tg.set_policy("default")


def test_autotune_rejects_bad_arguments(tg, tmp_path):
    p = str(tmp_path / "t.jsonl").encode()
    assert tg.lib.tgemm_autotune(0, 4, 4, 0, 3, p) == -1
    assert tg.lib.tgemm_autotune(4, 4, 4, 7, 3, p) == -2
    assert tg.lib.tgemm_autotune(4, 4, 4, 0, 0, p) == -1
    assert tg.lib.tgemm_autotune(4, 4, 4, 0, 3, None) == -1


def test_default_rule_packs_large_problems_only(tg):
    # Large problems take the packed-operand kernels (the packing pass is O(MK + KN)
    # against O(MNK)); small ones the direct kernels, which need no workspace.
    tg.set_policy("default")
    for dt in ("f32", "x3", "bf16", "fp8"):
        big = tg.schedule_info(tg.select_schedule(8192, 8192, 8192, dt)[0])
        assert big["vec"] == 0, (dt, big)
        small = tg.schedule_info(tg.select_schedule(256, 256, 256, dt)[0])
        assert small["vec"] in (1, 4), (dt, small)
    assert tg.schedule_info(tg.select_schedule(8192, 8192, 8192, "f32")[0])["BM"] == 128
