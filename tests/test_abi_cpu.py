"""Host-side checks of the C ABI (no GPU needed).

The library loads and exports every function include/tgemm.h declares;
argument validation answers before any HIP call; the host tile planner is the
bijection the tiling map of the Tiramisu paper describes (the map a tiling
command of Section III-C becomes, given in the introduction of Section V), and
classifies full and partial tiles as Section V-A (code generation) defines them.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tgemm.h")


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    return tgemm


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tgemm\w*)\s*\(", text)))


def test_every_declared_symbol_is_exported(tg):
    names = declared_functions()
    assert "tgemm" in names and "tgemm_batched" in names and "tgemm_scaled" in names
    for n in names:
        assert hasattr(tg.lib, n), n
        getattr(tg.lib, n)  # resolves the symbol


def test_status_strings(tg):
    assert tg.status_string(0) == "TGEMM_SUCCESS"
    assert tg.status_string(5) == "TGEMM_CAPTURE_UNPLANNED"
    assert tg.status_string(99) == "TGEMM_UNKNOWN_STATUS"


FAKE = 0x10000  # a non-null pointer that is never dereferenced


@pytest.mark.parametrize("args,code", [
    ((-1, 4, 4, 1.0, FAKE, 4, FAKE, 4, 0.0, FAKE, 4, 0), 1),   # M < 0
    ((4, -1, 4, 1.0, FAKE, 4, FAKE, 4, 0.0, FAKE, 4, 0), 1),   # N < 0
    ((4, 4, -2, 1.0, FAKE, 4, FAKE, 4, 0.0, FAKE, 4, 0), 1),   # K < 0
    ((4, 4, 8, 1.0, FAKE, 7, FAKE, 4, 0.0, FAKE, 4, 0), 1),    # lda < K
    ((4, 5, 8, 1.0, FAKE, 8, FAKE, 4, 0.0, FAKE, 5, 0), 1),    # ldb < N
    ((4, 5, 8, 1.0, FAKE, 8, FAKE, 5, 0.0, FAKE, 4, 0), 1),    # ldc < N
    ((4, 4, 4, 1.0, None, 4, FAKE, 4, 0.0, FAKE, 4, 0), 1),    # A null while read
    ((4, 4, 4, 1.0, FAKE, 4, None, 4, 0.0, FAKE, 4, 0), 1),    # B null while read
    ((4, 4, 4, 1.0, FAKE, 4, FAKE, 4, 0.0, None, 4, 0), 1),    # C null
    ((4, 4, 4, 1.0, FAKE, 4, FAKE, 4, 0.0, FAKE, 4, 9), 2),    # unknown dtype
    ((4, 4, 4, float("nan"), FAKE, 4, FAKE, 4, 0.0, FAKE, 4, 0), 1),
    ((0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 0), 0),    # empty: no-op, no HIP call
    ((4, 0, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 1), 0),
])
def test_validation_before_any_hip_call(tg, args, code):
    assert tg.lib.tgemm(*args, None) == code


def test_with_schedule_validation(tg):
    fid = [i for i, info in tg.schedules("f32") if info["vec"] == 4][0]
    xid = [i for i, info in tg.schedules("x3")][0]
    base = (64, 64, 64, 1.0, FAKE, 64, FAKE, 64, 0.0, FAKE, 64)
    assert tg.lib.tgemm_with_schedule(*base, 0, 10 ** 6, 8, 1, None) == 2   # no such schedule
    assert tg.lib.tgemm_with_schedule(*base, 0, xid, 8, 1, None) == 2       # wrong dtype
    assert tg.lib.tgemm_with_schedule(*base, 0, fid, 0, 1, None) == 1       # group_m < 1
    # misaligned base pointer cannot use a 16-byte-load schedule
    mis = (64, 64, 64, 1.0, FAKE + 4, 64, FAKE, 64, 0.0, FAKE, 64)
    assert tg.lib.tgemm_with_schedule(*mis, 0, fid, 8, 1, None) == 2


def test_policy_strings(tg):
    assert tg.lib.tgemm_set_policy(b"bogus") == 1
    assert tg.lib.tgemm_set_policy(b"force:-3") == 1
    assert tg.lib.tgemm_set_policy(b"force:abc") == 1
    assert tg.lib.tgemm_set_policy(b"default") == 0
    assert tg.lib.tgemm_set_policy(b"tuned") == 0
    tg.set_policy("default")


def test_schedule_table_is_consistent(tg):
    n = tg.schedule_count()
    assert n >= 8
    for i in range(n):
        s = tg.schedule_info(i)
        assert s["dtype"] in (0, 1, 2, 3)
        assert s["BM"] % (32 * s["WGM"]) == 0 and s["BN"] % (32 * s["WGN"]) == 0
        assert s["lds_bytes"] <= 160 * 1024            # gfx950 LDS per workgroup
        assert s["vec"] in (0, 1, 4)     # 0: packed operands
    for dt in ("f32", "x3"):
        assert len(tg.schedules(dt)) >= 4


@pytest.mark.parametrize("M,N,BM,BN", [(1000, 777, 128, 128), (8192, 8192, 256, 128),
                                       (4097, 3001, 128, 128), (33, 1, 64, 64), (17, 4000, 64, 128)])
@pytest.mark.parametrize("group_m,xcd", [(1, 0), (8, 1), (5, 1), (16, 0)])
def test_tile_map_is_a_bijection(tg, M, N, BM, BN, group_m, xcd):
    tm, tn, full = tg.tile_map(M, N, BM, BN, group_m, xcd)
    Tm, Tn = -(-M // BM), -(-N // BN)
    seen = set(zip(tm, tn))
    assert len(seen) == len(tm) == Tm * Tn
    assert all(0 <= a < Tm for a in tm) and all(0 <= b < Tn for b in tn)
    # every (i, j) is covered by exactly one tile: i0 = floor(i / BM) etc.
    cover = np.zeros((Tm * BM, Tn * BN), dtype=np.int8) if Tm * Tn <= 4096 else None
    if cover is not None:
        for a, b in zip(tm, tn):
            cover[a * BM:(a + 1) * BM, b * BN:(b + 1) * BN] += 1
        assert (cover[:M, :N] == 1).all()
    # a tile is full iff it lies inside M x N (size a multiple of the tile size)
    for a, b, f in zip(tm, tn, full):
        assert f == int((a + 1) * BM <= M and (b + 1) * BN <= N)


def test_tile_map_xcd_runs_are_contiguous(tg):
    # With the remap on, the workgroups of one XCD (wg % 8) get consecutive tile ranks
    # of the grouped order, i.e. neighbouring tiles.
    M = N = 2048
    tm, tn, _ = tg.tile_map(M, N, 128, 128, 1, 1)
    tiles_n = 16
    rank = {(a, b): a * tiles_n + b for a, b in zip(tm, tn)}   # group_m = 1: row-major rank
    by_xcd = {}
    for w, (a, b) in enumerate(zip(tm, tn)):
        by_xcd.setdefault(w % 8, []).append(rank[(a, b)])
    for ranks in by_xcd.values():
        assert ranks == list(range(ranks[0], ranks[0] + len(ranks)))


def test_select_schedule_serves_dtype(tg):
    for dt in ("f32", "x3"):
        for shape in [(256, 256, 256), (8192, 8192, 8192), (4097, 3001, 2053), (16, 16, 16)]:
            sid, gm, xcd = tg.select_schedule(*shape, dt)
            assert tg.schedule_info(sid)["dtype"] == tg.DTYPES[dt]
            assert gm >= 1


def test_schedule_keys_are_unique(tg):
    keys = [tg.schedule_key(i) for i in range(tg.schedule_count())]
    assert len(keys) == len(set(keys))


def test_conv_packed_shapes_and_path_validation(tg):
    # tile shapes of the packed 3x3 convolution kernel: host table, no HIP call
    for dt in ("f32", "x3"):
        shapes = tg.conv3x3_packed_shapes(dt)
        assert len(shapes) >= 2 and len(set(shapes)) == len(shapes)
        for bm, bn, bk, st in shapes:
            assert bm in (128, 256) and bn in (128, 256) and 128 % bk == 0 and st >= 2
    assert tg.conv3x3_packed_shapes("bf16") == []
    # an unknown kernel choice is refused before any HIP call
    args = (1, 4, 4, 8, 8, 1.0, FAKE, FAKE, 0.0, FAKE, 0)
    assert tg.lib.tgemm_conv3x3_path(*args, 99 - 100, None) == 1
    assert tg.lib.tgemm_conv3x3_path(*args, 2 + len(tg.conv3x3_packed_shapes("f32")), None) == 1
    # empty layers are no-ops on every path
    assert tg.lib.tgemm_conv3x3_path(0, 4, 4, 8, 8, 1.0, None, None, 0.0, None, 0, 2, None) == 0
