"""The built-in schedule rule (host only, no GPU): which form each kind of problem takes.

The rule was set from exhaustive measurements on MI355X (the cost-model study); these
checks pin its documented boundaries, so that a change to them is deliberate.
"""
import pytest


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    tgemm.set_policy("default")
    yield tgemm


def _kind(tg, M, N, K, dt):
    i = tg.schedule_info(tg.select_schedule(M, N, K, dt)[0])
    if i["inplace"]:
        return f"inplace{i['BM']}"
    if i["split"]:
        return "streamk"
    return "packed" if i["vec"] == 0 else f"direct{i['BM']}"


@pytest.mark.parametrize("shape,kind", [
    ((4097, 3001, 2053), "inplace64"),     # 128 x 128 tiles would fill half of their second wave
    ((4096, 4096, 4096), "inplace128"),
    ((700, 700, 700), "inplace64"),
    ((1000, 1000, 8192), "streamk"),       # deep K on few tiles: stream-K spreads K over every CU
    ((256, 256, 8192), "streamk"),
    ((200, 4000, 8192), "inplace64"),      # M < 256: in place even with deep K
    ((100, 4096, 4096), "inplace64"),      # narrow
    ((401408, 64, 1152), "inplace64"),     # im2col of a 3x3 convolution, 64 output channels
    ((8192, 512, 8192), "inplace64"),      # M or N <= 512: in place at any size
    ((8192, 8192, 8192), "packed"),        # 2048 tiles of 128 x 256 and M, N > 512
    ((8448, 8192, 640), "streamk"),        # packed range, whole tiles would fill 82% of their waves
])
def test_f32_rule(tg, shape, kind):
    assert _kind(tg, *shape, "f32") == kind


@pytest.mark.parametrize("shape,kind", [
    ((4097, 3001, 2053), "packed"),        # 3055 tiles of 64 x 64, K >= 1024: packing pays
    ((8192, 8192, 8192), "packed"),
    ((2048, 2048, 1024), "packed"),
    ((300, 5000, 2000), "inplace64"),      # M <= 512
    ((1000, 1000, 8192), "streamk"),       # deep K on few tiles
    ((700, 700, 700), "inplace64"),        # 121 tiles
    ((6000, 2000, 700), "inplace128"),     # K < 1024, 2945 tiles
    ((100352, 256, 2304), "inplace128"),   # im2col, N <= 512
    ((100352, 64, 1152), "direct64"),      # N <= 64: direct 64 x 64 tiles
    ((1024, 1024, 1024), "direct64"),      # whole 64 x 64 tiles, 16-byte loads, M, N in [512, 4096]
])
def test_x3_rule(tg, shape, kind):
    assert _kind(tg, *shape, "x3") == kind
