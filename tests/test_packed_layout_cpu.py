"""Index algebra of the packed kernels' LDS layout, restated on the host (no GPU).

tile_packed.h places a panel row's 16-byte units in LDS at
    slot(row, u) = row * UK + (u ^ ((row / (16 / UK)) & (UK - 1)))
and fills a panel with wave instructions of 64 lanes, lane l of instruction ig
writing LDS unit ig * 64 + l from global byte offset
    voff = lane_off ^ ((4 * ig) & (UK - 1)) * 16,   soff = ig * (64 / UK) * row_bytes
    lane_off = (l / UK) * row_bytes + (((l % UK) ^ (l / 16)) & (UK - 1)) * 16.
These checks pin that the loads put every (row, unit) where the MFMA operand
reads look for it, and that those reads (16 consecutive rows at one unit) hit
16 distinct 16-byte bank groups, for every panel depth the schedules use."""
import pytest


def slot(row, u, uk):
    return row * uk + (u ^ ((row // (16 // uk)) & (uk - 1)))


@pytest.mark.parametrize("uk", [2, 4, 8, 16])
@pytest.mark.parametrize("rows", [64, 128, 256])
def test_loads_land_where_reads_look(uk, rows):
    row_bytes = 4096                       # any multiple of 16 * uk leaves the XOR to the unit bits
    where = {}
    for ig in range(rows * uk // 64):
        for lane in range(64):
            lane_off = (lane // uk) * row_bytes + (((lane % uk) ^ (lane // 16)) & (uk - 1)) * 16
            voff = lane_off ^ (((4 * ig) & (uk - 1)) * 16)
            byte = voff + ig * (64 // uk) * row_bytes
            row, u = byte // row_bytes, (byte % row_bytes) // 16
            assert (row, u) not in where, "two lanes load the same unit"
            where[(row, u)] = ig * 64 + lane
    assert len(where) == rows * uk
    for (row, u), lds_unit in where.items():
        assert lds_unit == slot(row, u, uk)


@pytest.mark.parametrize("uk", [2, 4, 8, 16])
def test_operand_reads_are_conflict_free(uk):
    # a wave's read of one unit for 32 consecutive rows: each aligned group of 16 rows
    # covers all 16 bank groups of 16 bytes (64 banks of 4 bytes)
    for u in range(uk):
        for r0 in range(0, 256, 16):
            groups = {slot(r0 + i, u, uk) % 16 for i in range(16)}
            assert len(groups) == 16, (uk, u, r0)


# ------------------------------------------------------------------ in-place tiles
# tile_inplace.h fills the same A layout from the caller's row-major A, and a k-major B
# layout from the caller's row-major B:
#   A, 16-byte loads: lane l of instruction ig takes unit u = ((l % UK) ^ (l / 16) ^ 4 ig) & (UK - 1)
#                     of row ig * (64 / UK) + l / UK (global byte row * row_bytes + 4u * 4);
#   A, 4-byte loads:  lane l of instruction ig writes LDS float ig * 64 + l, i.e. element l % 4 of
#                     physical unit s = ig * 16 + l / 4 = row * UK + c, whose logical unit is
#                     u = c ^ ((row / (16 / UK)) & (UK - 1)) (global element row, 4u + l % 4);
#   B slot of (k, unit u): k * UN + (u ^ (((k / HS) & 1) * 8)), HS = 4 (f32) or 8 (x3);
#   B, 16-byte loads: LDS unit s = ig * 64 + l is (k, physical unit) = divmod(s, UN);
#   B, 4-byte loads:  LDS float s = ig * 64 + l is (k, physical float) = divmod(s, BN).

def ip_bslot(k, u, un, hs):
    return k * un + (u ^ (((k // hs) & 1) * 8))


@pytest.mark.parametrize("uk", [4, 8])
@pytest.mark.parametrize("rows", [64, 128])
def test_inplace_a_loads_of_both_widths_fill_the_packed_layout(uk, rows):
    # 16-byte loads: every (row, unit) once, at the packed slot
    seen = {}
    for ig in range(rows * uk // 64):
        for lane in range(64):
            u = ((lane % uk) ^ (lane // 16) ^ (4 * ig)) & (uk - 1)
            row = ig * (64 // uk) + lane // uk
            assert (row, u) not in seen
            seen[(row, u)] = ig * 64 + lane
    assert len(seen) == rows * uk and all(s == slot(r, u, uk) for (r, u), s in seen.items())
    # 4-byte loads: every (row, k) once, at float e of the packed slot of its unit
    seen = {}
    for ig in range(rows * uk * 4 // 64):
        for lane in range(64):
            s = ig * 16 + lane // 4
            row, c = divmod(s, uk)
            u = c ^ ((row // (16 // uk)) & (uk - 1))
            k = 4 * u + lane % 4
            assert (row, k) not in seen
            seen[(row, k)] = ig * 64 + lane           # LDS float index
    assert len(seen) == rows * uk * 4
    for (row, k), f in seen.items():
        assert f == slot(row, k // 4, uk) * 4 + k % 4


@pytest.mark.parametrize("bn", [64, 128, 256])
@pytest.mark.parametrize("hs", [4, 8])
def test_inplace_b_loads_and_reads(bn, hs):
    bk, un = 16, bn // 4
    # 16-byte loads: LDS unit s holds (k, logical unit u) with ip_bslot(k, u) == s
    for s in range(bk * un):
        k, c = divmod(s, un)
        u = c ^ (((k // hs) & 1) * 8)
        assert ip_bslot(k, u, un, hs) == s
    # 4-byte loads: LDS float s holds column 4u + e of row k, at float e of the unit's slot
    cols = set()
    for s in range(bk * bn):
        k, d = divmod(s, bn)
        u, e = (d // 4) ^ (((k // hs) & 1) * 8), d % 4
        assert ip_bslot(k, u, un, hs) * 4 + e == s
        cols.add((k, 4 * u + e))
    assert len(cols) == bk * bn
    # operand reads: lanes 0-31 take 32 consecutive columns of row k, lanes 32-63 the same columns
    # of row k + hs; the 64 floats fall on 64 distinct banks (4 bytes each, 64 banks)
    for k in range(0, bk - hs):
        if (k // hs) % 2:
            continue
        for n0 in range(0, bn, 32):
            banks = set()
            for lane in range(64):
                kk = k + (hs if lane >= 32 else 0)
                n = n0 + lane % 32
                banks.add((ip_bslot(kk, n // 4, un, hs) * 4 + n % 4) % 64)
            assert len(banks) == 64, (bn, hs, k, n0)
