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
