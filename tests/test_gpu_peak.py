"""The matrix-core throughput probe (tgemm_mfma_loop) runs for every MFMA form it offers,
reports the flops it launched, and refuses bad arguments."""
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    return tgemm


@pytest.mark.parametrize("dtype,per", [("f32", 4096), ("bf16", 32768), ("fp8", 131072)])
def test_probe_runs_and_counts_flops(tg, dtype, per):
    sink = torch.full((8192,), float("nan"), device=DEV)
    fl = tg.mfma_loop(dtype, 10, sink)
    torch.cuda.synchronize()
    assert fl == per * 4 * 10 * 8192
    assert torch.isfinite(sink).all()            # every wave wrote its sum


def test_probe_rejects_bad_arguments(tg):
    short = torch.zeros(100, device=DEV)
    with pytest.raises(tg.TgemmError):
        tg.mfma_loop("f32", 10, short)
    with pytest.raises(tg.TgemmError):
        tg.mfma_loop("x3", 10, torch.zeros(8192, device=DEV))
