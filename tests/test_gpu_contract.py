"""GPU parity of the tensor contraction (tgemm_contract) against the FP64 oracle.

Operation: C[modes_c] = alpha * sum A[modes_a] B[modes_b] + beta * C over the modes C lacks
(the dense tensor contraction of the Tiramisu paper's Baryon benchmark, Section VI-A), run
as gemms after copying operands into [batch, row, contracted] order where needed.  Bars as
for the gemm: bit-exact on small-integer inputs, normwise <= 1e-5 on U[-1, 1] inputs.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import contract as OT

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    yield tgemm
    tgemm.shutdown()


def _tensor(shape, g, integer):
    if integer:
        return torch.randint(-3, 4, shape, generator=g).float()
    return 2 * torch.rand(shape, generator=g) - 1


# (modes and extents of A, of B, of C): labels are arbitrary integers
CASES = {
    "matrix": (([0, 1], [33, 20]), ([1, 2], [20, 45]), ([0, 2], [33, 45])),
    "batched": (([9, 0, 1], [5, 40, 24]), ([9, 1, 2], [5, 24, 70]), ([9, 0, 2], [5, 40, 70])),
    "permuted_operands": (([1, 9, 0], [24, 5, 40]), ([9, 2, 1], [5, 70, 24]), ([9, 0, 2], [5, 40, 70])),
    "permuted_result": (([9, 0, 1], [4, 30, 17]), ([9, 1, 2], [4, 17, 22]), ([2, 9, 0], [22, 4, 30])),
    "two_row_two_contracted": (([0, 5, 3, 6], [6, 3, 7, 4]), ([6, 8, 5], [4, 9, 3]), ([3, 8, 0], [7, 9, 6])),
    "outer": (([0], [50]), ([1], [37]), ([0, 1], [50, 37])),
    "dot": (([4], [300]), ([4], [300]), ([], [])),
    "batched_dot": (([2, 4], [64, 129]), ([2, 4], [64, 129]), ([2], [64])),
    "site_blocks": (([7, 0, 1], [300, 12, 12]), ([7, 1, 2], [300, 12, 12]), ([7, 0, 2], [300, 12, 12])),
}


def _run(tg, case, dtype, alpha, beta, integer, seed):
    (ma, ea), (mb, eb), (mc, ec) = CASES[case]
    g = torch.Generator().manual_seed(seed)
    A, B, C0 = _tensor(ea, g, integer), _tensor(eb, g, integer), _tensor(ec, g, integer)
    C = C0.clone().to(DEV)
    tg.contract(A.to(DEV), ma, B.to(DEV), mb, C, mc, alpha, beta, dtype)
    torch.cuda.synchronize()
    return C.cpu(), OT.contract(A, ma, B, mb, mc, C0, alpha, beta)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_integer_inputs_bit_exact(tg, dtype, case):
    print(f"contract {dtype} {case}", flush=True)
    got, ref = _run(tg, case, dtype, 1.5, 0.5, True, seed=len(case))
    np.testing.assert_array_equal(got.numpy().astype(np.float64), ref, err_msg=f"{dtype} {case}")


@pytest.mark.parametrize("case", ["permuted_operands", "two_row_two_contracted", "batched_dot"])
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_uniform_inputs_within_tolerance(tg, dtype, case):
    got, ref = _run(tg, case, dtype, 1.0, 1.0, False, seed=7)
    err = oracle.normwise_error(got.numpy(), ref)
    print(f"{dtype} {case} normwise error {err:.3e}")
    assert err <= 1e-5


def test_degenerate_and_invalid(tg):
    g = torch.Generator().manual_seed(11)
    A, B = _tensor((6, 0), g, True).to(DEV), _tensor((0, 5), g, True).to(DEV)
    C0 = _tensor((6, 5), g, True)
    C = C0.clone().to(DEV)
    tg.contract(A, [0, 1], B, [1, 2], C, [0, 2], 1.0, 0.5)          # no contracted element: C = beta C
    torch.cuda.synchronize()
    np.testing.assert_array_equal(C.cpu().numpy(), (0.5 * C0).numpy())
    A2, B2 = _tensor((6, 4), g, True).to(DEV), _tensor((4, 5), g, True).to(DEV)
    C = torch.full((6, 5), float("nan"), device=DEV)                 # beta == 0 does not read C
    tg.contract(A2, [0, 1], B2, [1, 2], C, [0, 2], 1.0, 0.0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(C.cpu().numpy().astype(np.float64), OT.contract(A2.cpu(), [0, 1], B2.cpu(), [1, 2], [0, 2]))
    with pytest.raises(tg.TgemmError):                               # one label, two extents
        tg.contract(A2, [0, 1], torch.zeros(3, 5, device=DEV), [1, 2], torch.zeros(6, 5, device=DEV), [0, 2])
    with pytest.raises(tg.TgemmError):                               # a label twice in one tensor
        tg.contract(A2, [0, 0], B2, [1, 2], torch.zeros(6, 5, device=DEV), [0, 2])
    with pytest.raises(tg.TgemmError):                               # a mode summed within A alone
        tg.contract(torch.zeros(6, 4, 2, device=DEV), [0, 1, 3], B2, [1, 2], torch.zeros(6, 5, device=DEV), [0, 2])


def test_graph_replay_after_planning(tg):
    # the copies, the grouped launch and the copy back captured once the workspace and the
    # grouped plan exist; replays match the eager result
    (ma, ea), (mb, eb), (mc, ec) = CASES["permuted_result"]
    g = torch.Generator().manual_seed(12)
    A, B, C0 = (_tensor(e, g, True).to(DEV) for e in (ea, eb, ec))
    s = torch.cuda.Stream()
    eager = C0.clone()
    with torch.cuda.stream(s):
        tg.contract(A, ma, B, mb, eager, mc, 1.0, 0.5, "x3", stream=s)
    torch.cuda.synchronize()
    Cg = C0.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        tg.contract(A, ma, B, mb, Cg, mc, 1.0, 0.5, "x3", stream=s)
    for _ in range(3):
        Cg.copy_(C0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(Cg, eager)
