"""GPU parity of the 3x3 convolution layer (tgemm_conv3x3, an implicit gemm) against the
FP64 convolution oracle.

Operation: Y = alpha * conv3x3(X, Wt) + beta * Y, NHWC, stride 1, zero padding 1 (the
Conv layer of the Tiramisu paper's Section VI-A, built on its gemm).  Bars as for the
gemm: bit-exact on small-integer inputs (every partial sum an integer below 2^24),
normwise relative error <= 1e-5 for f32 and x3 on U[-1, 1] inputs.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import conv as OC

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def tg():
    from paper_1804_10694_amd import tgemm
    return tgemm


def _inputs(nb, H, W, cin, cout, seed, integer):
    g = torch.Generator().manual_seed(seed)
    if integer:
        X = torch.randint(-4, 5, (nb, H, W, cin), generator=g).float()
        Wt = torch.randint(-4, 5, (3, 3, cin, cout), generator=g).float()
        Y0 = torch.randint(-4, 5, (nb, H, W, cout), generator=g).float()
    else:
        X = 2 * torch.rand(nb, H, W, cin, generator=g) - 1
        Wt = 2 * torch.rand(3, 3, cin, cout, generator=g) - 1
        Y0 = 2 * torch.rand(nb, H, W, cout, generator=g) - 1
    return X, Wt, Y0


def _run(tg, X, Wt, Y0, alpha, beta, dtype, path="auto", shape=0):
    Yd = Y0.clone().to(DEV)
    tg.conv3x3(X.to(DEV), Wt.to(DEV), Yd, alpha, beta, dtype, path=path, shape=shape)
    torch.cuda.synchronize()
    return Yd.cpu()


# every kernel: the direct one and each packed tile shape (the host table is fixed, so the
# count is known without a GPU)
KERNELS = [("direct", 0)] + [("packed", i) for i in range(4)]

# ragged pixel counts, both direct tile sizes, packed tiles over one and several K panels
# (Cin 8: 72 = 9 * 8 taps, not a panel multiple), Cout with and without 16-byte filter rows
# and across several 128- and 256-column tiles
SHAPES = [(2, 5, 7, 8, 12), (3, 9, 11, 16, 13), (1, 16, 16, 64, 64), (2, 17, 19, 24, 130),
          (4, 24, 24, 32, 200), (1, 20, 23, 16, 300)]


@pytest.mark.parametrize("kernel", KERNELS, ids=lambda k: f"{k[0]}{k[1]}")
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_integer_inputs_bit_exact(tg, dtype, shape, kernel):
    print(f"conv {dtype} {shape} {kernel}", flush=True)
    X, Wt, Y0 = _inputs(*shape, seed=sum(shape), integer=True)
    ref = OC.conv3x3(X, Wt, Y0, 1.5, 0.5)
    got = _run(tg, X, Wt, Y0, 1.5, 0.5, dtype, *kernel)
    np.testing.assert_array_equal(got.numpy().astype(np.float64), ref, err_msg=f"{dtype} {shape} {kernel}")


def test_kernel_list_matches_library(tg):
    for dt in ("f32", "x3"):
        assert len(tg.conv3x3_packed_shapes(dt)) == len(KERNELS) - 1


def test_f32_four_channel_input(tg):
    # Cin = 4: one 16-byte unit per tap, K = 36 below one panel
    X, Wt, Y0 = _inputs(3, 7, 9, 4, 24, seed=75, integer=True)
    ref = OC.conv3x3(X, Wt, Y0, 1.0, -1.0)
    for kernel in KERNELS:
        got = _run(tg, X, Wt, Y0, 1.0, -1.0, "f32", *kernel)
        np.testing.assert_array_equal(got.numpy().astype(np.float64), ref, err_msg=str(kernel))


@pytest.mark.parametrize("shape", [(2, 13, 11, 32, 48), (1, 28, 28, 64, 96), (1, 9, 10, 512, 40)])
@pytest.mark.parametrize("dtype", ["f32", "x3"])
@pytest.mark.parametrize("path", ["direct", "packed"])
def test_uniform_inputs_within_tolerance(tg, dtype, shape, path):
    print(f"conv {dtype} {shape} {path}", flush=True)
    X, Wt, Y0 = _inputs(*shape, seed=7 + sum(shape), integer=False)
    ref = OC.conv3x3(X, Wt, Y0, 1.0, 1.0)
    err = oracle.normwise_error(_run(tg, X, Wt, Y0, 1.0, 1.0, dtype, path).numpy(), ref)
    print(f"{dtype} {shape} {path} normwise error {err:.3e}")
    assert err <= 1e-5


def test_same_result_as_explicit_im2col_gemm(tg):
    # the implicit gemm and the library's gemm on a materialised im2col matrix agree on
    # integer inputs bit for bit (both exact)
    nb, H, W, cin, cout = 2, 10, 9, 16, 40
    X, Wt, Y0 = _inputs(nb, H, W, cin, cout, seed=70, integer=True)
    Xp = torch.nn.functional.pad(X, (0, 0, 1, 1, 1, 1))
    cols = torch.cat([Xp[:, dy:dy + H, dx:dx + W, :] for dy in range(3) for dx in range(3)], dim=3)
    C = Y0.clone().reshape(-1, cout).to(DEV)
    tg.gemm(cols.reshape(-1, 9 * cin).contiguous().to(DEV), Wt.reshape(9 * cin, cout).to(DEV), C, 1.0, 0.5,
            "f32")
    for kernel in KERNELS:
        got = _run(tg, X, Wt, Y0, 1.0, 0.5, "f32", *kernel)
        assert torch.equal(got.reshape(-1, cout), C.cpu()), kernel


def test_degenerate_cases(tg):
    X, Wt, Y0 = _inputs(2, 6, 5, 8, 16, seed=71, integer=True)
    for kernel in KERNELS[:2]:
        # alpha == 0: Y = beta * Y, X and Wt not read (NaN there)
        nanX = torch.full_like(X, float("nan"))
        np.testing.assert_array_equal(_run(tg, nanX, Wt, Y0, 0.0, 0.5, "f32", *kernel).numpy(),
                                      (0.5 * Y0).numpy())
        # beta == 0 does not read Y (NaN there)
        got = _run(tg, X, Wt, torch.full_like(Y0, float("nan")), 1.0, 0.0, "x3", *kernel)
        np.testing.assert_array_equal(got.numpy().astype(np.float64), OC.conv3x3(X, Wt))
    # Cin not a multiple of the 16-byte unit is refused; empty batch is a no-op
    Xo, Wo, Yo = _inputs(1, 4, 4, 6, 8, seed=72, integer=True)
    with pytest.raises(tg.TgemmError):
        _run(tg, Xo, Wo, Yo, 1.0, 0.0, "f32")
    Xe = torch.zeros(0, 4, 4, 8, device=DEV)
    tg.conv3x3(Xe, Wt.to(DEV)[:, :, :8, :], torch.zeros(0, 4, 4, 16, device=DEV), 1.0, 0.0)


@pytest.mark.parametrize("dtype", ["f32", "x3"])
@pytest.mark.parametrize("path", ["auto", "direct"])
def test_full_size_layer_sampled(tg, dtype, path):
    # a 3x3 layer at the benchmark's size (batch 32, 56 x 56, 256 -> 256 channels), sampled
    # output pixels against the oracle, including image borders and corners
    nb, H, W, cin, cout = 32, 56, 56, 256, 256
    X, Wt, Y0 = _inputs(nb, H, W, cin, cout, seed=73, integer=False)
    got = _run(tg, X, Wt, Y0, 1.0, 1.0, dtype, path).reshape(-1, cout)
    rng = np.random.default_rng(74)
    pix = np.concatenate([rng.choice(nb * H * W, 400, replace=False),
                          [0, W - 1, (H - 1) * W, H * W - 1, nb * H * W - 1]])
    ref = OC.conv3x3(X, Wt, Y0, 1.0, 1.0, pixels=pix)
    err = oracle.normwise_error(got[torch.from_numpy(pix)].numpy(), ref)
    print(f"{dtype} full-size layer sampled normwise error {err:.3e}")
    assert err <= 1e-5


def test_packed_path_refuses_inputs_beyond_its_reach(tg):
    # X of 2^31 bytes or more is beyond the packed kernel's 32-bit buffer offsets: the packed
    # path is refused before any launch (pointers are never read), the direct one takes it
    X = torch.zeros(16, device=DEV)
    rc = tg.lib.tgemm_conv3x3_path(1, 1 << 15, 1 << 12, 4, 8, 1.0, X.data_ptr(), X.data_ptr(), 0.0,
                                   X.data_ptr(), 0, tg.CONV_PACKED, None)
    assert rc == 2


def test_graph_replay(tg):
    # the packed path (filter packing, x3 input split and the conv kernel) captured in a HIP
    # graph after a warm-up call has sized its workspace; every replay matches the eager result
    X, Wt, Y0 = _inputs(2, 12, 13, 16, 40, seed=76, integer=True)
    Xd, Wd = X.to(DEV), Wt.to(DEV)
    for dt in ("f32", "x3"):
        eager = Y0.clone().to(DEV)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            tg.conv3x3(Xd, Wd, eager, 1.0, 0.5, dt, stream=s)
        torch.cuda.synchronize()
        Yg = Y0.clone().to(DEV)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            tg.conv3x3(Xd, Wd, Yg, 1.0, 0.5, dt, stream=s)
        for _ in range(3):
            Yg.copy_(Y0.to(DEV))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(Yg, eager), dt


# ---------------------------------------------------------------- R x R filters (tgemm_conv2d)
def _inputs_r(nb, H, W, cin, cout, R, seed, integer):
    g = torch.Generator().manual_seed(seed)
    if integer:
        mk = lambda *s: torch.randint(-4, 5, s, generator=g).float()      # noqa: E731
    else:
        mk = lambda *s: 2 * torch.rand(*s, generator=g) - 1               # noqa: E731
    return mk(nb, H, W, cin), mk(R, R, cin, cout), mk(nb, H, W, cout)


def _run_r(tg, X, Wt, Y0, alpha, beta, dtype, path="auto", shape=0, runtime_r=False):
    Yd = Y0.clone().to(DEV)
    tg.conv2d(X.to(DEV), Wt.to(DEV), Yd, alpha, beta, dtype, path=path, shape=shape, runtime_r=runtime_r)
    torch.cuda.synchronize()
    return Yd.cpu()


@pytest.mark.parametrize("R", [1, 5, 7, 11])
@pytest.mark.parametrize("kernel", KERNELS, ids=lambda k: f"{k[0]}{k[1]}")
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_rxr_integer_inputs_bit_exact(tg, dtype, kernel, R):
    # ragged pixel counts (more than one 128-row tile), filter taps reaching past every border
    for shape in [(2, 9, 13, 8, 20), (1, 17, 15, 16, 130)]:
        print(f"conv{R}x{R} {dtype} {kernel} {shape}", flush=True)
        X, Wt, Y0 = _inputs_r(*shape, R, seed=R + sum(shape), integer=True)
        ref = OC.conv2d(X, Wt, Y0, 1.0, 0.5)
        got = _run_r(tg, X, Wt, Y0, 1.0, 0.5, dtype, *kernel)
        np.testing.assert_array_equal(got.numpy().astype(np.float64), ref, err_msg=f"R={R} {dtype} {kernel} {shape}")


@pytest.mark.parametrize("kernel", KERNELS, ids=lambda k: f"{k[0]}{k[1]}")
@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_3x3_through_the_runtime_r_kernels(tg, dtype, kernel):
    X, Wt, Y0 = _inputs_r(2, 11, 10, 16, 40, 3, seed=77, integer=True)
    got = _run_r(tg, X, Wt, Y0, 1.5, 0.5, dtype, *kernel, runtime_r=True)
    np.testing.assert_array_equal(got.numpy().astype(np.float64), OC.conv2d(X, Wt, Y0, 1.5, 0.5))


@pytest.mark.parametrize("dtype", ["f32", "x3"])
def test_5x5_uniform_within_tolerance(tg, dtype):
    X, Wt, Y0 = _inputs_r(2, 20, 18, 64, 96, 5, seed=78, integer=False)
    err = oracle.normwise_error(_run_r(tg, X, Wt, Y0, 1.0, 1.0, dtype).numpy(), OC.conv2d(X, Wt, Y0, 1.0, 1.0))
    print(f"5x5 {dtype} normwise error {err:.3e}")
    assert err <= 1e-5


def test_even_filter_is_refused(tg):
    X, _, Y0 = _inputs_r(1, 4, 4, 8, 8, 3, seed=79, integer=True)
    with pytest.raises(tg.TgemmError):
        _run_r(tg, X, torch.zeros(4, 4, 8, 8), Y0, 1.0, 0.0, "f32")
