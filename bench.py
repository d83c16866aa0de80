"""Benchmark of the gemm hot path on one MI355X.

Workload (one "step"): C = alpha*A*B + beta*C with alpha = beta = 1 on seeded
U[-1, 1] float32 inputs, for
  - M = N = K = 8192 (seed 2), plain F32 and split-bf16x3;
  - the ragged M = 4097, N = 3001, K = 2053 (seed 3, partial tiles), plain F32
    and split-bf16x3.
Inputs are resident in device memory before the timed region starts.  A step
is the four launches, stream-ordered on torch's current stream; `value` is the
step's algorithmic flops (2*M*N*K per gemm) divided by its wall time.  Every
launch is also bracketed by HIP events, which give the per-path kernel time
and the roofline of the dominant kernel.

The cpu_baseline leg times the FP64 oracle on a bounded sample of rows of the
8192^3 product (about ten seconds of host work) and reuses those rows to report
the GPU paths' sampled normwise error; the ragged paths get their own sample of
rows.  Every other row below reports its error against the oracle too, computed
outside its timed region: sampled rows (16384^3 against both the dequantised and
the unquantised inputs, the back-to-back pair), sampled output pixels
(convolutions), the worst problem (grouped launch) or the whole result (256^3).

The 256^3 row (seed 1, alpha = 1.5, beta = 0.5, plain F32 and split-bf16x3) is
timed on its own: it is bound by launch latency, so it is reported in
microseconds and kept out of the step.

The matrix-core and HBM-copy probes run before the timed steps and again after
the extra rows; both are reported, with the shader clock read from sysfs when
the driver exposes it.

The extra_rows leg (outside the step and its value) measures the other rows of
the path on their own workloads:
  - per-128x128-tile scaled gemm at 16384^3 (A, B ~ N(0,1) with 1% of rows x1e3,
    seed 30), quantised on the GPU, e4m3 and bf16, alpha = 1, beta = 0;
  - a 3x3 convolution layer (batch 32, 56 x 56, 256 -> 256 channels, NHWC, seed 5) as an
    implicit gemm, F32 and split-bf16x3, beside a materialised im2col matrix fed to the gemm;
  - a back-to-back pair of 256-wide layers over the same 100352 pixels, E = relu(A B) D with
    relu(A B) kept on chip (U[-1, 1], seed 6), beside two gemm calls with the ReLU between;
  - 5 x 5 and 7 x 7 layers (batch 32, 56 x 56, 128 -> 128 channels, seed 8), and the 3 x 3
    layer through the kernels that take the filter size at run time;
  - two synthetic tensor contractions (seed 7): 64 products of 256^3 whose operands need
    reordering, and 16384 site blocks of 12 x 12 x 12;
  - the grouped persistent launch over 512 problems with M, N, K log-uniform in
    [16, 2048] (seed 4, matrices from seeds 4000 + p), alpha = 1, beta = 0.5,
    F32 and split-bf16x3, tile shapes tuned on the set (tgemm_batched_autotune),
    replayed from a HIP graph.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-extras] [--extras-only]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

KERNEL_SOURCES = ["paper_1804_10694_amd/csrc/tile_f32x3.h", "paper_1804_10694_amd/csrc/gemm_tile.hip",
                  "paper_1804_10694_amd/csrc/tile_packed.h",
                  "paper_1804_10694_amd/csrc/gemm_packed.hip", "paper_1804_10694_amd/csrc/kargs.h"]
TRAFFIC_FILE = "profiles/traffic.json"

PEAK_TFLOPS = {"f32": 157.3, "x3": 2516.6 / 3.0,   # MI355X dense: FP32 MFMA; bf16 MFMA / 3
               "bf16": 2516.6, "fp8": 5033.2}
HBM_PEAK_GBS = 8000.0


def cpu_model():
    """The host CPU's model string (as lscpu prints it), from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def shader_clock_mhz():
    """Current shader clock of the first GPU that exposes pp_dpm_sclk (the line marked
    '*'), or None."""
    import glob
    for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            with open(path) as f:
                for line in f:
                    if line.rstrip().endswith("*"):
                        return int("".join(ch for ch in line.split(":", 1)[1] if ch.isdigit()))
        except (OSError, ValueError, IndexError):
            continue
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras-only", action="store_true",
                    help="run only the extra rows (for profiling them) and print them as JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with one plain 1 GiB device copy (reference for the HBM counters)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target host time of the oracle sample")
    return ap.parse_args()


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_symbol):
    """HBM bytes per call of `kernel_symbol` ("schedule key@MxNxK") from the committed counter
    summary (written by paper_1804_10694_amd.profsum), or None
    when there is none or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    rec = table.get(kernel_symbol)
    if not rec or rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline(A, B, C0, dev_results, seconds):
    """Times the oracle on sampled rows of the 8192^3 problem; returns (baseline, errors)."""
    import numpy as np
    import oracle

    M, K = A.shape
    N = B.shape[1]
    Bn = B.numpy()
    rng = np.random.default_rng(2)
    # calibration on a few rows, then a sample sized to the time budget
    probe = np.sort(rng.choice(M, size=2 * oracle.num_threads(), replace=False))
    t0 = time.perf_counter()
    oracle.gemm_rows(A.numpy(), Bn, C0.numpy(), 1.0, 1.0, probe)
    rows_per_s = len(probe) / (time.perf_counter() - t0)
    nrows = int(max(8, min(M, seconds * rows_per_s)))
    rows = np.sort(rng.choice(M, size=nrows, replace=False))
    t0 = time.perf_counter()
    ref = oracle.gemm_rows(A.numpy(), Bn, C0.numpy(), 1.0, 1.0, rows)
    dt = time.perf_counter() - t0
    flops = 2.0 * nrows * N * K
    base = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": oracle.num_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"{nrows} of {M} rows of the 8192^3 F32 problem (FP64 i-k-j loop, "
                      f"{dt:.1f} s, {flops:.3e} flops)"}
    errors = {}
    for name, C in dev_results.items():
        errors[name] = oracle.normwise_error(C[rows], ref)
    return base, errors


def oracle_checks(checks):
    """Errors of the other rows against the oracle (part of the cpu_baseline leg): each
    check holds the row's host inputs and the GPU's result (sampled where the oracle
    would take long); returns {row name: {error name: value}}."""
    import numpy as np
    import oracle
    from oracle import conv as oconv
    from oracle import gemm2 as ogemm2
    from oracle import precision as P

    out = {}
    for c in checks:
        kind, name = c["kind"], c["row"]
        if kind == "gemm":           # whole result
            ref = oracle.gemm(c["A"], c["B"], c["C0"], c["alpha"], c["beta"])
            out[name] = {"normwise_error": oracle.normwise_error(c["got"], ref)}
        elif kind == "gemm_rows":    # sampled rows
            ref = oracle.gemm_rows(c["A"], c["B"], c["C0"], c["alpha"], c["beta"], c["rows"])
            out[name] = {"sampled_normwise_error": oracle.normwise_error(c["got"], ref),
                         "sample": f"{len(c['rows'])} rows"}
        elif kind == "scaled":       # sampled rows against dequantised and unquantised inputs
            rows, dt = c["rows"], c["dtype"]
            Arows = np.stack([P.decode(q, dt) for q in c["QA_rows"]])
            for n, r in enumerate(rows):
                Arows[n] *= np.repeat(c["SA"][r // 128].astype(np.float64), 128)[:Arows.shape[1]]
            Bd = P.dequantize_tiles(P.decode(c["QB"], dt), c["SB"], 128)
            deq = oracle.gemm(Arows, Bd, None, 1.0, 0.0)
            del Bd
            unq = oracle.gemm_rows(c["A"], c["B"], None, 1.0, 0.0, rows)
            out[name] = {"sampled_normwise_error_vs_dequantised": oracle.normwise_error(c["got"], deq),
                         "sampled_normwise_error_vs_unquantised": oracle.normwise_error(c["got"], unq),
                         "sample": f"{len(rows)} rows"}
        elif kind == "conv":         # sampled output pixels
            ref = oconv.conv2d(c["X"], c["Wt"], c["Y0"], c["alpha"], c["beta"], pixels=c["pixels"])
            out[name] = {"sampled_normwise_error": oracle.normwise_error(c["got"], ref),
                         "sample": f"{len(c['pixels'])} output pixels"}
        elif kind == "gemm2":        # sampled rows
            ref = ogemm2.gemm2(c["A"], c["B"], c["D"], c["E0"], c["alpha"], c["beta"], c["relu"],
                               rows=c["rows"])
            out[name] = {"sampled_normwise_error": oracle.normwise_error(c["got"], ref),
                         "sample": f"{len(c['rows'])} rows"}
        elif kind == "grouped":      # every problem; the worst one is reported
            worst = 0.0
            for (A, B, C0), got in zip(c["host"], c["got"]):
                ref = oracle.gemm(A, B, C0, c["alpha"], c["beta"])
                worst = max(worst, oracle.normwise_error(got, ref))
            out[name] = {"worst_problem_normwise_error": worst}
    return out


def measured_peaks(tg):
    """What the chip delivers at its running clock: the matrix-core probe (independent MFMA
    chains on every SIMD) per dtype, and a 1 GiB device copy for HBM (read + write bytes)."""
    import torch
    dev = torch.device("cuda:0")
    sink = torch.zeros(8192, device=dev)
    out = {}
    for dt, key in (("f32", "f32_mfma_tflops"), ("bf16", "bf16_mfma_tflops"), ("fp8", "fp8_mfma_tflops")):
        fl = tg.mfma_loop(dt, 10000, sink)
        _, med = _time_events(lambda: tg.mfma_loop(dt, 10000, sink), 3, warmup=1)
        out[key] = round(fl / (med * 1e-3) / 1e12, 1)
    src = torch.empty(2 ** 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    _, med = _time_events(lambda: dst.copy_(src), 5, warmup=1)
    out["hbm_copy_gbs"] = round(2 * 2 ** 30 / (med * 1e-3) / 1e9, 1)
    out["shader_clock_mhz"] = shader_clock_mhz()
    del src, dst, sink
    torch.cuda.empty_cache()
    return out


def _time_events(fn, reps, warmup=2):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        evs.append((e0, e1))
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in evs)
    return sum(ts) / len(ts), ts[len(ts) // 2]


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _sample_rows(n, count, seed):
    import numpy as np
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(n, count), replace=False))


def extra_rows(tg, inputs, checks):
    """The other rows of the path on their own workloads; `checks` receives what the
    oracle needs to state each row's error (host inputs, sampled GPU results)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    out = {}
    n = 16384
    A, B = inputs.lowprec_inputs(n, n, n, seed=30)
    Ad, Bd = A.to(dev), B.to(dev)
    C = torch.empty(n, n, device=dev)
    flops = 2.0 * n ** 3
    srows = _sample_rows(n, 4, 30)
    srows_d = torch.from_numpy(srows).to(dev)
    for dt in ("fp8", "bf16"):
        qa, sa = tg.quantize_tiles(Ad, dt)
        qb, sb = tg.quantize_tiles(Bd, dt)
        q_avg, _ = _time_events(lambda: tg.quantize_tiles(Ad, dt), 5)
        avg, med = _time_events(lambda: tg.gemm_scaled(qa, sa, qb, sb, C, 1.0, 0.0, dt), 10)
        tf = flops / (avg * 1e-3) / 1e12
        es = 1 if dt == "fp8" else 2
        row = f"scaled_{dt}_16384"
        out[row] = {
            "avg_ms": round(avg, 4), "median_ms": round(med, 4), "tflops": round(tf, 1),
            "peak_tflops": PEAK_TFLOPS[dt], "frac_peak": round(tf / PEAK_TFLOPS[dt], 4),
            "schedule": tg.select_schedule(n, n, n, dt),
            "quantize_ms_per_matrix": round(q_avg, 4),
            "quantize_hbm_frac": round(n * n * (4 + es) / (q_avg * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "algorithmic_bytes": 2 * n * n * es + 4 * n * n}
        view = np.uint16 if dt == "bf16" else np.uint8
        checks.append({"kind": "scaled", "row": row, "dtype": dt, "rows": srows, "A": A, "B": B,
                       "got": C[srows_d].cpu().numpy(),
                       "QA_rows": qa[srows_d].cpu().numpy().view(view), "SA": sa.cpu().numpy(),
                       "QB": qb.cpu().numpy().view(view), "SB": sb.cpu().numpy()})
        del qa, qb
    del Ad, Bd, C
    torch.cuda.empty_cache()

    progress("scaled 16384^3 rows done")
    # 3x3 convolution layer as an implicit gemm, against a materialised im2col matrix
    # (built with torch ops) fed to the gemm
    nb, H, W, cin, cout = 32, 56, 56, 256, 256
    Xh, Wth, Y0h = inputs.conv_layer_inputs(nb, H, W, cin, cout, 5)
    X, Wt, Y0 = Xh.to(dev), Wth.to(dev), Y0h.to(dev)
    cflops = 2.0 * nb * H * W * cout * 9 * cin
    pix = np.concatenate([_sample_rows(nb * H * W, 256, 5), [0, W - 1, (H - 1) * W, nb * H * W - 1]])
    pix_d = torch.from_numpy(pix).to(dev)
    for dt in ("f32", "x3"):
        Y = Y0.clone()
        avg, med = _time_events(lambda: tg.conv3x3(X, Wt, Y, 1.0, 0.0, dt), 10)
        d_avg, _ = _time_events(lambda: tg.conv3x3(X, Wt, Y, 1.0, 0.0, dt, path="direct"), 10)
        r_avg, _ = _time_events(lambda: tg.conv2d(X, Wt, Y, 1.0, 0.0, dt, runtime_r=True), 10)
        tg.conv3x3(X, Wt, Y, 1.0, 0.0, dt)
        torch.cuda.synchronize()
        row = f"conv3x3_{dt}_b32_56x56_256"
        checks.append({"kind": "conv", "row": row, "X": Xh, "Wt": Wth, "Y0": None, "alpha": 1.0,
                       "beta": 0.0, "pixels": pix, "got": Y.reshape(-1, cout)[pix_d].cpu().numpy()})

        def im2col():
            Xp = torch.nn.functional.pad(X, (0, 0, 1, 1, 1, 1))
            return torch.cat([Xp[:, dy:dy + H, dx:dx + W, :] for dy in range(3) for dx in range(3)],
                             dim=3).reshape(nb * H * W, 9 * cin)
        cols = im2col()
        Wm = Wt.reshape(9 * cin, cout)
        Ym = Y0.reshape(nb * H * W, cout).clone()
        i_avg, _ = _time_events(im2col, 5)
        g_avg, _ = _time_events(lambda: tg.gemm(cols, Wm, Ym, 1.0, 0.0, dt), 10)
        out[row] = {
            "avg_ms": round(avg, 4), "median_ms": round(med, 4), "tflops": round(cflops / (avg * 1e-3) / 1e12, 2),
            "peak_tflops": round(PEAK_TFLOPS[dt], 1),
            "frac_peak": round(cflops / (avg * 1e-3) / 1e12 / PEAK_TFLOPS[dt], 4),
            "direct_kernel_ms": round(d_avg, 4),
            "runtime_filter_size_ms": round(r_avg, 4), "specialised_over_runtime": round(r_avg / avg, 3),
            "im2col_materialised_ms": round(i_avg, 4), "gemm_on_im2col_ms": round(g_avg, 4),
            "implicit_over_materialised": round((i_avg + g_avg) / avg, 3)}
        del cols, Ym, Y
    del X, Wt, Y0
    torch.cuda.empty_cache()

    # 5 x 5 and 7 x 7 layers (batch 32, 56 x 56, 128 -> 128 channels, seed 8): R at run time
    for R in (5, 7):
        Xh, Wth, Y0h = inputs.conv_layer_inputs(nb, H, W, 128, 128, 8, R)
        X, Wt, Y0 = Xh.to(dev), Wth.to(dev), Y0h.to(dev)
        rflops = 2.0 * nb * H * W * 128 * R * R * 128
        for dt in ("f32", "x3"):
            Y = Y0.clone()
            avg, med = _time_events(lambda: tg.conv2d(X, Wt, Y, 1.0, 0.0, dt), 10)
            row = f"conv{R}x{R}_{dt}_b32_56x56_128"
            out[row] = {
                "avg_ms": round(avg, 4), "median_ms": round(med, 4),
                "tflops": round(rflops / (avg * 1e-3) / 1e12, 2), "peak_tflops": round(PEAK_TFLOPS[dt], 1),
                "frac_peak": round(rflops / (avg * 1e-3) / 1e12 / PEAK_TFLOPS[dt], 4)}
            checks.append({"kind": "conv", "row": row, "X": Xh, "Wt": Wth, "Y0": None, "alpha": 1.0,
                           "beta": 0.0, "pixels": pix, "got": Y.reshape(-1, 128)[pix_d].cpu().numpy()})
        del X, Wt, Y0, Y
    torch.cuda.empty_cache()

    # back-to-back gemm E = act(A B) D with act(A B) on chip, against two library gemms with
    # the ReLU between (the intermediate through memory)
    M, K, N1, N2 = nb * H * W, 256, 256, 256
    g = torch.Generator().manual_seed(6)
    host2 = [(2 * torch.rand(r, c, generator=g) - 1) for r, c in ((M, K), (K, N1), (N1, N2), (M, N2))]
    A2, B2, D2, E2 = (t.to(dev) for t in host2)
    T2 = torch.empty(M, N1, device=dev)
    fflops = 2.0 * M * N1 * (K + N2)
    grows = _sample_rows(M, 256, 6)
    for dt in ("f32", "x3"):
        avg, med = _time_events(lambda: tg.gemm2(A2, B2, D2, E2, 1.0, 0.0, True, dt), 10)
        row = f"gemm2_relu_{dt}_{M}x{K}x{N1}x{N2}"
        torch.cuda.synchronize()
        checks.append({"kind": "gemm2", "row": row, "A": host2[0], "B": host2[1], "D": host2[2], "E0": None,
                       "alpha": 1.0, "beta": 0.0, "relu": True, "rows": grows,
                       "got": E2[torch.from_numpy(grows).to(dev)].cpu().numpy()})

        def unfused():
            tg.gemm(A2, B2, T2, 1.0, 0.0, dt)
            torch.relu_(T2)
            tg.gemm(T2, D2, E2, 1.0, 0.0, dt)
        u_avg, _ = _time_events(unfused, 10)
        out[row] = {
            "avg_ms": round(avg, 4), "median_ms": round(med, 4), "tflops": round(fflops / (avg * 1e-3) / 1e12, 2),
            "peak_tflops": round(PEAK_TFLOPS[dt], 1),
            "frac_peak": round(fflops / (avg * 1e-3) / 1e12 / PEAK_TFLOPS[dt], 4),
            "unfused_ms": round(u_avg, 4), "fused_over_unfused": round(u_avg / avg, 3)}
    del A2, B2, D2, E2, T2
    torch.cuda.empty_cache()

    # tensor contractions (synthetic; the Baryon benchmark's own tensors are not available):
    # a batched contraction whose operands need reordering, and many 12 x 12 site blocks
    g = torch.Generator().manual_seed(7)
    work = {
        "contract_permuted_64x256x256x256": (([1, 9, 0], (256, 64, 256)), ([9, 2, 1], (64, 256, 256)),
                                             ([9, 0, 2], (64, 256, 256))),
        "contract_site_blocks_16384x12x12x12": (([7, 0, 1], (16384, 12, 12)), ([7, 1, 2], (16384, 12, 12)),
                                                ([7, 0, 2], (16384, 12, 12))),
    }
    for name, ((ma, ea), (mb, eb), (mc, ec)) in work.items():
        At = (2 * torch.rand(ea, generator=g) - 1).to(dev)
        Bt = (2 * torch.rand(eb, generator=g) - 1).to(dev)
        Ct = torch.zeros(ec, device=dev)
        ext = dict(zip(ma, ea))
        ext.update(zip(mb, eb))
        cfl = 2.0
        for m in ext:
            cfl *= ext[m]
        for dt in ("f32", "x3"):
            avg, med = _time_events(lambda: tg.contract(At, ma, Bt, mb, Ct, mc, 1.0, 0.0, dt), 10)
            out[f"{name}_{dt}"] = {"avg_ms": round(avg, 4), "median_ms": round(med, 4),
                                   "tflops": round(cfl / (avg * 1e-3) / 1e12, 3)}
        del At, Bt, Ct
    tg.shutdown()
    torch.cuda.empty_cache()

    progress("convolution, back-to-back and contraction rows done")
    dims = inputs.grouped_dims()
    host = inputs.grouped_inputs(dims, 4000)
    As = [h[0].to(dev) for h in host]
    Bs = [h[1].to(dev) for h in host]
    C0s = [h[2].to(dev) for h in host]
    Cs = [c.clone() for c in C0s]
    gflops = float(sum(2.0 * m * n_ * k for m, n_, k in dims))
    gbytes = float(sum(4.0 * (m * k + k * n_ + 2 * m * n_) for m, n_, k in dims))
    for dt in ("f32", "x3"):
        al, be = [1.0] * len(dims), [0.5] * len(dims)
        shape = tg.gemm_batched_autotune(As, Bs, Cs, al, be, dt, reps=5)   # plan shape
        tg.gemm_batched(As, Bs, Cs, al, be, dt)          # plans
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            tg.gemm_batched(As, Bs, Cs, al, be, dt)
        avg, med = _time_events(graph.replay, 20)
        # one replay from the initial C, for the error against the oracle
        for c, c0 in zip(Cs, C0s):
            c.copy_(c0)
        graph.replay()
        torch.cuda.synchronize()
        row = f"grouped_{dt}_512"
        checks.append({"kind": "grouped", "row": row, "host": host, "alpha": 1.0, "beta": 0.5,
                       "got": [c.cpu().numpy() for c in Cs]})
        floor_ms = max(gflops / (PEAK_TFLOPS[dt] * 1e12), gbytes / (HBM_PEAK_GBS * 1e9)) * 1e3
        out[row] = {
            "avg_ms": round(avg, 4), "median_ms": round(med, 4),
            "gemm_per_s": round(len(dims) / (avg * 1e-3), 1),
            "tflops": round(gflops / (avg * 1e-3) / 1e12, 2),
            "hbm_gbs_compulsory": round(gbytes / (avg * 1e-3) / 1e9, 1),
            "floor_ms": round(floor_ms, 4), "frac_of_floor": round(floor_ms / avg, 4),
            "tile128_threshold": shape["threshold"], "packed_256_threshold": shape["large"],
            "tile128_cost_ratio_permille": shape["ratio"],
            "bound": "mfma" if gflops / (PEAK_TFLOPS[dt] * 1e12) > gbytes / (HBM_PEAK_GBS * 1e9)
            else "hbm"}
        del graph
    return out


def small_gemm_row(tg, inputs, checks):
    """The 256^3 gemm (seed 1, alpha 1.5, beta 0.5): bound by launch latency, timed alone
    (median of 30 launches after 5 warm-ups, in microseconds)."""
    import torch
    dev = torch.device("cuda:0")
    A, B, C0 = inputs.gemm_inputs(256, 256, 256, seed=1)
    Ad, Bd = A.to(dev), B.to(dev)
    out = {}
    for dt in ("f32", "x3"):
        C = C0.to(dev)
        avg, med = _time_events(lambda: tg.gemm(Ad, Bd, C, 1.5, 0.5, dt), 30, warmup=5)
        C = C0.to(dev)
        tg.gemm(Ad, Bd, C, 1.5, 0.5, dt)
        torch.cuda.synchronize()
        row = f"{dt}_256x256x256"
        checks.append({"kind": "gemm", "row": row, "A": A, "B": B, "C0": C0, "alpha": 1.5, "beta": 0.5,
                       "got": C.cpu().numpy()})
        out[row] = {"median_us": round(med * 1e3, 2), "avg_us": round(avg * 1e3, 2),
                    "tflops": round(2.0 * 256 ** 3 / (med * 1e-3) / 1e12, 3),
                    "schedule": tg.select_schedule(256, 256, 256, dt), "alpha": 1.5, "beta": 0.5}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1804_10694_amd import inputs
    from paper_1804_10694_amd import tgemm as tg

    dev = torch.device("cuda:0")
    tg.set_policy("default")
    checks = []
    if args.extras_only:
        print(json.dumps({"extra_rows": extra_rows(tg, inputs, checks)}))
        return
    peaks_before = measured_peaks(tg)
    progress(f"probes before the timed steps: {peaks_before}")
    small = small_gemm_row(tg, inputs, checks)
    progress("256^3 row done")
    sq = (8192, 8192, 8192)
    rg = (4097, 3001, 2053)
    host = {sq: inputs.gemm_inputs(*sq, seed=2), rg: inputs.gemm_inputs(*rg, seed=3)}
    devm = {s: tuple(t.to(dev) for t in host[s]) for s in host}
    C = {s: devm[s][2].clone() for s in host}
    paths = [("f32", sq), ("x3", sq), ("f32", rg), ("x3", rg)]

    def flops(shape):
        return 2.0 * shape[0] * shape[1] * shape[2]

    def launch(dt, s):
        A, B, _ = devm[s]
        tg.gemm(A, B, C[s], 1.0, 1.0, dt)

    for _ in range(args.warmup):
        for dt, s in paths:
            launch(dt, s)
    torch.cuda.synchronize()

    ev = {p: [] for p in paths}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for p in paths:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            launch(*p)
            e1.record()
            ev[p].append((e0, e1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    progress(f"{args.steps} timed steps: {ms_per_step:.3f} ms per step")
    step_flops = sum(flops(s) for _, s in paths)
    value = step_flops / (ms_per_step * 1e-3) / 1e12

    per_path = {}
    for (dt, s), lst in ev.items():
        times = sorted(a.elapsed_time(b) for a, b in lst)
        avg = sum(times) / len(times)
        med = times[len(times) // 2]
        tf = flops(s) / (avg * 1e-3) / 1e12
        sched = tg.select_schedule(*s, dt)
        info = tg.schedule_info(sched[0])
        tiles = -(-s[0] // info["BM"]) * -(-s[1] // info["BN"])
        per_path[f"{dt}_{s[0]}x{s[1]}x{s[2]}"] = {
            "avg_ms": round(avg, 4), "median_ms": round(med, 4), "tflops": round(tf, 2),
            "peak_tflops": round(PEAK_TFLOPS[dt], 1), "frac_peak": round(tf / PEAK_TFLOPS[dt], 4),
            "schedule": sched, "schedule_key": tg.schedule_key(sched[0]),
            "packed": info["vec"] == 0, "stream_k": info["split"] == 1, "inplace": info["inplace"] == 1,
            # threads of the main kernel's grid: how a profile tells the paths apart (a
            # stream-K form launches one resident wave instead, and is told by its name)
            "grid_threads": None if info["split"] else tiles * 64 * info["WGM"] * info["WGN"]}

    # dominant kernel = the path with the largest share of the step
    dom_key = max(per_path, key=lambda k: per_path[k]["avg_ms"])
    dom = per_path[dom_key]
    dt_dom, shape_dom = [p for p in paths if f"{p[0]}_{p[1][0]}x{p[1][1]}x{p[1][2]}" == dom_key][0]
    sym = f"{dom['schedule_key']}@{shape_dom[0]}x{shape_dom[1]}x{shape_dom[2]}"
    # a packed schedule's call is three kernels (A packing, B packing, main kernel);
    # the events, and so `achieved`, cover the whole call
    roofline = {"bound": "mfma", "kernel": dom_key, "kernel_symbol": sym,
                "kernels_per_call": (["pack_rows_kernel", "pack_cols_kernel", "packed_kernel"]
                                     if dom["packed"] else ["inplace_gemm_kernel"] if dom["inplace"]
                                     else ["gemm_kernel"]),
                "achieved": dom["tflops"],
                "peak": dom["peak_tflops"], "unit": "TFLOP/s",
                "frac": round(dom["tflops"] / dom["peak_tflops"], 4),
                "traffic": measured_traffic(sym), "traffic_unit": "HBM bytes per call",
                "compulsory_bytes": 4 * (shape_dom[0] * shape_dom[2] + shape_dom[2] * shape_dom[1]
                                         + 2 * shape_dom[0] * shape_dom[1]),
                "kernel_source_sha256": kernel_source_hash()}

    # fresh results for the error report (outside the timed region): whole 8192^3 results
    # (sampled by the cpu_baseline leg) and sampled rows of the ragged ones
    results = {}
    rrows = _sample_rows(rg[0], 256, 3)
    for dt, s in paths:
        Cx = devm[s][2].clone()
        A, B, _ = devm[s]
        tg.gemm(A, B, Cx, 1.0, 1.0, dt)
        torch.cuda.synchronize()
        if s == sq:
            results[dt] = Cx.cpu().numpy()
        else:
            checks.append({"kind": "gemm_rows", "row": f"{dt}_{s[0]}x{s[1]}x{s[2]}", "A": host[s][0],
                           "B": host[s][1], "C0": host[s][2], "alpha": 1.0, "beta": 1.0, "rows": rrows,
                           "got": Cx[torch.from_numpy(rrows).to(dev)].cpu().numpy()})

    del devm, C
    torch.cuda.empty_cache()
    extras = None if args.no_extras else extra_rows(tg, inputs, checks)
    peaks_after = measured_peaks(tg)
    progress(f"extra rows done; probes after: {peaks_after}")
    # the probe is a ceiling only where it is at least the achieved rate
    mp = max(peaks_before["f32_mfma_tflops"], peaks_after["f32_mfma_tflops"]) if dt_dom == "f32" else \
        max(peaks_before["bf16_mfma_tflops"], peaks_after["bf16_mfma_tflops"]) / 3.0
    roofline["measured_peak"] = round(mp, 1)
    roofline["frac_of_measured_peak"] = round(dom["tflops"] / mp, 4)
    roofline["measured_peak_is_ceiling"] = bool(dom["tflops"] <= mp)

    base, errors = None, None
    if not args.no_cpu_baseline:
        base, errors = cpu_baseline(*host[sq], results, args.cpu_seconds)
        progress(f"oracle sample: {base['sample']}")
        errs = oracle_checks(checks)
        progress("oracle checks done")
        for key, e in errs.items():
            if key in per_path:
                per_path[key].update(e)
            elif key in small:
                small[key].update(e)
            elif extras is not None and key in extras:
                extras[key].update(e)
        for dt, e in errors.items():
            per_path[f"{dt}_8192x8192x8192"]["sampled_normwise_error"] = e

    x3 = per_path["x3_8192x8192x8192"]
    f32 = per_path["f32_8192x8192x8192"]
    out = {
        "metric": "GEMM TFLOP/s & % peak: FP32 vs split-BF16x3 MFMA at <=1e-5 rel err; "
                  "batched GEMM/s",
        "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16x3(f32 accumulate)",
        "data": "synthetic U[-1,1] float32, seeded",
        "config": {"workload": "gemm C=AB+C, 8192^3 and 4097x3001x2053, plain F32 and "
                               "split-bf16x3, one launch each per step", "alpha": 1.0,
                   "beta": 1.0, "layout": "row-major", "parallelism": "single GPU"},
        "paths": per_path,
        "x3_over_f32": round(x3["tflops"] / f32["tflops"], 3),
        "roofline": roofline,
        "measured_peaks": {"before_timed_steps": peaks_before, "after_extra_rows": peaks_after},
        "cpu_baseline": base,
        "sampled_normwise_error_8192": errors,
        "small_gemm_256": small,
        "extra_rows": extras,
    }
    if args.copy_calibration:
        # one plain device copy of 1 GiB: reads 2^30 bytes and writes 2^30 bytes of HBM
        src = torch.empty(2 ** 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
