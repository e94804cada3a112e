"""Benchmark of the randomized QLP hot path on one MI355X.

Default workload: mixed-precision ERQLP on A = U_256 diag(1/j) V_256^T +
1e-3 N(0,1) (32768 x 16384, stored FP32), k = 256, p = 16, q = 2 subspace
iterations, d = 2 inner QR steps, Omega generated inside the call and
rounded to bfloat16.  The 2q + 2 passes over A run as bfloat16 MFMA products
with FP32 accumulation, the panels are orthonormalised by FP32 CholeskyQR2
(FP64 Cholesky), and the CPQR, second factorisation and L stay in FP64.  One
step = one full rqlp_factor call with A already resident in HBM (the
FP32 -> bfloat16 encoding of A happens inside the call and is timed).

Prints ONE JSON line with the throughput (TFLOP/s under the fixed flop
model), the same call in FP64 on the same matrix and the speedup, the
L-value error against the FP64 CPU oracle (free pivots and the oracle re-run
on the GPU's pivots), a roofline figure for the dominant kernel (the 16-bit
projection product, timed with HIP events on the library's stream) and the
oracle's own throughput on the host cores, beside the same factorisation with
LAPACK's pivoted QR for the CPQR steps (the "best CPU" point).  ``--workload
erqlp_f64_20000x10000`` runs the FP64 ERQLP workload instead.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "fp16": 2500.0}   # dense TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0
METRIC = "RQLP TFLOP/s & factorizations/s, mixed vs FP64, at L-value rel err <=1e-3"
DEFAULT_WORKLOAD = "erqlp_bf16_32768x16384"
LVAL_BAR = 1e-3     # L-value relative error bar of the mixed path
PMC_PROFILES = {   # dominant kernel -> committed PMC summary (HBM bytes per launch)
    "f64": ("gemm_f64_tn_20000x10000_pmc.md", "gemm.hip"),
    "lp": ("gemm_lp_bf16_tn_32768x16384_pmc.md", "gemm_lp.hip"),
}


def flop_model(m, n, l, q):
    """Useful flops of one factorisation: the 2q+2 passes over A, the
    orthonormalisations (CholeskyQR2, 4 rows l^2 each) of the q+1 m x l
    panels and the q n x l panels, CPQR + second stage + assembly (fixed
    model)."""
    return (2.0 * (2 * q + 2) * m * n * l + 4.0 * l * l * ((q + 1) * m + q * n) + 6.0 * n * l * l
            + 2.0 * m * l * l)


def bound_ms(w):
    """Lower-bound time of one factorisation: the larger of (a) the flop
    model above with the 2q+2 passes over A at the MFMA peak of the product
    arithmetic and the rest (orthonormalisations, CPQR, second stage,
    assembly) at the MFMA peak of the arithmetic it runs in (FP64 for the
    FP64 path, FP32 otherwise: the FP64 small stages of the mixed paths are
    a lower-order term), and (b) the bytes of A over HBM bandwidth: 2q+2
    reads of A in the product's element size, plus, for the 16-bit paths,
    one read of the stored FP32 A and the write of its two tiled copies."""
    gemm = 2.0 * (2 * w.q + 2) * w.m * w.n * w.l
    rest = flop_model(w.m, w.n, w.l, w.q) - gemm
    prod = {"bf16x3": "bf16"}.get(w.precision, w.precision)
    tail = "f64" if w.precision == "f64" else "f32"
    t_flop = (gemm / PEAK[prod] + rest / PEAK[tail]) * 1e-9
    mn = float(w.m) * w.n
    if w.precision in ("f64", "f32"):
        nbytes = (2 * w.q + 2) * (8 if w.precision == "f64" else 4) * mn
    else:
        e = 4 if w.precision == "bf16x3" else 2       # bytes per element of the encoded A
        nbytes = 4 * mn + 2 * e * mn + (2 * w.q + 2) * e * mn
    return max(t_flop, nbytes / HBM_PEAK_GBS * 1e-6)


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 run on the mixed workload's matrix")
    ap.add_argument("--no-x3", action="store_true", help="skip the split-bfloat16 run on the headline matrix")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the short timings of the other workloads (FP64 ERQLP, block RQLP, backward)")
    ap.add_argument("--gaussian-input", action="store_true",
                    help="A = N(0,1) instead of the prescribed spectrum (hardware-counter runs only: "
                         "skips the QR-based generation)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one elementwise copy of 1 GiB (reference for the HBM byte counters)")
    return ap.parse_args()


def traffic_from_profile(name, src_file):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary, or None when it is absent or was taken on other kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    src = open(os.path.join(ROOT, "paper_1811_09334_amd", "csrc", src_file), "rb").read()
    txt = open(path).read()
    m_sha = re.search(r"source_sha256:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_sha or not m_b or m_sha.group(1) != hashlib.sha256(src).hexdigest():
        return None
    return float(m_b.group(1))


def timed(fn, steps, warmup):
    import torch
    out = None
    for _ in range(warmup):
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, out


def event_time(fn, stream, reps=10):
    """Average device time of fn() over reps calls, HIP events on ``stream``."""
    import torch
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def roofline_f64(rq, A, V, w, dev):
    import torch
    l = w.l
    nb = rq._lib.rqlp_gemm_workspace(w.m, w.n, l, 0)
    gw = torch.empty(nb, dtype=torch.uint8, device=dev)
    B = rq.empty_colmajor(l, w.n, torch.float64, dev)
    stream = torch.cuda.current_stream(dev)

    def proj():
        rq.check("rqlp_project", rq._lib.rqlp_project(A.data_ptr(), rq.ld(A), w.m, w.n, V.data_ptr(), rq.ld(V), l,
                                                      B.data_ptr(), rq.ld(B), 0, gw.data_ptr(), nb,
                                                      stream.cuda_stream))
    t = event_time(proj, stream)
    flops = 2.0 * w.m * w.n * l
    achieved = flops / t / 1e12
    name, src = PMC_PROFILES["f64"]
    print(f"# projection product: {t*1e3:.3f} ms, {achieved:.2f} TFLOP/s", file=sys.stderr, flush=True)
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f64"], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK["f64"], 4), "traffic": traffic_from_profile(name, src),
            "kernel": "gemm_skinny_kernel<double, A^T> + split-K reduce (B = V^T A)", "flops_per_launch": flops,
            "launch_ms": round(t * 1e3, 4)}


def roofline_lp(rq, A, V, w, dev):
    """The 16-bit projection product B = V^T A on the pre-encoded A: below the
    BF16 ridge (2 m n l flops over ~2 m n bytes = l flop/B < 312), so HBM
    bandwidth is the roof; algorithmic bytes = A once in 16 bits (twice for
    the split form) + V read in FP32 + B written in FP32."""
    import torch
    l = w.l
    E = rq.encode(A, w.precision)
    torch.cuda.synchronize()
    B = rq.empty_colmajor(l, w.n, torch.float32, dev)
    nb = rq._lib.rqlp_gemm_workspace(w.m, w.n, l, rq.PRECISIONS[w.precision])
    work = torch.empty(nb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    t = event_time(lambda: rq.project_encoded(E, V, B, work), stream)
    parts = 2 if w.precision == "bf16x3" else 1
    nbytes = 2.0 * parts * w.m * w.n + 4.0 * w.m * l + 4.0 * l * w.n
    flops = 2.0 * w.m * w.n * l
    gbs = nbytes / t / 1e9
    name, src = PMC_PROFILES["lp"]
    traffic = traffic_from_profile(name, src) if w.precision == "bf16" else None
    print(f"# 16-bit projection product: {t*1e3:.3f} ms, {gbs:.0f} GB/s, {flops/t/1e12:.1f} TFLOP/s",
          file=sys.stderr, flush=True)
    del E
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"gemm_lp_kernel<{w.precision}, A^T> + V encode + split-K reduce (B = V^T A)",
            "bytes_per_launch": nbytes, "launch_ms": round(t * 1e3, 4),
            "mfma_tflops": round(flops / t / 1e12, 2), "mfma_frac": round(flops / t / 1e12 / PEAK["bf16"], 4)}


def lval_vs(f, ref, w):
    """L-values j < k of factorisation f against ref, the FP64 GPU
    factorisation of the same matrix and Omega: the largest relative
    difference ("free": after the first-CPQR pivots diverge the two runs
    factor different column orders, and every L-value comes from the second
    factorisation of the whole R0^T, so this mixes pivot choice with
    rounding), the first step where the pivots differ (-1: none), and, for a
    matrix built from a prescribed spectrum, each run's largest relative
    distance max_j |sigma_j - |L_jj|| / sigma_j to it (the randomised
    approximation error plus that of the arithmetic)."""
    k = w.k
    lv, lr = f.lvals.cpu().numpy(), ref.lvals.cpu().numpy()
    d = np.flatnonzero(f.piv0.cpu().numpy() != ref.piv0.cpu().numpy())
    out = {"first_pivot_divergence_vs_f64": int(d[0]) if d.size else -1,
           "lval_rel_err_vs_f64": float(np.max(np.abs(lv[:k] - lr[:k]) / lr[:k]))}
    if w.kind == "svd":
        out["lval_err_vs_spectrum"] = spectrum_distance(f, w)
        out["lval_err_vs_spectrum_f64"] = spectrum_distance(ref, w)
    return out


def spectrum_distance(f, w):
    """max_{j < k} |sigma_j - |L_jj|| / sigma_j for a matrix built from a
    prescribed spectrum."""
    sig = w.spectrum_values()[: w.k]
    lv = f.lvals.cpu().numpy()[: w.k]
    return float(np.max(np.abs(sig - np.abs(lv)) / sig))


def lval_text(r):
    t = (f"free L-value rel err vs f64 {r['lval_rel_err_vs_f64']:.2e}, first pivot divergence at step "
         f"{r['first_pivot_divergence_vs_f64']}")
    if "lval_err_vs_spectrum_f64" in r:
        t += (f"; distance to the prescribed spectrum {r['lval_err_vs_spectrum']:.2e} "
              f"(f64: {r['lval_err_vs_spectrum_f64']:.2e})")
    return t


def other_workloads(rq, inputs, dev):
    """Short timings (3 steps after 1 warm-up) of the other workloads of the
    hot path, each on its own synthetic matrix: FP64 ERQLP (20000 x 10000),
    block RQLP in FP16 (65536 x 8192, b = 64) and the FP32 forward + backward
    of the differentiable workload (16384 x 4096).  Each record carries the
    lower-bound time of ``bound_ms`` and its fraction of the measured time,
    and an accuracy field: the distance of the L-values to the prescribed
    spectrum (FP64 path), or the L-values against one FP64 factorisation of
    the same matrix and Omega (the other paths)."""
    import torch
    out = {}
    for name in ("erqlp_f64_20000x10000", "brqlp_fp16_65536x8192", "drqlp_f32_16384x4096"):
        w = inputs.WORKLOADS[name]
        A = inputs.make_matrix_torch(w, dev)
        work = torch.empty(rq.workspace_size(w.m, w.n, w.k, w.p, w.q, w.d, w.b, w.precision), dtype=torch.uint8,
                           device=dev)
        ms, f = timed(lambda: rq.factor(A, w.k, w.p, q=w.q, d=w.d, b=w.b, precision=w.precision, seed=w.seed_omega,
                                        work=work), 3, 1)
        F = flop_model(w.m, w.n, w.l, w.q)
        lb = bound_ms(w)
        rec = {"ms_per_step": round(ms, 3), "tflops": round(F / (ms * 1e-3) / 1e12, 3), "precision": w.precision,
               "m": w.m, "n": w.n, "k": w.k, "p": w.p, "q": w.q, "d": w.d, "b": w.b, "info": int(f.info.item()),
               "bound_ms": round(lb, 3), "bound_frac": round(lb / ms, 4)}
        if w.precision == "f64" and w.kind == "svd":
            rec["lval_err_vs_spectrum"] = spectrum_distance(f, w)
        elif w.precision != "f64":
            # accuracy of the reduced-precision arithmetic: one FP64 factorisation of the same matrix and Omega
            del work
            A64 = rq.empty_colmajor(w.m, w.n, torch.float64, dev)
            A64.copy_(A)
            w64 = torch.empty(rq.workspace_size(w.m, w.n, w.k, w.p, w.q, w.d, w.b, "f64"), dtype=torch.uint8,
                              device=dev)
            f64r = rq.factor(A64, w.k, w.p, q=w.q, d=w.d, b=w.b, precision="f64", seed=w.seed_omega, work=w64)
            rec.update(lval_vs(f, f64r, w))
            del A64, w64, f64r
            work = None
            torch.cuda.empty_cache()
        if name.startswith("drqlp"):
            dT = torch.zeros(w.l, w.l, dtype=torch.float64, device=dev)
            dT.diagonal()[: w.k] = torch.as_tensor(inputs.uniform_weights(w.k, 3000), device=dev)
            bw = torch.empty(rq._lib.rqlp_backward_workspace_size(w.m, w.n, w.k, w.p, w.q, w.d, w.b,
                                                                  rq.PRECISIONS[w.precision]),
                             dtype=torch.uint8, device=dev)
            msb, _ = timed(lambda: rq.backward(A, w.k, w.p, f.piv0, f.piv1, dT, q=w.q, precision=w.precision,
                                               seed=w.seed_omega, work=bw), 3, 1)
            rec["backward_ms"] = round(msb, 3)
            del bw
        out[name] = rec
        acc = (lval_text(rec) if "lval_rel_err_vs_f64" in rec else
               f"distance to the prescribed spectrum {rec['lval_err_vs_spectrum']:.2e}"
               if "lval_err_vs_spectrum" in rec else "")
        print(f"# {name}: {ms:.3f} ms/step ({lb / ms:.0%} of the {lb:.2f} ms bound)"
              + (f", backward {rec['backward_ms']:.3f} ms" if "backward_ms" in rec else "")
              + (f"; {acc}" if acc else ""), file=sys.stderr, flush=True)
        del A, work, f
        torch.cuda.empty_cache()
    return out


def paper_tables(rq, inputs, dev):
    """The Section 5 replica workloads (Example 5.1: pds, eds at m = n = 2000,
    4000, 6000, k = 120, p = 5, FP64): GPU time of RQLP and ERQLP (d = 2, 4)
    and of the deterministic truncated pivoted QLP (kt = l = 125, rqlp_qlp),
    and err = max_{j <= k} |sigma_j - |L_jj|| against the prescribed spectrum,
    next to the paper's MATLAB times on an i5-7500 (Tables 1-2; its QLP column
    is the full, not truncated, deterministic QLP).  Context only: the paper's
    random orthogonal factors are not specified, so errors compare in order,
    not in value."""
    import torch
    paper = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_tables_1_2.txt")):
        t = line.split()
        if t and not line.startswith("#"):
            paper[(t[0], int(t[1]))] = dict(zip(["qlp_t", "qlp", "rqlp_t", "rqlp", "e2_t", "e2", "e4_t", "e4"],
                                                map(float, t[2:])))
    rows = []
    for ex in ("pds", "eds"):
        for n in inputs.PAPER_EXAMPLE_SIZES:
            w = inputs.paper_example(ex, n)
            A = inputs.make_matrix_torch(w, dev)
            sig = w.spectrum_values()
            rec = {"example": ex, "n": n}
            for d, key in ((0, "rqlp"), (2, "erqlp2"), (4, "erqlp4")):
                work = torch.empty(rq.workspace_size(n, n, w.k, w.p, 0, d, 0, "f64"), dtype=torch.uint8, device=dev)
                ms, f = timed(lambda: rq.factor(A, w.k, w.p, q=0, d=d, seed=w.seed_omega, work=work), 5, 2)
                lv = f.lvals.cpu().numpy()
                rec[key + "_ms"] = round(ms, 3)
                rec[key + "_err"] = float(np.max(np.abs(sig[: w.k] - np.abs(lv[: w.k]))))
            qwork = torch.empty(rq._lib.rqlp_qlp_workspace_size(n, n, w.l), dtype=torch.uint8, device=dev)
            ms, f = timed(lambda: rq.pivoted_qlp(A, w.l, work=qwork), 2, 1)
            lv = f.lvals.cpu().numpy()
            rec["qlp_truncated_ms"] = round(ms, 3)
            rec["qlp_truncated_err"] = float(np.max(np.abs(sig[: w.k] - np.abs(lv[: w.k]))))
            pp = paper.get((ex, n), {})
            rec["paper_i5_7500_s"] = {"qlp": pp.get("qlp_t"), "rqlp": pp.get("rqlp_t"), "erqlp2": pp.get("e2_t"),
                                      "erqlp4": pp.get("e4_t")}
            rec["paper_err"] = {"qlp": pp.get("qlp"), "rqlp": pp.get("rqlp"), "erqlp2": pp.get("e2"),
                                "erqlp4": pp.get("e4")}
            rows.append(rec)
            print(f"# {ex} n={n}: RQLP {rec['rqlp_ms']:.2f} ms (err {rec['rqlp_err']:.2e}), ERQLP(4) "
                  f"{rec['erqlp4_ms']:.2f} ms (err {rec['erqlp4_err']:.2e}), QLP(kt=125) {rec['qlp_truncated_ms']:.2f}"
                  f" ms (err {rec['qlp_truncated_err']:.2e}); paper RQLP {pp.get('rqlp_t')} s", file=sys.stderr,
                  flush=True)
            del A, work, qwork, f
            torch.cuda.empty_cache()
    return rows


def autorank_leg(rq, inputs, dev):
    """Auto-rank RQLP (Section 6) on the FP64 ERQLP workload's matrix
    (20000 x 10000): lmax = 256, b = 64, q = 1, eps = 1e-4 ||A||_F^2."""
    import torch
    w = inputs.WORKLOADS["erqlp_f64_20000x10000"]
    A = inputs.make_matrix_torch(w, dev)
    eps = 1e-4 * float((A * A).sum().item())
    lmax, b = 256, 64
    work = torch.empty(rq._lib.rqlp_autorank_workspace_size(w.m, w.n, lmax, b, 1, 0), dtype=torch.uint8, device=dev)
    ms, out = timed(lambda: rq.factor_autorank(A, lmax, b, eps, q=1, seed=w.seed_omega, work=work), 3, 1)
    f, rank, err2 = out
    print(f"# autorank 20000x10000: rank {rank}, ||E||^2 / ||A||^2 {err2 * 1e-4 / eps:.2e}, {ms:.3f} ms",
          file=sys.stderr, flush=True)
    del A, work, f
    torch.cuda.empty_cache()
    return {"m": w.m, "n": w.n, "lmax": lmax, "b": b, "q": 1, "eps_rel": 1e-4, "rank": rank,
            "err2_rel": err2 * 1e-4 / eps, "ms_per_call": round(ms, 3)}


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1811_09334_amd as rq
    from paper_1811_09334_amd import inputs

    rq.load()
    dev = torch.device("cuda:0")
    w = inputs.WORKLOADS[args.workload]
    mixed = w.precision in ("bf16", "fp16", "bf16x3")
    l = w.l
    t0 = time.time()
    if args.gaussian_input:
        g = torch.Generator(device=dev)
        g.manual_seed(w.seed_a)
        dt = torch.float64 if w.storage == "f64" else torch.float32
        A = torch.randn(w.n, w.m, generator=g, dtype=dt, device=dev).t()
    else:
        A = inputs.make_matrix_torch(w, dev)       # column-major (m, n) in HBM
    torch.cuda.synchronize()
    print(f"# generated A {w.m}x{w.n} ({A.dtype}) in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)     # 1 GiB read, 1 GiB written
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    seed = w.seed_omega
    work = torch.empty(rq.workspace_size(w.m, w.n, w.k, w.p, w.q, w.d, w.b, w.precision),
                       dtype=torch.uint8, device=dev)
    ms, f = timed(lambda: rq.factor(A, w.k, w.p, q=w.q, d=w.d, b=w.b, precision=w.precision, seed=seed,
                                    work=work), args.steps, args.warmup)
    info = int(f.info.item())
    F = flop_model(w.m, w.n, l, w.q)
    tflops = F / (ms * 1e-3) / 1e12
    print(f"# {w.precision}: {ms:.3f} ms/step, {tflops:.2f} TFLOP/s, info={info:#x}", file=sys.stderr, flush=True)
    backward = None
    if w.name.startswith("drqlp"):
        # the differentiable workload: the adjoint of the same call, loss sum_j w_j L_jj
        dT = torch.zeros(l, l, dtype=torch.float64, device=dev)
        dT.diagonal()[: w.k] = torch.as_tensor(inputs.uniform_weights(w.k, 3000), device=dev)
        bw = torch.empty(rq._lib.rqlp_backward_workspace_size(w.m, w.n, w.k, w.p, w.q, w.d, w.b,
                                                              rq.PRECISIONS[w.precision]), dtype=torch.uint8,
                         device=dev)
        msb, _ = timed(lambda: rq.backward(A, w.k, w.p, f.piv0, f.piv1, dT, q=w.q, precision=w.precision,
                                           seed=seed, work=bw), args.steps, args.warmup)
        backward = {"ms_per_step": round(msb, 4)}
        print(f"# backward: {msb:.3f} ms/step", file=sys.stderr, flush=True)

    # ---- the same call in FP64 on the same matrix (the "mixed vs FP64" ratio) ----
    fp64 = None
    if mixed and not args.no_fp64:
        A64 = rq.empty_colmajor(w.m, w.n, torch.float64, dev)
        A64.copy_(A)
        w64 = torch.empty(rq.workspace_size(w.m, w.n, w.k, w.p, w.q, w.d, w.b, "f64"), dtype=torch.uint8,
                          device=dev)
        steps64 = max(3, args.steps // 4)
        ms64, f64r = timed(lambda: rq.factor(A64, w.k, w.p, q=w.q, d=w.d, b=w.b, precision="f64", seed=seed,
                                             work=w64), steps64, 1)
        fp64 = {"ms_per_step": round(ms64, 4), "tflops": round(F / (ms64 * 1e-3) / 1e12, 4), "steps": steps64,
                "info": int(f64r.info.item()), **lval_vs(f, f64r, w)}
        print(f"# f64 on the same matrix: {ms64:.3f} ms/step ({ms64 / ms:.2f}x the {w.precision} time); "
              f"{lval_text(fp64)}", file=sys.stderr, flush=True)
        del A64, w64, f64r
        torch.cuda.empty_cache()

    # ---- the split-bfloat16 form on the same matrix (free-pivot accuracy leg) ----
    x3 = None
    x3_fact = None
    if w.precision == "bf16" and not args.no_x3:
        wx3 = torch.empty(rq.workspace_size(w.m, w.n, w.k, w.p, w.q, w.d, w.b, "bf16x3"), dtype=torch.uint8,
                          device=dev)
        steps_x3 = max(3, args.steps // 4)
        msx3, x3_fact = timed(lambda: rq.factor(A, w.k, w.p, q=w.q, d=w.d, b=w.b, precision="bf16x3", seed=seed,
                                                work=wx3), steps_x3, 1)
        x3 = {"ms_per_step": round(msx3, 4), "tflops": round(F / (msx3 * 1e-3) / 1e12, 4), "steps": steps_x3,
              "info": int(x3_fact.info.item())}
        if fp64:
            x3["speedup_vs_fp64"] = round(fp64["ms_per_step"] / msx3, 3)
        print(f"# bf16x3 on the same matrix: {msx3:.3f} ms/step", file=sys.stderr, flush=True)
        del wx3
        torch.cuda.empty_cache()

    # ---- roofline of the dominant kernel: the projection product B = V^T A ----
    roof = None
    if not args.no_roofline:
        V = rq.empty_colmajor(w.m, l, f.Q.dtype, dev)
        V.copy_(f.Q)
        roof = roofline_lp(rq, A, V, w, dev) if mixed else roofline_f64(rq, A, V, w, dev)
        del V

    others = None
    tables = None
    autorank = None
    if not args.no_others and args.workload == DEFAULT_WORKLOAD:
        del work
        torch.cuda.empty_cache()
        others = other_workloads(rq, inputs, dev)
        tables = paper_tables(rq, inputs, dev)
        autorank = autorank_leg(rq, inputs, dev)

    # ---- CPU baseline: the FP64 oracle on the host cores, same A and Omega ----
    cpu = None
    cpu_best = None
    acc = {}
    if not args.no_cpu_baseline:
        from oracle.rqlp import brqlp as oracle_brqlp
        from oracle.rqlp import rqlp as oracle_rqlp

        def run_oracle(A_, Om_, piv0=None, piv1=None):
            if w.b:
                return oracle_brqlp(A_, Om_, w.k, w.p, w.b, q=w.q, piv0=piv0, piv1=piv1)
            return oracle_rqlp(A_, Om_, w.k, w.p, q=w.q, d=w.d, piv0=piv0, piv1=piv1)
        Om = rq.generate_omega(w.n, l, seed, w.precision, dev)
        torch.cuda.synchronize()
        A_h = np.asfortranarray(A.double().cpu().numpy()) if A.dtype != torch.float64 else \
            np.asfortranarray(A.cpu().numpy())
        Om_h = np.asfortranarray(Om.double().cpu().numpy())
        try:
            cores = len(os.sched_getaffinity(0))
        except AttributeError:
            cores = os.cpu_count()
        threads = int(os.environ.get("OMP_NUM_THREADS", cores))
        t0 = time.perf_counter()
        ref = run_oracle(A_h, Om_h)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": round(F / t_cpu / 1e12, 5), "unit": "TFLOP/s", "cores": min(threads, cores),
               "kind": "oracle", "sample": f"one full factorisation of the same {w.m}x{w.n} matrix in FP64 "
                                           f"({t_cpu:.1f} s)"}
        if w.b == 0:
            # the "best CPU" point: the same factorisation with LAPACK's pivoted
            # QR (dgeqp3) for the CPQR steps, all of it in the host's BLAS/LAPACK
            from oracle.lapack_rqlp import rqlp_lapack
            t0 = time.perf_counter()
            _, T_best, _, piv_best, _ = rqlp_lapack(A_h, Om_h, w.k, w.p, q=w.q, d=w.d)
            t_best = time.perf_counter() - t0
            lv_best = np.abs(np.diag(T_best))[: w.k]
            cpu_best = {"value": round(F / t_best / 1e12, 5), "unit": "TFLOP/s", "cores": min(threads, cores),
                        "kind": "lapack_dgeqp3",
                        "sample": f"one full factorisation of the same {w.m}x{w.n} matrix in FP64 "
                                  f"({t_best:.1f} s)",
                        "lval_rel_diff_vs_oracle": float(np.max(np.abs(lv_best - ref.lvals[: w.k])
                                                                / ref.lvals[: w.k])),
                        "same_pivots_as_oracle": bool(np.array_equal(piv_best, ref.piv0))}
            print(f"# LAPACK-backed CPU point {t_best:.1f} s", file=sys.stderr, flush=True)
        lv = f.lvals.cpu().numpy()
        piv0 = f.piv0.cpu().numpy()
        acc["lval_rel_err_free"] = float(np.max(np.abs(lv[: w.k] - ref.lvals[: w.k]) / ref.lvals[: w.k]))
        d = np.flatnonzero(piv0 != ref.piv0)
        acc["first_pivot_divergence"] = int(d[0]) if d.size else -1
        print(f"# oracle {t_cpu:.1f} s; free L-value rel err {acc['lval_rel_err_free']:.2e}, first pivot "
              f"divergence {acc['first_pivot_divergence']}", file=sys.stderr, flush=True)
        if mixed:
            piv1 = f.piv1.cpu().numpy() if w.d == 0 else None
            fr = run_oracle(A_h, Om_h, piv0=piv0, piv1=piv1)
            acc["lval_rel_err_frozen"] = float(np.max(np.abs(lv[: w.k] - fr.lvals[: w.k]) / fr.lvals[: w.k]))
            print(f"# frozen-pivot L-value rel err {acc['lval_rel_err_frozen']:.2e}", file=sys.stderr, flush=True)
            # the value above is reported under the frozen-pivot reading of the
            # accuracy bar (the oracle re-run on the GPU's pivots); both readings
            # are stated against the 1e-3 bar
            acc["lval_gate"] = "frozen_pivots"
            acc["lval_gate_frozen_pass"] = bool(acc["lval_rel_err_frozen"] <= LVAL_BAR)
            acc["lval_gate_free_pass"] = bool(acc["lval_rel_err_free"] <= LVAL_BAR)
        if x3 is not None:
            lv3 = x3_fact.lvals.cpu().numpy()
            p3 = x3_fact.piv0.cpu().numpy()
            x3["lval_rel_err_free"] = float(np.max(np.abs(lv3[: w.k] - ref.lvals[: w.k]) / ref.lvals[: w.k]))
            d3 = np.flatnonzero(p3 != ref.piv0)
            x3["first_pivot_divergence"] = int(d3[0]) if d3.size else -1
            if d3.size:
                fr3 = run_oracle(A_h, Om_h, piv0=p3,
                                  piv1=x3_fact.piv1.cpu().numpy() if w.d == 0 else None)
                x3["lval_rel_err_frozen"] = float(np.max(np.abs(lv3[: w.k] - fr3.lvals[: w.k]) / fr3.lvals[: w.k]))
            else:
                x3["lval_rel_err_frozen"] = x3["lval_rel_err_free"]
            x3["lval_gate_free_pass"] = bool(x3["lval_rel_err_free"] <= LVAL_BAR)
            print(f"# bf16x3: free L-value rel err {x3['lval_rel_err_free']:.2e}, first pivot divergence "
                  f"{x3['first_pivot_divergence']}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(tflops, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.precision,
        "data": "synthetic",
        "config": {"workload": w.name, "m": w.m, "n": w.n, "k": w.k, "p": w.p, "q": w.q, "d": w.d, "b": w.b,
                   "precision": w.precision,
                   "arithmetic": ("16-bit MFMA products with FP32 accumulation, FP32 CholeskyQR2, FP64 CPQR / "
                                  "second factorisation / L") if mixed else
                                 ("FP32 products and CholeskyQR, FP64 CPQR / second factorisation / L"
                                  if w.precision == "f32" else "FP64 throughout"),
                   "input": "gaussian" if args.gaussian_input else "prescribed spectrum"},
        "factorizations_per_s": round(1e3 / ms, 3),
        "flops_per_step": F,
        "bound_ms": round(bound_ms(w), 4),
        "bound_frac": round(bound_ms(w) / ms, 4),
        "info": info,
        "fp64_same_matrix": fp64,
        "speedup_vs_fp64": round(fp64["ms_per_step"] / ms, 3) if fp64 else None,
        "bf16x3_same_matrix": x3,
        "backward": backward,
        **acc,
        "other_workloads": others,
        "paper_tables_1_2": tables,
        "autorank": autorank,
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_best": cpu_best,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
