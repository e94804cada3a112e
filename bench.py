"""Benchmark of the randomized QLP hot path on one MI355X.

Default workload: ERQLP in FP64, A = U diag(s) V^T (20000 x 10000,
s_j = 10^(-4(j-1)/199) for j <= 200, 1e-6 beyond), k = 200, p = 10,
q = 1 subspace iteration, d = 2 inner QR steps, Omega generated inside the
call.  One step = one full rqlp_factor call (test matrix, sketch, subspace
iteration, orthonormalisations, projection, both factorisations, assembly)
with A already resident in HBM.

Prints ONE JSON line (rank 0) with the throughput, a roofline figure for
the dominant kernel (the FP64 MFMA skinny product, timed with HIP events on
the library's stream) and the FP64 CPU oracle timed on the host cores.
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


def flop_model(m, n, l, q):
    """Useful flops of one factorisation: the 2q+2 passes over A, the 2q+1
    orthonormalisations, CPQR + second stage + assembly (fixed model)."""
    return 2.0 * (2 * q + 2) * m * n * l + (2 * q + 1) * 4.0 * m * l * l + 6.0 * n * l * l + 2.0 * m * l * l


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="erqlp_f64_20000x10000")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--gaussian-input", action="store_true",
                    help="A = N(0,1) instead of the prescribed spectrum (hardware-counter runs only: "
                         "skips the QR-based generation)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one elementwise copy of 1 GiB (reference for the HBM byte counters)")
    return ap.parse_args()


def traffic_from_profile(src_sha):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary, or None when it is absent or was taken on other kernel source."""
    path = os.path.join(ROOT, "profiles", "gemm_f64_tn_20000x10000_pmc.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"source_sha256:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_sha or not m_b or m_sha.group(1) != src_sha:
        return None
    return float(m_b.group(1))


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1811_09334_amd as rq
    from paper_1811_09334_amd import inputs

    rq.load()
    dev = torch.device("cuda:0")
    w = inputs.WORKLOADS[args.workload]
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
    gen_s = time.time() - t0
    print(f"# generated A {w.m}x{w.n} in {gen_s:.1f} s", file=sys.stderr, flush=True)

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)     # 1 GiB read, 1 GiB written
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    work = torch.empty(rq.workspace_size(w.m, w.n, w.k, w.p, w.q, w.d, w.b, w.precision),
                       dtype=torch.uint8, device=dev)
    seed = w.seed_omega

    def step():
        return rq.factor(A, w.k, w.p, q=w.q, d=w.d, b=w.b, precision=w.precision, seed=seed, work=work)

    for _ in range(args.warmup):
        f = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    info = int(f.info.item())
    F = flop_model(w.m, w.n, l, w.q)
    tflops = F / (ms * 1e-3) / 1e12
    print(f"# {ms:.3f} ms/step, {tflops:.2f} TFLOP/s, info={info:#x}", file=sys.stderr, flush=True)

    # ---- roofline of the dominant kernel: the FP64 MFMA product B^T = A^T V ----
    roof = None
    if not args.no_roofline:
        V = rq.empty_colmajor(w.m, l, torch.float64, dev)
        V.copy_(f.Q)
        nb = rq._lib.rqlp_gemm_workspace(w.m, w.n, l, 0)
        gw = torch.empty(nb, dtype=torch.uint8, device=dev)
        B = rq.empty_colmajor(l, w.n, torch.float64, dev)
        stream = torch.cuda.current_stream(dev)
        reps = 10

        def proj():
            rq.check("rqlp_project", rq._lib.rqlp_project(A.data_ptr(), rq.ld(A), w.m, w.n, V.data_ptr(),
                                                          rq.ld(V), l, B.data_ptr(), rq.ld(B), 0,
                                                          gw.data_ptr(), nb, stream.cuda_stream))
        proj()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            proj()
        e1.record(stream)
        torch.cuda.synchronize()
        t_launch = e0.elapsed_time(e1) * 1e-3 / reps
        flops = 2.0 * w.m * w.n * l
        achieved = flops / t_launch / 1e12
        src = open(os.path.join(ROOT, "paper_1811_09334_amd", "csrc", "gemm.hip"), "rb").read()
        traffic = traffic_from_profile(hashlib.sha256(src).hexdigest())
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f64"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK["f64"], 4), "traffic": traffic,
                "kernel": "gemm_skinny_kernel<double, A^T>", "flops_per_launch": flops,
                "launch_ms": round(t_launch * 1e3, 4)}
        print(f"# projection product: {t_launch*1e3:.3f} ms, {achieved:.2f} TFLOP/s", file=sys.stderr, flush=True)

    # ---- CPU baseline: the FP64 oracle on the host cores, same A and Omega ----
    cpu = None
    lval_err = None
    if not args.no_cpu_baseline:
        from oracle.rqlp import rqlp as oracle_rqlp
        Om = rq.generate_omega(w.n, l, seed, "f64", dev)
        torch.cuda.synchronize()
        A_h = np.asfortranarray(A.cpu().numpy())
        Om_h = np.asfortranarray(Om.cpu().numpy())
        try:
            cores = len(os.sched_getaffinity(0))
        except AttributeError:
            cores = os.cpu_count()
        threads = int(os.environ.get("OMP_NUM_THREADS", cores))
        t0 = time.perf_counter()
        ref = oracle_rqlp(A_h, Om_h, w.k, w.p, q=w.q, d=w.d)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": round(F / t_cpu / 1e12, 5), "unit": "TFLOP/s", "cores": min(threads, cores),
               "kind": "oracle", "sample": f"one full factorisation of the same {w.m}x{w.n} matrix "
                                           f"({t_cpu:.1f} s)"}
        lv = f.lvals.cpu().numpy()
        lval_err = float(np.max(np.abs(lv[: w.k] - ref.lvals[: w.k]) / ref.lvals[: w.k]))
        print(f"# oracle {t_cpu:.1f} s; GPU vs oracle max L-value rel err {lval_err:.2e}", file=sys.stderr,
              flush=True)

    out = {
        "metric": "RQLP TFLOP/s & factorizations/s, mixed vs FP64, at L-value rel err <=1e-3",
        "value": round(tflops, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "m": w.m, "n": w.n, "k": w.k, "p": w.p, "q": w.q, "d": w.d,
                   "precision": w.precision,
                   "input": "gaussian" if args.gaussian_input else "prescribed spectrum"},
        "factorizations_per_s": round(1e3 / ms, 3),
        "flops_per_step": F,
        "info": info,
        "lval_rel_err_vs_oracle": lval_err,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
