"""GPU checks of the mixed-precision path (bfloat16 / IEEE half / split
bfloat16 MFMA products with FP32 accumulation, FP32 CholeskyQR2, FP64 CPQR
and second stage) through the C ABI.

Products: against an FP64 product of exactly the 16-bit operands the kernels
are fed (host emulation of the encodings), within the worst-case FP32
accumulation bound gamma_K |a| |x|.

Whole factorisation: the mixed path rounds A and the bases, so its pivots may
legitimately differ from the FP64 oracle's where residual norms are close.
The gate is the frozen-pivot comparison: the oracle re-run in FP64 on the same
A and Omega with the GPU's pivots (any pivot order gives a valid QLP), L-value
relative error <= 1e-3 for j <= k.  The free comparison (oracle's own pivots)
is reported, and the split-bfloat16 form must pass it too."""
import numpy as np
import pytest

from oracle.rqlp import rqlp as oracle_rqlp
from paper_1811_09334_amd import inputs

from _helpers import first_difference, to_dev, to_np
from _lowprec import project_reference, sketch_reference

pytestmark = pytest.mark.gpu

LVAL_GATE = 1e-3
KINDS = ["bf16", "fp16", "bf16x3"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("m,n,c", [(1000, 500, 25), (777, 333, 47), (4096, 2048, 272), (64, 16, 16),
                                   (130, 70, 3), (1500, 3000, 120), (5000, 700, 288), (300, 200, 300),
                                   # the block workload's panel width l = 1056 (four column tiles)
                                   (2048, 4096, 1056)])
def test_lowprec_products_match_encoded_reference(gpu, kind, m, n, c):
    import torch
    rng = np.random.default_rng(m * 3 + n + c)
    # column scales spread over a few binades (exercises the FP16 per-column exponents)
    A = (rng.standard_normal((m, n)) * np.exp2(rng.integers(-14, -6, n))[None, :]).astype(np.float32)
    X = rng.standard_normal((n, c)).astype(np.float32)
    V = (rng.standard_normal((m, c)) / np.sqrt(m)).astype(np.float32)
    Y = to_np(gpu.sketch(to_dev(A, torch.float32), to_dev(X, torch.float32), precision=kind)).astype(np.float64)
    ref, bound = sketch_reference(A, X, kind)
    assert Y.shape == (m, c)
    excess = np.abs(Y - ref) - bound
    assert excess.max() <= 0, f"sketch off by {np.abs(Y - ref).max():.3e} (bound {bound.max():.3e})"
    B = to_np(gpu.project(to_dev(A, torch.float32), to_dev(V, torch.float32), precision=kind)).astype(np.float64)
    refB, boundB = project_reference(A, V, kind)
    assert B.shape == (c, n)
    excess = np.abs(B - refB) - boundB
    assert excess.max() <= 0, f"projection off by {np.abs(B - refB).max():.3e} (bound {boundB.max():.3e})"


def _mixed_factor(gpu, A32, Om, k, p, q, d, kind, lda_pad=0):
    import torch
    m, n = A32.shape
    Ad = to_dev(A32, torch.float32)
    if lda_pad:
        big = torch.zeros((n, m + lda_pad), dtype=torch.float32, device=Ad.device)
        big[:, :m] = Ad.t()
        Ad = big.t()[:m]
    f = gpu.factor(Ad, k, p, q=q, d=d, precision=kind, Omega=to_dev(Om, torch.float32))
    return f, {key: to_np(getattr(f, key)) for key in ("Q", "T", "P", "piv0", "piv1", "lvals", "info")}


def _check_mixed(gpu, A32, Om, k, p, q, d, kind, free_gate=None, lda_pad=0, allowed_info=0):
    l = k + p
    f, g = _mixed_factor(gpu, A32, Om, k, p, q, d, kind, lda_pad)
    A = A32.astype(np.float64)
    Q, T, P = g["Q"].astype(np.float64), g["T"], g["P"].astype(np.float64)
    lv, piv0, piv1 = g["lvals"], g["piv0"], g["piv1"]
    assert int(g["info"][0]) & ~allowed_info == 0, f"info flags {int(g['info'][0]):#x}"
    assert np.array_equal(np.diag(T), lv) and np.all(lv >= 0)
    assert len(set(piv0.tolist())) == l and piv0.min() >= 0 and piv0.max() < A.shape[1]
    frozen = oracle_rqlp(A, Om, k, p, q=q, d=d, piv0=piv0, piv1=piv1 if d == 0 else None)
    rel = np.abs(lv[:k] - frozen.lvals[:k]) / frozen.lvals[:k]
    assert rel.max() <= LVAL_GATE, f"{kind}: frozen-pivot L-value rel err {rel.max():.3e} at j={rel.argmax()}"
    free = oracle_rqlp(A, Om, k, p, q=q, d=d)
    rel_free = np.abs(lv[:k] - free.lvals[:k]) / free.lvals[:k]
    div = first_difference(piv0, free.piv0)
    print(f"[{kind} {A.shape} k={k} q={q} d={d}] frozen {rel.max():.2e}  free {rel_free.max():.2e}  "
          f"first pivot divergence {div}")
    if free_gate is not None:
        assert rel_free.max() <= free_gate, f"{kind}: free L-value rel err {rel_free.max():.3e}"
    assert f.uplo == frozen.uplo
    tri = np.triu(T, 1) if f.uplo == "L" else np.tril(T, -1)
    assert np.all(tri == 0.0)
    assert np.abs(Q.T @ Q - np.eye(l)).max() < 2e-5
    assert np.abs(P.T @ P - np.eye(l)).max() < 2e-5
    nA = np.linalg.norm(A)
    err_g = np.linalg.norm(A - Q @ T @ P.T) / nA
    err_o = np.linalg.norm(A - frozen.Q @ frozen.T @ frozen.P.T) / nA
    assert abs(err_g - err_o) <= 1e-2 * err_o + 1e-5, f"residual {err_g:.4e} vs oracle {err_o:.4e}"
    return rel.max(), rel_free.max()


def _c3_like(m, n, rank, k, p, seed=1002):
    """The mixed workload's recipe at a reduced size: rank-r signal s_j = 1/j
    plus 1e-3 N(0,1) noise, stored FP32; Omega rounded to bfloat16."""
    A = inputs.lowrank_plus_noise(m, n, inputs.spectrum_poly(rank, 1.0), 1e-3, seed).astype(np.float32)
    Om = inputs.round_to_bf16(inputs.gaussian(n, k + p, seed + 1000))
    return A, Om


@pytest.mark.parametrize("kind", KINDS)
def test_mixed_erqlp_scaled_workload(gpu, kind):
    """Mixed ERQLP (q = 2, d = 2) on the low-rank-plus-noise recipe at 4096 x 2048."""
    A, Om = _c3_like(4096, 2048, 64, 64, 8)
    if kind == "fp16":
        Om = inputs.round_to_fp16(Om)
    _check_mixed(gpu, A, Om, 64, 8, 2, 2, kind, free_gate=LVAL_GATE if kind == "bf16x3" else None)


@pytest.mark.parametrize("kind", ["bf16", "bf16x3"])
@pytest.mark.parametrize("m,n,k,p,q,d,pad", [
    (1001, 517, 20, 5, 0, 0, 0),     # ragged tiles, plain RQLP (pivoted second CPQR)
    (1000, 500, 20, 5, 1, 1, 3),     # odd d (lower T), padded leading dimension
    (2048, 1024, 100, 12, 2, 3, 0),
    (600, 600, 30, 10, 1, 0, 0),     # square
])
def test_mixed_shapes(gpu, kind, m, n, k, p, q, d, pad):
    rng = np.random.default_rng(m + n + k)
    s = np.logspace(0, -3, n)
    A = inputs.svd_matrix(m, n, s, m * 7 + n).astype(np.float32)
    Om = inputs.round_to_bf16(rng.standard_normal((n, k + p)))
    _check_mixed(gpu, A, Om, k, p, q, d, kind, lda_pad=pad)


def test_mixed_full_rank_sketch_shifted_cholqr(gpu):
    """l = n (square Gaussian sketch of a matrix with a three-decade spectrum):
    the FP32 Gram of Y (condition ~1e6) breaks down, the shifted retry flags
    0x1 and the conditional third CholeskyQR pass restores orthonormality.
    Run in the split-bfloat16 form: a single bfloat16 (8-bit significand)
    cannot resolve L-values three decades below the largest to 1e-3."""
    m, n, k, p = 700, 300, 288, 12
    rng = np.random.default_rng(m + n + k)
    A = inputs.svd_matrix(m, n, np.logspace(0, -3, n), m * 7 + n).astype(np.float32)
    Om = inputs.round_to_bf16(rng.standard_normal((n, k + p)))
    _check_mixed(gpu, A, Om, k, p, 1, 2, "bf16x3", allowed_info=0x1)


def test_mixed_library_omega_and_determinism(gpu):
    """Omega drawn inside the call (rounded to bfloat16) equals the exported
    generator's, and two calls give bitwise-identical results."""
    import torch
    A, _ = _c3_like(2000, 1000, 32, 32, 8)
    Ad = to_dev(A, torch.float32)
    f1 = gpu.factor(Ad, 32, 8, q=2, d=2, precision="bf16", seed=2002)
    Om = gpu.generate_omega(1000, 40, 2002, "bf16")
    f2 = gpu.factor(Ad, 32, 8, q=2, d=2, precision="bf16", Omega=Om)
    f3 = gpu.factor(Ad, 32, 8, q=2, d=2, precision="bf16", seed=2002)
    for a, b in [(f1, f2), (f1, f3)]:
        assert np.array_equal(to_np(a.T), to_np(b.T))
        assert np.array_equal(to_np(a.Q), to_np(b.Q))
        assert np.array_equal(to_np(a.P), to_np(b.P))
        assert np.array_equal(to_np(a.piv0), to_np(b.piv0))


@pytest.mark.parametrize("kind", KINDS)
def test_encoding_layout_and_encoded_products(gpu, kind):
    """rqlp_encode writes exactly the documented fragment tiles of the rounded
    A (both forms, zero padding, ragged sizes), and the products on the
    encoded A give bitwise the same results as rqlp_project / rqlp_sketch."""
    import torch
    from _lowprec import bits16, column_exponents, untile
    rng = np.random.default_rng(11)
    m, n, c = 3001, 1003, 136
    A = (rng.standard_normal((m, n)) * 1e-3).astype(np.float32)
    V = rng.standard_normal((m, c)).astype(np.float32)
    X = rng.standard_normal((n, c)).astype(np.float32)
    Ad, Vd, Xd = to_dev(A, torch.float32), to_dev(V, torch.float32), to_dev(X, torch.float32)
    Ec = gpu.encode(Ad, kind, form="cols")
    Er = gpu.encode(Ad, kind, form="rows")
    e = column_exponents(A) if kind == "fp16" else None
    if kind == "fp16":
        assert np.array_equal(to_np(Ec.colexp), e)
        assert int(to_np(Ec.gexp)[0]) == int(e.max())
    hi, lo = bits16(A, kind, e)
    for E, R, K, ref_hi, ref_lo in [(Ec, n, m, hi.T, None if lo is None else lo.T), (Er, m, n, hi, lo)]:
        got, pad = untile(to_np(E.hi).view(np.uint16), R, K)
        assert np.array_equal(got, ref_hi)
        assert not pad.any()
        if ref_lo is not None:
            got, pad = untile(to_np(E.lo).view(np.uint16), R, K)
            assert np.array_equal(got, ref_lo)
            assert not pad.any()
    B1 = to_np(gpu.project_encoded(Ec, Vd))
    B2 = to_np(gpu.project(Ad, Vd, precision=kind))
    assert np.array_equal(B1, B2)
    Y1 = to_np(gpu.sketch_encoded(Er, Xd))
    Y2 = to_np(gpu.sketch(Ad, Xd, precision=kind))
    assert np.array_equal(Y1, Y2)


@pytest.mark.parametrize("m,n,k,p,q,d", [(1000, 500, 20, 5, 1, 0), (2048, 1024, 100, 12, 2, 2), (777, 333, 40, 8, 0, 1)])
def test_f32_path_matches_oracle(gpu, m, n, k, p, q, d):
    """FP32 forward (FP32 MFMA products and CholeskyQR, FP64 small stage): L-values
    within 1e-5 of the FP64 oracle run on the same pivots; free comparison reported."""
    rng = np.random.default_rng(m + 3 * n)
    A = (rng.standard_normal((m, n)) / np.sqrt(n) +
         inputs.svd_matrix(m, n, np.r_[10.0 / np.arange(1, 17), np.zeros(n - 16)], m + n)).astype(np.float32)
    Om = rng.standard_normal((n, k + p)).astype(np.float32).astype(np.float64)
    f, g = _mixed_factor(gpu, A, Om, k, p, q, d, "f32")
    assert int(g["info"][0]) == 0
    frozen = oracle_rqlp(A.astype(np.float64), Om, k, p, q=q, d=d, piv0=g["piv0"], piv1=g["piv1"] if d == 0 else None)
    rel = np.abs(g["lvals"][:k] - frozen.lvals[:k]) / frozen.lvals[:k]
    free = oracle_rqlp(A.astype(np.float64), Om, k, p, q=q, d=d)
    rel_free = np.abs(g["lvals"][:k] - free.lvals[:k]) / free.lvals[:k]
    print(f"[f32 {A.shape} k={k} q={q} d={d}] frozen {rel.max():.2e} free {rel_free.max():.2e} "
          f"divergence {first_difference(g['piv0'], free.piv0)}")
    assert rel.max() < 1e-5
    Q, P = g["Q"].astype(np.float64), g["P"].astype(np.float64)
    l = k + p
    assert np.abs(Q.T @ Q - np.eye(l)).max() < 2e-5 and np.abs(P.T @ P - np.eye(l)).max() < 2e-5


@pytest.mark.parametrize("kind", ["bf16", "bf16x3"])
def test_mixed_rank_deficient_input(gpu, kind):
    """rank(A) = 40 < l = 72 with 16-bit products: the sketch's null
    directions sit at the products' rounding level instead of zero, so the
    leading L-values meet the frozen-pivot gate while the trailing ones and the
    residual are at the 16-bit rounding level (not exactly zero as in FP64)."""
    import torch
    m, n, k, p, rank = 2048, 1024, 64, 8, 40
    l = k + p
    A = inputs.svd_matrix(m, n, inputs.spectrum_poly(rank, 1.0), 77).astype(np.float32)
    Om = inputs.round_to_bf16(inputs.gaussian(n, l, 78))
    f, g = _mixed_factor(gpu, A, Om, k, p, 1, 2, kind)
    lv, piv0 = g["lvals"], g["piv0"]
    assert int(g["info"][0]) & ~0x3 == 0, f"info {int(g['info'][0]):#x}"
    frozen = oracle_rqlp(A.astype(np.float64), Om, k, p, q=1, d=2, piv0=piv0)
    rel = np.abs(lv[:rank] - frozen.lvals[:rank]) / frozen.lvals[:rank]
    tail = lv[rank:].max() / lv[0]
    Q, T, P = g["Q"].astype(np.float64), g["T"], g["P"].astype(np.float64)
    res = np.linalg.norm(A - Q @ T @ P.T) / np.linalg.norm(A)
    print(f"[{kind} rank {rank} < l {l}] leading frozen {rel.max():.2e}, trailing/L11 {tail:.2e}, residual {res:.2e}")
    assert rel.max() <= LVAL_GATE
    bound = 1e-2 if kind == "bf16" else 1e-4
    assert tail < bound and res < bound
    assert np.abs(Q.T @ Q - np.eye(l)).max() < 2e-5
