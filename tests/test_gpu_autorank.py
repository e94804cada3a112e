"""GPU parity of auto-rank RQLP (rqlp_factor_autorank; Section 6) against
the FP64 oracle's block-by-block loop (oracle.rqlp.autorank_rqlp) on the
same A and Omega: the rank taken, the indicator ||A||_F^2 - ||B||_F^2, the
L-values (1e-10 in FP64), Q T P^T (1e-10), zero columns past the rank,
orthonormality, and the not-converged flag.  Tolerances eps are placed
between blocks' indicators (never within rounding of one), so both sides
must stop at the same block."""
import numpy as np
import pytest

from oracle.rqlp import autorank_rqlp
from paper_1811_09334_amd import inputs

from _helpers import first_difference, to_dev, to_np

pytestmark = pytest.mark.gpu


def _check(f, rank, err2, ref, A, lmax, b, tol):
    l = ref.extra["rank"]
    assert rank == l
    nA2 = float(np.sum(A * A))
    assert abs(err2 - ref.extra["err2"]) < 1e-11 * nA2
    Q, T, P = to_np(f.Q).astype(np.float64), to_np(f.T), to_np(f.P).astype(np.float64)
    lv, piv0 = to_np(f.lvals), to_np(f.piv0)
    assert np.all(Q[:, l:] == 0) and np.all(P[:, l:] == 0) and np.all(T[l:, :] == 0) and np.all(T[:, l:] == 0)
    assert np.all(piv0[l:] == -1) and np.all(lv[l:] == 0)
    if first_difference(piv0[:l], ref.piv0) >= 0 or first_difference(to_np(f.piv1)[:l], ref.piv1) >= 0:
        return "pivots differ"
    good = ref.lvals > 1e-12 * ref.lvals.max()
    rel = np.abs(lv[:l][good] - ref.lvals[good]) / ref.lvals[good]
    assert rel.max() < tol, rel.max()
    nA = np.sqrt(nA2)
    assert np.linalg.norm(Q[:, :l] @ T[:l, :l] @ P[:, :l].T - ref.Q @ ref.T @ ref.P.T) < tol * nA
    assert np.abs(Q[:, :l].T @ Q[:, :l] - np.eye(l)).max() < 1e3 * tol
    for s0 in range(0, l, b):
        Pj = P[:, s0:min(l, s0 + b)]
        assert np.abs(Pj.T @ Pj - np.eye(Pj.shape[1])).max() < 1e3 * tol
    return "ok"


def _between(hist, j):
    """A tolerance halfway (in log scale) between hist[j] and hist[j + 1], the
    indicators after blocks j + 1 and j + 2: the loop stops after block j + 2."""
    return float(np.sqrt(hist[j] * hist[j + 1]))


@pytest.mark.parametrize("q", [0, 1])
def test_autorank_f64_matches_oracle(gpu, q):
    m, n, lmax, b = 700, 400, 96, 16
    A = inputs.svd_matrix(m, n, inputs.spectrum_exp(n, 25.0), 21)
    Om = inputs.gaussian(n, lmax, 22)
    full = autorank_rqlp(A, Om, b, 0.0, q=q)
    eps = _between(full.extra["err2_history"], 2)          # stops after 4 blocks
    ref = autorank_rqlp(A, Om, b, eps, q=q)
    assert ref.extra["rank"] == 64
    f, rank, err2 = gpu.factor_autorank(to_dev(A), lmax, b, eps, q=q, Omega=to_dev(Om))
    assert int(to_np(f.info)[0]) & ~0x1 == 0
    assert _check(f, rank, err2, ref, A, lmax, b, 1e-10) == "ok"


def test_autorank_exact_rank(gpu):
    """rank(A) = 37, b = 8: the indicator drops to rounding once 40 columns are
    taken, so a tolerance of 1e-10 ||A||^2 stops there."""
    m, n, lmax, b, r = 300, 160, 64, 8, 37
    A = inputs.svd_matrix(m, n, np.linspace(1.0, 0.2, r), 23)
    Om = inputs.gaussian(n, lmax, 24)
    eps = 1e-10 * float(np.sum(A * A))
    ref = autorank_rqlp(A, Om, b, eps, q=1)
    f, rank, err2 = gpu.factor_autorank(to_dev(A), lmax, b, eps, q=1, Omega=to_dev(Om))
    assert rank == 40 == ref.extra["rank"]
    assert err2 <= eps
    Q, T, P = to_np(f.Q)[:, :rank], to_np(f.T)[:rank, :rank], to_np(f.P)[:, :rank]
    assert np.linalg.norm(A - Q @ T @ P.T) < 1e-10 * np.linalg.norm(A)
    lv = to_np(f.lvals)
    assert np.max(np.abs(lv[:r] - ref.lvals[:r]) / ref.lvals[:r]) < 1e-10


def test_autorank_not_converged_ragged(gpu):
    """An unreachable tolerance takes every column of Omega (lmax = 50 with
    b = 16: a ragged last block of 2) and raises the not-converged flag."""
    m, n, lmax, b = 400, 200, 50, 16
    A = inputs.svd_matrix(m, n, inputs.spectrum_poly(n, 0.5), 25)
    Om = inputs.gaussian(n, lmax, 26)
    ref = autorank_rqlp(A, Om, b, 1e-30, q=0)
    f, rank, err2 = gpu.factor_autorank(to_dev(A), lmax, b, 1e-30, q=0, Omega=to_dev(Om))
    assert rank == lmax == ref.extra["rank"]
    assert int(to_np(f.info)[0]) & 0x40
    assert _check(f, rank, err2, ref, A, lmax, b, 1e-10) == "ok"


def test_autorank_single_block_is_rqlp(gpu):
    """b >= lmax: one block, plain RQLP of lmax columns."""
    m, n, lmax = 300, 150, 24
    A = inputs.svd_matrix(m, n, inputs.spectrum_poly(n, 2.0), 27)
    Om = inputs.gaussian(n, lmax, 28)
    ref = autorank_rqlp(A, Om, lmax, 1e-3, q=1)
    f, rank, err2 = gpu.factor_autorank(to_dev(A), lmax, lmax, 1e-3, q=1, Omega=to_dev(Om))
    assert rank == lmax
    assert _check(f, rank, err2, ref, A, lmax, lmax, 1e-10) == "ok"


@pytest.mark.parametrize("precision", ["f32", "bf16x3"])
def test_autorank_reduced_precision(gpu, precision):
    """FP32 and split-bfloat16 products: the same stopping block as the FP64
    oracle when eps sits between blocks' indicators (rounding of the
    indicator is far below the gap), L-values within 1e-5 (FP32) / 1e-4."""
    import torch
    m, n, lmax, b = 2048, 512, 128, 32
    A = inputs.svd_matrix(m, n, inputs.spectrum_exp(n, 40.0), 29).astype(np.float32)
    Om = inputs.gaussian(n, lmax, 30)
    Om = inputs.round_to_bf16(Om) if precision == "bf16x3" else Om.astype(np.float32).astype(np.float64)
    A64 = A.astype(np.float64)
    full = autorank_rqlp(A64, Om, b, 0.0, q=1)
    eps = _between(full.extra["err2_history"], 1)         # above after 2 blocks, below after 3
    ref = autorank_rqlp(A64, Om, b, eps, q=1)
    f, rank, err2 = gpu.factor_autorank(to_dev(A, torch.float32), lmax, b, eps, q=1, precision=precision,
                                        Omega=to_dev(Om, torch.float32))
    assert rank == ref.extra["rank"] == 96
    lv = to_np(f.lvals)
    rel = np.abs(lv[:rank] - ref.lvals) / ref.lvals
    print(f"[autorank {precision}] rank {rank}, L-value rel err {rel.max():.2e}, err2 {err2:.4e} "
          f"(oracle {ref.extra['err2']:.4e})")
    assert rel.max() < (1e-5 if precision == "f32" else 1e-4)
