"""GPU parity of the deterministic truncated pivoted QLP (rqlp_qlp; Stewart's
QLP, eq. (1.2); the QLP method of Section 5) against the oracle's
stewart_qlp(A, kt) on the same A: pivots identical where the top two
residual norms are separated (else the oracle is replayed on the GPU's
first pivots), L-values within 1e-10, Q T P^T equal to the oracle's within
1e-10, Q and P orthonormal; the full QLP (kt = min(m, n)) reconstructs A;
a rank-deficient A stops at its rank with trailing L-values 0; the paper's
pds replica at n = 2000 with kt = 125."""
import numpy as np
import pytest

from oracle.qr import cpqr as oracle_cpqr
from oracle.rqlp import stewart_qlp
from paper_1811_09334_amd import inputs

from _helpers import first_difference, to_dev, to_np

pytestmark = pytest.mark.gpu


def _run(gpu, A, kt):
    f = gpu.pivoted_qlp(to_dev(A), kt)
    return (to_np(f.Q), to_np(f.T), to_np(f.P), to_np(f.piv0), to_np(f.piv1), to_np(f.lvals),
            int(to_np(f.info)[0]))


def _compare(A, kt, out, tol=1e-10):
    Q, T, P, p0, p1, lv, info = out
    Qr, Lr, Pr, p0r, p1r = stewart_qlp(A, kt=kt)
    d0 = first_difference(p0, p0r[:kt])
    if d0 >= 0:
        # the GPU's pivot at the first difference must be a maximal column too
        tr = oracle_cpqr(A, piv=p0, want_q=False, want_trace=True, steps=kt).trace
        assert tr[d0, 1] >= tr[d0, 0] * (1 - 1e-8), f"first-CPQR pivot {d0} not maximal"
        return "pivots differ"
    assert first_difference(p1, p1r) < 0
    lr = np.diag(Lr)
    good = lr > 1e-12 * lr.max()
    assert np.max(np.abs(lv[good] - lr[good]) / lr[good]) < tol
    nA = np.linalg.norm(A)
    assert np.linalg.norm(Q @ T @ P.T - Qr @ Lr @ Pr.T) < tol * nA
    assert np.abs(Q.T @ Q - np.eye(kt)).max() < 1e-12
    assert np.abs(P.T @ P - np.eye(kt)).max() < 1e-12
    assert np.allclose(np.triu(T, 1), 0.0)
    return "ok"


@pytest.mark.parametrize("m,n,kt", [(60, 40, 12), (50, 50, 20), (300, 200, 50), (1000, 800, 125), (777, 333, 64),
                                    (4100, 600, 40)])
def test_truncated_qlp_matches_oracle(gpu, m, n, kt):
    A = inputs.svd_matrix(m, n, inputs.spectrum_exp(n, n / 8.0), m + kt)
    assert _compare(A, kt, _run(gpu, A, kt)) == "ok"


@pytest.mark.parametrize("m,n", [(80, 30), (40, 40)])
def test_full_qlp_reconstructs(gpu, m, n):
    A = inputs.svd_matrix(m, n, inputs.spectrum_poly(n, 1.0), m * n)
    kt = min(m, n)
    out = _run(gpu, A, kt)
    assert _compare(A, kt, out) == "ok"
    Q, T, P = out[:3]
    assert np.linalg.norm(Q @ T @ P.T - A) < 1e-12 * np.linalg.norm(A)


def test_rank_deficient_qlp(gpu):
    m, n, r, kt = 120, 90, 10, 20
    A = inputs.svd_matrix(m, n, inputs.spectrum_poly(r, 1.0), 41)
    Q, T, P, p0, p1, lv, info = _run(gpu, A, kt)
    Qr, Lr, Pr, p0r, p1r = stewart_qlp(A, kt=kt)
    assert info & 0x2 and not info & (0x4 | 0x8 | 0x10)
    assert np.all(lv[r:] == 0.0)
    assert np.array_equal(p0[:r], p0r[:r])
    assert np.max(np.abs(lv[:r] - np.diag(Lr)[:r]) / np.diag(Lr)[:r]) < 1e-10
    assert np.linalg.norm(Q @ T @ P.T - A) < 1e-12 * np.linalg.norm(A)
    assert np.abs(Q.T @ Q - np.eye(kt)).max() < 1e-12


@pytest.mark.timeout(300)
def test_qlp_paper_example(gpu):
    w = inputs.paper_example("pds", 2000)
    A = inputs.make_matrix(w)
    out = _run(gpu, A, 125)
    assert _compare(A, 125, out) == "ok"
