"""Pins for the oracle's hand-written Householder QR and column-pivoted QR.

The oracle is checked against things other than itself: LAPACK's dgeqp3 /
dgeqrf (via SciPy / NumPy), closed forms and the rank/tie rules."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.qr import cpqr, householder_qr


def _check_factor(M, f, tol=1e-13):
    rows, cols = M.shape
    kmax = min(rows, cols)
    scale = max(1.0, np.linalg.norm(M))
    assert f.Q.shape == (rows, kmax) and f.R.shape == (kmax, cols)
    assert np.allclose(np.tril(f.R, -1), 0.0)
    assert np.all(np.diag(f.R) >= 0.0)
    assert np.abs(f.Q.T @ f.Q - np.eye(kmax)).max() < 10 * tol * max(rows, cols)
    assert np.linalg.norm(M[:, f.perm] - f.Q @ f.R) <= tol * scale * max(rows, cols)
    assert sorted(f.perm.tolist()) == list(range(cols))


@pytest.mark.parametrize("shape", [(40, 25), (25, 40), (30, 30), (7, 90), (90, 7)])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cpqr_matches_lapack_dgeqp3(shape, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal(shape) * np.logspace(0, -3, shape[1])[None, :]
    f = cpqr(M)
    _check_factor(M, f)
    _, R, P = sla.qr(M, pivoting=True, mode="economic")
    kmax = min(shape)
    assert np.array_equal(f.perm[:kmax], P[:kmax])
    # dgeqp3 does not normalise signs: flip its rows so that diag(R) >= 0
    sgn = np.where(np.diag(R[:kmax, :kmax]) < 0, -1.0, 1.0)
    assert np.allclose(R[:kmax, :kmax] * sgn[:, None], f.R[:, :kmax], rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("shape", [(50, 20), (20, 20), (20, 50)])
def test_unpivoted_qr_matches_lapack(shape):
    rng = np.random.default_rng(5)
    M = rng.standard_normal(shape)
    f = householder_qr(M)
    _check_factor(M, f)
    assert np.array_equal(f.perm, np.arange(shape[1]))
    q, r = np.linalg.qr(M)
    s = np.sign(np.diag(r))
    assert np.allclose(q * s, f.Q, atol=1e-12)
    assert np.allclose(r * s[:, None], f.R, atol=1e-12)


def test_cpqr_diagonal_closed_form():
    d = np.array([0.3, -2.0, 1.5, 0.01, -0.7])
    M = np.diag(d)
    f = cpqr(M)
    order = np.argsort(-np.abs(d), kind="stable")
    assert np.array_equal(f.perm, order)
    assert np.allclose(f.R, np.diag(np.abs(d)[order]), rtol=1e-15, atol=1e-15)
    # Q is the signed permutation
    assert np.allclose(np.abs(f.Q), np.eye(5)[:, order])


def test_cpqr_ties_go_to_smallest_index():
    f = cpqr(np.eye(6))
    assert np.array_equal(f.perm, np.arange(6))
    M = np.zeros((3, 5))
    M[0, 4] = M[1, 2] = M[2, 0] = 1.0     # three unit columns of equal norm
    f = cpqr(M)
    assert f.perm[:3].tolist() == [0, 2, 4]


def test_cpqr_rank_one_closed_form():
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(12), rng.standard_normal(9)
    M = np.outer(u, v)
    f = cpqr(M)
    assert f.rank == 1
    assert f.perm[0] == int(np.argmax(np.abs(v)))
    assert np.isclose(f.R[0, 0], np.linalg.norm(u) * np.abs(v).max(), rtol=1e-14)
    assert np.allclose(f.R[1:, :], 0.0)
    # first row of R is |u| * v[perm] up to the sign of the pivot entry
    assert np.allclose(f.R[0, :], np.linalg.norm(u) * v[f.perm] * np.sign(v[f.perm[0]]), rtol=1e-13)


def test_cpqr_rank_deficient_stop():
    rng = np.random.default_rng(4)
    M = rng.standard_normal((30, 5)) @ rng.standard_normal((5, 40))
    f = cpqr(M)
    assert f.rank == 5
    assert np.allclose(f.R[5:], 0.0)
    # remaining pivots follow in ascending original index
    assert np.all(np.diff(f.perm[5:]) > 0)
    assert np.linalg.norm(M[:, f.perm] - f.Q @ f.R) < 1e-12 * np.linalg.norm(M)
    assert np.abs(f.Q.T @ f.Q - np.eye(30)).max() < 1e-13


def test_cpqr_frozen_pivots_reproduce_free_run():
    rng = np.random.default_rng(6)
    M = rng.standard_normal((15, 40))
    f = cpqr(M)
    g = cpqr(M, piv=f.perm[:15])
    assert np.array_equal(f.perm[:15], g.perm[:15])
    assert np.allclose(f.R[:, :15], g.R[:, :15], atol=1e-14)
    # an arbitrary frozen order is still a valid QR of the permuted matrix
    piv = rng.permutation(40)[:15]
    h = cpqr(M, piv=piv)
    assert np.array_equal(h.perm[:15], piv)
    _check_factor(M, h)


def test_cpqr_trace_records_step_norms():
    rng = np.random.default_rng(8)
    M = rng.standard_normal((6, 20))
    f = cpqr(M, want_trace=True)
    assert f.trace.shape == (6, 3)
    # free run: the chosen norm is the largest; the first largest is the largest column norm of M
    assert np.allclose(f.trace[:, 0], f.trace[:, 1])
    assert np.isclose(f.trace[0, 0], np.linalg.norm(M, axis=0).max())
    assert np.all(f.trace[:, 2] <= f.trace[:, 0])
    # a frozen run records the norm of the imposed pivot
    piv = f.perm[:6][::-1]
    g = cpqr(M, piv=piv, want_trace=True)
    assert np.isclose(g.trace[0, 1], np.linalg.norm(M[:, piv[0]]))
