"""Pins of the reference gradient (oracle/adjoint.py): the torch forward with
frozen pivots reproduces the NumPy oracle's T, and the autograd gradient
matches central finite differences of the NumPy oracle (an independent
implementation) along random directions and single coordinates."""
import numpy as np
import pytest

from oracle.adjoint import directional_fd, t_factor_torch, vjp, weights_cotangent
from oracle.rqlp import rqlp
from paper_1811_09334_amd import inputs


def _fd_problem(m=200, n=100, k=10, p=8, seed=7):
    """The finite-difference configuration: N(0,1)/sqrt(n) plus a rank-min(64,
    n/2) signal with s_j = 10/j (the differentiable workload's recipe at
    200 x 100), FP64."""
    rank = min(64, n // 2)
    A = inputs.lowrank_plus_noise(m, n, 10.0 * inputs.spectrum_poly(rank, 1.0), 1.0 / np.sqrt(n), seed,
                                  noise_first=True)
    Om = inputs.gaussian(n, k + p, seed + 1)
    w = inputs.uniform_weights(k, seed + 2)
    return A, Om, w


@pytest.mark.parametrize("q,d", [(0, 0), (1, 0), (1, 1), (1, 2), (2, 3)])
def test_torch_forward_matches_numpy_oracle(q, d):
    import torch
    A, Om, _ = _fd_problem()
    k, p = 10, 8
    ref = rqlp(A, Om, k, p, q=q, d=d)
    T, uplo = t_factor_torch(torch.tensor(A), torch.tensor(Om), k, p, q, d, ref.piv0,
                             ref.piv1 if d == 0 else None)
    assert uplo == ref.uplo
    assert np.allclose(T.numpy(), ref.T, atol=1e-12 * np.abs(ref.T).max())


@pytest.mark.parametrize("q,d", [(1, 0), (0, 0), (1, 1), (2, 2)])
def test_gradient_matches_directional_finite_differences(q, d):
    A, Om, w = _fd_problem()
    k, p = 10, 8
    l = k + p
    ref = rqlp(A, Om, k, p, q=q, d=d)
    dT = weights_cotangent(w, l)
    G, _ = vjp(A, Om, k, p, q, d, ref.piv0, ref.piv1, dT)
    rng = np.random.default_rng(11)
    h = 1e-6 * np.abs(A).max()
    for _ in range(4):
        E = rng.standard_normal(A.shape)
        fd = directional_fd(A, Om, k, p, q, d, ref.piv0, ref.piv1, dT, E, h)
        an = float(np.sum(G * E))
        assert abs(an - fd) <= 1e-7 * max(abs(fd), np.linalg.norm(G) * np.linalg.norm(E) * 1e-3)


def test_gradient_single_coordinates_and_full_cotangent():
    """Coordinate-wise FD on a sample of entries, with a general lower
    triangular cotangent dT (every entry of T, not only its diagonal)."""
    A, Om, _ = _fd_problem(m=120, n=60, k=8, p=6, seed=3)
    k, p, q = 8, 6, 1
    l = k + p
    ref = rqlp(A, Om, k, p, q=q, d=0)
    rng = np.random.default_rng(5)
    dT = np.tril(rng.standard_normal((l, l)))
    G, _ = vjp(A, Om, k, p, q, 0, ref.piv0, ref.piv1, dT)
    h = 1e-6 * np.abs(A).max()
    idx = rng.choice(A.size, 40, replace=False)
    for flat in idx:
        i, j = np.unravel_index(flat, A.shape)
        E = np.zeros_like(A)
        E[i, j] = 1.0
        fd = directional_fd(A, Om, k, p, q, 0, ref.piv0, ref.piv1, dT, E, h)
        assert abs(G[i, j] - fd) <= 1e-6 * np.abs(G).max()


def test_gradient_of_leading_lvalue_of_rank_one_matrix():
    """A = s u v^T: L_11 = s (exact), so d L_11 / dA = u v^T (the gradient of
    the largest singular value); a closed form independent of any QR code."""
    rng = np.random.default_rng(9)
    m, n = 40, 20
    u = rng.standard_normal(m)
    u /= np.linalg.norm(u)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    A = 3.0 * np.outer(u, v) + 1e-9 * rng.standard_normal((m, n))   # the tiny term keeps every QR full rank
    Om = rng.standard_normal((n, 6))
    ref = rqlp(A, Om, 4, 2, q=0, d=0)
    G, T = vjp(A, Om, 4, 2, 0, 0, ref.piv0, ref.piv1, weights_cotangent(np.array([1.0]), 6))
    assert abs(T[0, 0] - 3.0) < 1e-7
    assert np.abs(G - np.outer(u, v)).max() < 1e-6
