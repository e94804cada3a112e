"""Pins of the auto-rank (fixed-accuracy) RQLP oracle (Section 6; the
identity (fixedrank) of Section 2), against what the mathematics fixes:

  * at the stop, ||A - Q T P^T||_F^2 equals the indicator ||A||_F^2 - ||B||_F^2;
  * the indicator after every block equals the brute-force
    ||A - V V^T A||_F^2 of the blocks so far, and never increases;
  * exact rank r: once the columns taken reach r the sketch holds range(A),
    so with a tolerance above rounding the loop stops at the first block
    boundary >= r, and not before (Eckart-Young: fewer columns leave at least
    sigma_r^2);
  * known spectrum: the rank taken is at least the smallest l with
    sum_{i > l} sigma_i^2 <= eps (no rank-l matrix does better), the block
    before the stop is still above eps, and an unreachable tolerance uses
    every column of Omega and reports no convergence;
  * the factors are those of block RQLP on the columns taken."""
import numpy as np
import pytest

from oracle.rqlp import autorank_rqlp, brqlp
from paper_1811_09334_amd import inputs


def _spectrum_matrix(m, n, s, seed):
    return inputs.svd_matrix(m, n, np.asarray(s, dtype=np.float64), seed)


@pytest.mark.parametrize("q", [0, 1])
def test_identity_at_stop(q):
    A = _spectrum_matrix(120, 80, inputs.spectrum_exp(80, 10.0), 3)
    Om = inputs.gaussian(80, 48, 4)
    nA2 = float(np.sum(A * A))
    r = autorank_rqlp(A, Om, 8, 1e-3 * nA2, q=q)
    E = A - r.Q @ r.T @ r.P.T
    assert abs(float(np.sum(E * E)) - r.extra["err2"]) < 1e-12 * nA2
    assert r.extra["converged"]


@pytest.mark.parametrize("q", [0, 2])
def test_history_is_projection_error_and_nonincreasing(q):
    A = _spectrum_matrix(100, 60, inputs.spectrum_poly(60, 1.0), 5)
    Om = inputs.gaussian(60, 40, 6)
    r = autorank_rqlp(A, Om, 8, 0.0, q=q)                 # never converges: every block
    hist = r.extra["err2_history"]
    assert len(hist) == 5 and not r.extra["converged"] and r.extra["rank"] == 40
    for j in range(1, len(hist) + 1):
        V = r.V[:, :8 * j]
        E = A - V @ (V.T @ A)
        assert abs(hist[j - 1] - float(np.sum(E * E))) < 1e-12 * float(np.sum(A * A))
    assert all(hist[j + 1] <= hist[j] + 1e-12 for j in range(len(hist) - 1))


@pytest.mark.parametrize("q", [0, 1])
def test_exact_rank_stops_at_first_block_past_rank(q):
    rank, b = 37, 8
    A = _spectrum_matrix(150, 90, np.linspace(1.0, 0.2, rank), 7)
    Om = inputs.gaussian(90, 64, 8)
    nA2 = float(np.sum(A * A))
    r = autorank_rqlp(A, Om, b, 1e-10 * nA2, q=q)
    assert r.extra["rank"] == 40                           # ceil(37 / 8) blocks
    assert r.extra["err2_history"][-2] >= 0.2 ** 2 * (1 - 1e-8)   # 32 columns leave >= sigma_37^2
    assert np.linalg.norm(A - r.Q @ r.T @ r.P.T) < 1e-10 * np.sqrt(nA2)


def test_rank_at_least_eckart_young_minimum_and_first_crossing():
    n = 80
    s = inputs.spectrum_exp(n, 12.0)
    A = _spectrum_matrix(140, n, s, 9)
    Om = inputs.gaussian(n, 64, 10)
    tail = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1][1:], [0.0]])   # tail[l-1] = sum_{i > l} s_i^2
    for eps_rel in (1e-2, 1e-3, 1e-4):
        eps = eps_rel * float(np.sum(s ** 2))
        r = autorank_rqlp(A, Om, 8, eps, q=1)
        l = r.extra["rank"]
        lstar = int(np.argmax(tail <= eps)) + 1
        assert l >= lstar
        assert r.extra["err2"] <= eps and r.extra["converged"]
        if len(r.extra["err2_history"]) > 1:
            assert r.extra["err2_history"][-2] > eps


def test_unreachable_tolerance_uses_every_column():
    A = _spectrum_matrix(60, 40, inputs.spectrum_poly(40, 0.5), 11)
    Om = inputs.gaussian(40, 20, 12)
    r = autorank_rqlp(A, Om, 6, 1e-30, q=0)               # 20 = 3 x 6 + 2: ragged last block
    assert r.extra["rank"] == 20 and not r.extra["converged"]
    assert r.T.shape == (20, 20) and r.Q.shape == (60, 20)


def test_factors_are_block_rqlp_of_columns_taken():
    A = _spectrum_matrix(110, 70, inputs.spectrum_exp(70, 9.0), 13)
    Om = inputs.gaussian(70, 48, 14)
    nA2 = float(np.sum(A * A))
    r = autorank_rqlp(A, Om, 8, 1e-3 * nA2, q=1)
    l = r.extra["rank"]
    assert l < 48
    ref = brqlp(A, Om[:, :l], l - 2, 2, 8, q=1, deflate=False)
    assert np.array_equal(r.piv0, ref.piv0) and np.array_equal(r.piv1, ref.piv1)
    assert np.allclose(r.T, ref.T, atol=1e-12) and np.allclose(r.Q, ref.Q, atol=1e-12)
