"""RQLP / ERQLP (Algorithms 2.1 and 2.2) with LAPACK's pivoted QR for the
CPQR steps: the "best CPU" timing point beside the hand-written oracle.

TEST INFRASTRUCTURE: only tests and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the GPU library.

The arithmetic is the oracle's (FP64 throughout; Y = A Omega, orthonormal
basis of range(Y) with q subspace iterations, B = V^T A, the pivoted QLP of
B), but every column-pivoted QR is LAPACK's dgeqp3 (through
scipy.linalg.qr with pivoting) and every unpivoted one LAPACK's dgeqrf,
so that the products and factorisations all run in the host's multithreaded
BLAS/LAPACK.  dgeqp3 downdates its column norms and breaks ties by its own
rule, so on matrices with near-equal residual norms its pivots can differ
from the oracle's (which recomputes norms and takes the smallest index);
on well-separated spectra both give the same pivots and the same L-values.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .rqlp import range_finder


def _positive_diag(Q: np.ndarray, R: np.ndarray):
    """Flip signs so that diag(R) >= 0 (Q's matching columns flipped too)."""
    s = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return Q * s[None, :], R * s[:, None]


def _cpqr_lapack(M: np.ndarray):
    """M[:, perm] = Q R by dgeqp3 (economic), diag(R) >= 0."""
    Q, R, perm = scipy.linalg.qr(M, mode="economic", pivoting=True, check_finite=False)
    Q, R = _positive_diag(Q, R)
    return Q, R, np.asarray(perm)


def _qr_lapack(M: np.ndarray):
    """M = Q R by dgeqrf (economic), diag(R) >= 0."""
    Q, R = np.linalg.qr(M, mode="reduced")
    return _positive_diag(Q, R)


def rqlp_lapack(A: np.ndarray, Omega: np.ndarray, k: int, p: int, q: int = 0, d: int = 0):
    """Return (Q, T, P, piv0, uplo) with A ~= Q T P^T, as the oracle's rqlp
    (Section 2: the two-stage reduction; the pivoted QLP of B for d = 0, the
    CPQR followed by d unpivoted QR steps of the transposed factor for
    d >= 1; T upper triangular for even d >= 2)."""
    A = np.asarray(A, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    l = k + p
    V = range_finder(A, Omega, q)
    B = V.T @ A
    Q0, R0, perm0 = _cpqr_lapack(B)                 # B Pi0 = Q0 R0
    if d == 0:
        Q1, R1, perm1 = _cpqr_lapack(R0.T)          # R0^T Pi1 = Q1 L^T
        T = R1.T
        QB = Q0[:, perm1]
        PB = np.empty_like(Q1)
        PB[perm0, :] = Q1
        return V @ QB, T, PB, perm0[:l].copy(), "L"
    left, right, Rprev = Q0, None, R0
    for i in range(1, d + 1):
        Qi, Ri = _qr_lapack(Rprev.T)                # R(i-1)^T = Q(i) R(i)
        if i % 2 == 1:
            right = Qi if right is None else right @ Qi
        else:
            left = left @ Qi
        Rprev = Ri
    PB = np.empty_like(right)
    PB[perm0, :] = right
    if d % 2 == 1:
        return V @ left, Rprev.T.copy(), PB, perm0[:l].copy(), "L"
    return V @ left, Rprev.copy(), PB, perm0[:l].copy(), "U"
