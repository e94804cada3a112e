"""Householder QR and column-pivoted Householder QR, written out by hand in FP64.

TEST INFRASTRUCTURE: part of the CPU oracle.  Only tests, the smoke check
and the benchmark's CPU-baseline leg may import this module.

Definitions followed
--------------------
* CPQR (Section 1, the R-values paragraph): A Pi = Q R with a permutation Pi,
  upper-triangular R, orthogonal Q.  The pivot rule is Businger-Golub: at step
  j the column of the trailing block with the largest residual 2-norm is
  moved to position j.  Residual norms are recomputed exactly every step (no
  downdating).  Ties go to the column with the smallest original index.
* Every factor is normalised so that diag(R) >= 0 (Q's matching column is
  negated), which makes Q and R unique for fixed pivots.
* Numerical rank stop: when the largest residual norm is <= tol
  (default max(rows, cols) * eps * ||M||_F) the factorisation stops at step
  r; rows r.. of R are set to zero, the remaining positions of the
  permutation list the untouched columns in ascending original index, and
  ``rank = r`` is reported.

The reflector is the textbook one: v = x + sign(x_0) ||x|| e_1,
H = I - 2 v v^T / (v^T v), H x = -sign(x_0) ||x|| e_1; the sign is fixed
afterwards by the normalisation above.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

EPS = float(np.finfo(np.float64).eps)


@dataclass
class QRResult:
    Q: np.ndarray          # rows x kmax, orthonormal columns
    R: np.ndarray          # kmax x cols, upper trapezoidal, diag >= 0
    perm: np.ndarray       # cols: M[:, perm] = Q R  (perm[:kmax] are the pivots)
    rank: int              # kmax unless the numerical-rank stop fired
    trace: Optional[np.ndarray] = None   # per step: (largest, chosen, second largest) residual norm


def _reflector(x: np.ndarray):
    """Return v (or None for x == 0) with (I - 2 v v^T / v^T v) x = -sign(x0) ||x|| e_1."""
    nx = float(np.sqrt(np.sum(x * x)))
    if nx == 0.0:
        return None
    v = x.copy()
    v[0] += nx if x[0] >= 0.0 else -nx
    return v


def _apply(v: np.ndarray, M: np.ndarray) -> None:
    """In place: M <- (I - 2 v v^T / v^T v) M  (M has len(v) rows)."""
    M -= np.outer(v, (2.0 / float(v @ v)) * (v @ M))


def _householder_qr(M: np.ndarray, piv: Optional[Sequence[int]], pivoting: bool,
                    tol: Optional[float], want_q: bool, want_trace: bool = False,
                    steps: Optional[int] = None) -> QRResult:
    R = np.array(M, dtype=np.float64, copy=True, order="F")
    rows, cols = R.shape
    kmax = min(rows, cols) if steps is None else min(rows, cols, int(steps))
    perm = np.arange(cols)
    if tol is None:
        tol = max(rows, cols) * EPS * float(np.sqrt(np.sum(R * R)))
    refl = []
    rank = kmax
    trace = []
    for j in range(kmax):
        if want_trace:
            nrm = np.sqrt(np.sum(R[j:, j:] * R[j:, j:], axis=0))
            srt = np.sort(nrm)[::-1]
            chosen = nrm[int(np.flatnonzero(perm[j:] == int(piv[j]))[0])] if piv is not None else srt[0]
            trace.append((srt[0], chosen, srt[1] if len(srt) > 1 else 0.0))
        if piv is not None:
            p = j + int(np.flatnonzero(perm[j:] == int(piv[j]))[0])
        elif pivoting:
            norms = np.sqrt(np.sum(R[j:, j:] * R[j:, j:], axis=0))
            best = float(norms.max())
            if best <= tol:
                rank = j
                break
            cand = np.flatnonzero(norms == best)
            p = j + int(cand[np.argmin(perm[j + cand])])
        else:
            p = j
        if p != j:
            R[:, [j, p]] = R[:, [p, j]]
            perm[[j, p]] = perm[[p, j]]
        v = _reflector(R[j:, j])
        if v is not None:
            _apply(v, R[j:, j:])
            refl.append((j, v))
        R[j + 1:, j] = 0.0
    if rank < kmax:
        R[rank:, :] = 0.0
        rest = np.argsort(perm[rank:], kind="stable")
        perm[rank:] = perm[rank:][rest]
        R[:, rank:] = R[:, rank:][:, rest]
    R = R[:kmax, :]
    # sign normalisation: diag(R) >= 0
    sgn = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    R = R * sgn[:, None]
    Q = None
    if want_q:
        E = np.zeros((rows, kmax))
        E[np.arange(kmax), np.arange(kmax)] = 1.0
        for j, v in reversed(refl):
            _apply(v, E[j:, :])
        Q = E * sgn[None, :]
    return QRResult(Q=Q, R=np.triu(R), perm=perm, rank=rank,
                    trace=np.array(trace) if want_trace else None)


def cpqr(M: np.ndarray, piv: Optional[Sequence[int]] = None, tol: Optional[float] = None,
         want_q: bool = True, want_trace: bool = False, steps: Optional[int] = None) -> QRResult:
    """Column-pivoted QR M[:, perm] = Q R (Businger-Golub, exact norm recompute).

    ``piv`` (optional) freezes the first min(rows, cols) pivots (original
    column indices); the rank stop is then disabled.  ``want_trace`` records,
    for every step, the largest residual column norm, the norm of the column
    taken and the second largest norm (used to judge pivot ties).  ``steps``
    (optional) stops after that many Householder steps (truncated CPQR): Q has
    ``steps`` columns, R is steps x cols, perm[:steps] are the pivots and the
    other columns of R hold the leading rows of the untouched trailing block."""
    return _householder_qr(M, piv, True, tol, want_q, want_trace, steps)


def householder_qr(M: np.ndarray, want_q: bool = True) -> QRResult:
    """Unpivoted Householder QR, M = Q R with diag(R) >= 0 (thin Q)."""
    return _householder_qr(M, None, False, 0.0, want_q)
