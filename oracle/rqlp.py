"""FP64 CPU oracle for randomized QLP: RQLP (Algorithm 2.1), ERQLP
(Algorithm 2.2) and block RQLP (Algorithm 4.1).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library; it takes the Gaussian test matrix Omega as data.

Notation follows the paper: A is m x n, k the target rank, p the
oversampling, l = k + p, d the number of inner (unpivoted) QR steps of ERQLP,
b the block size of block RQLP.  q (subspace/power iterations of the range
finder, Halko et al. 2011, Sec. 4.5) is an extra input here: with
q = 0 the range finder is exactly the paper's (Section 2, three steps).

Readings taken where the paper is silent or inconsistent (listed with the
reasons in the design notes):
  * Omega is N(0,1) (the listing writes rand but its comment says Gaussian).
  * Orthonormalisation uses Householder QR (LAPACK via numpy.linalg.qr); any
    orthonormal basis of range(Y) gives the same B-factors.
  * Power iterations re-orthonormalise after every product.
  * Every QR / CPQR has diag(R) >= 0; pivots tie-break to the smallest index.
  * ERQLP assembly for even d: from R_{i-1}^T = Q_i R_i one gets
    B Pi = Q0 Q2 ... Q_d  R_d  (Q1 Q3 ... Q_{d-1})^T, so the middle factor is
    the UPPER triangular R_d (the printed L = R_d^T does not reproduce B for
    even d).  T is returned with uplo = 'U' for even d >= 2 and 'L' otherwise.
  * Block RQLP with q > 0: per-block power iterations on the original A,
    then the reorthogonalisation of step 5 applied twice.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from .qr import cpqr, householder_qr


@dataclass
class QLPResult:
    Q: np.ndarray            # m x l
    T: np.ndarray            # l x l triangular ("L")
    P: np.ndarray            # n x l
    piv0: np.ndarray         # first l pivots of the CPQR of B (original column indices)
    piv1: np.ndarray         # pivots of the second CPQR (identity for d >= 1)
    uplo: str                # 'L' or 'U'
    rank0: int               # numerical rank found by the first CPQR
    V: Optional[np.ndarray] = None   # range-finder basis
    B: Optional[np.ndarray] = None   # reduced matrix V^T A
    extra: dict = field(default_factory=dict)

    @property
    def lvals(self) -> np.ndarray:
        return np.diag(self.T).copy()


# ---------------------------------------------------------------------------
# range finder (Section 2: draw Omega, Y = A Omega, orthonormalise Y)
# ---------------------------------------------------------------------------
def orthonormal_basis(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis V of range(Y): thin Householder QR (LAPACK)."""
    V, _ = np.linalg.qr(Y, mode="reduced")
    return V


def range_finder(A: np.ndarray, Omega: np.ndarray, q: int = 0) -> np.ndarray:
    """V = orth(A Omega), followed by q subspace iterations W = orth(A^T V), V = orth(A W)."""
    V = orthonormal_basis(A @ Omega)
    for _ in range(q):
        W = orthonormal_basis(A.T @ V)
        V = orthonormal_basis(A @ W)
    return V


# ---------------------------------------------------------------------------
# pivoted QLP of the reduced matrix B (Alg. 2.1 and Alg. 2.2)
# ---------------------------------------------------------------------------
def _rows_by_perm(perm: np.ndarray, M: np.ndarray) -> np.ndarray:
    """Pi M for the permutation matrix Pi with (X Pi) = X[:, perm]: row perm[i] <- row i."""
    out = np.empty_like(M)
    out[perm, :] = M
    return out


def qlp_reduced(B: np.ndarray, d: int = 0, piv0: Optional[Sequence[int]] = None,
                piv1: Optional[Sequence[int]] = None):
    """Return (QB, T, PB, piv0, piv1, uplo, rank0) with B ~= QB T PB^T.

    d = 0: pivoted QLP (Stewart): B Pi0 = Q0 R0, R0^T Pi1 = Q1 L^T,
           QB = Q0 Pi1, PB = Pi0 Q1, T = L.
    d >= 1: B Pi0 = Q(0) R(0); R(i-1)^T = Q(i) R(i), i = 1..d (unpivoted);
           QB = Q(0) prod_{even i} Q(i), PB = Pi0 prod_{odd i} Q(i),
           T = R(d)^T (d odd) or R(d) (d even)."""
    l, n = B.shape
    f0 = cpqr(B, piv=piv0)
    Q0, R0, perm0 = f0.Q, f0.R, f0.perm            # Q0: l x l, R0: l x n
    if d == 0:
        f1 = cpqr(R0.T, piv=piv1)                   # R0^T Pi1 = Q1 L^T, Q1: n x l
        T = f1.R.T
        QB = Q0[:, f1.perm]
        PB = _rows_by_perm(perm0, f1.Q)
        return QB, T, PB, perm0[:l].copy(), f1.perm[:l].copy(), "L", f0.rank
    left = Q0
    right = None
    Rprev = R0
    for i in range(1, d + 1):
        fi = householder_qr(Rprev.T)                # R(i-1)^T = Q(i) R(i)
        if i % 2 == 1:
            right = fi.Q if right is None else right @ fi.Q
        else:
            left = left @ fi.Q
        Rprev = fi.R
    PB = _rows_by_perm(perm0, right)
    if d % 2 == 1:
        T, uplo = Rprev.T.copy(), "L"
    else:
        T, uplo = Rprev.copy(), "U"
    return left, T, PB, perm0[:l].copy(), np.arange(l), uplo, f0.rank


def qlp_reduced_printed_even(B: np.ndarray, d: int):
    """ERQLP step 9 exactly as printed for even d (L = R(d)^T).  Kept only so a
    test can show it fails to reproduce B; not used by the oracle."""
    l, n = B.shape
    f0 = cpqr(B)
    left, right, Rprev = f0.Q, None, f0.R
    for i in range(1, d + 1):
        fi = householder_qr(Rprev.T)
        if i % 2 == 1:
            right = fi.Q if right is None else right @ fi.Q
        else:
            left = left @ fi.Q
        Rprev = fi.R
    return left, Rprev.T.copy(), _rows_by_perm(f0.perm, right)


# ---------------------------------------------------------------------------
# RQLP / ERQLP (Alg. 2.1 / 2.2)
# ---------------------------------------------------------------------------
def rqlp(A: np.ndarray, Omega: np.ndarray, k: int, p: int, q: int = 0, d: int = 0,
         piv0: Optional[Sequence[int]] = None, piv1: Optional[Sequence[int]] = None) -> QLPResult:
    """Randomized QLP of A (m x n) with the given n x (k+p) Gaussian matrix Omega.

    Steps: Y = A Omega; V an orthonormal basis of range(Y) (+ q power iterations); B = V^T A;
    pivoted QLP of B (d = 0) or CPQR + d inner QRs (d >= 1); Q = V QB, P = PB."""
    A = np.asarray(A, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    l = k + p
    assert Omega.shape == (A.shape[1], l)
    V = range_finder(A, Omega, q)
    B = V.T @ A
    QB, T, PB, p0, p1, uplo, rank0 = qlp_reduced(B, d, piv0, piv1)
    return QLPResult(Q=V @ QB, T=T, P=PB, piv0=p0, piv1=p1, uplo=uplo, rank0=rank0, V=V, B=B)


# ---------------------------------------------------------------------------
# block RQLP (Alg. 4.1)
# ---------------------------------------------------------------------------
def brqlp(A: np.ndarray, Omega: np.ndarray, k: int, p: int, b: int, q: int = 0,
          deflate: bool = True, piv0: Optional[Sequence[int]] = None,
          piv1: Optional[Sequence[int]] = None) -> QLPResult:
    """Block randomized QLP.  Blocks of b columns of Omega (the last one ragged
    when b does not divide l).  Per block j: Y_j = A Omega_j, V_j orthonormal with range Y_j
    (+ q power iterations on the original A), V_j re-orthogonalised against
    V_1..V_{j-1} (twice), B_j = V_j^T A^(j-1), A^(j) = A^(j-1) - V_j B_j,
    pivoted QLP of B_j, Q_j = V_j QB_j, P_j = PB_j; T = blkdiag(L_j).
    piv0 / piv1 (optional, per block and concatenated as returned) freeze the
    pivots of the per-block factorisations."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = k + p
    starts = list(range(0, l, b))
    Aj = A.copy() if deflate else A
    Vs, Qs, Ps, Ts, p0s, p1s = [], [], [], [], [], []
    for s0 in starts:
        s1 = min(l, s0 + b)
        Vj = range_finder(A, Omega[:, s0:s1], q)
        for _ in range(2):
            if Vs:
                Vprev = np.hstack(Vs)
                Vj = Vj - Vprev @ (Vprev.T @ Vj)
            Vj = orthonormal_basis(Vj)
        Bj = Vj.T @ Aj
        if deflate:
            Aj = Aj - Vj @ Bj
        f0 = None if piv0 is None else np.asarray(piv0)[s0:s1]
        f1 = None if piv1 is None else np.asarray(piv1)[s0:s1]
        QB, Lj, PB, p0, p1, _, _ = qlp_reduced(Bj, 0, f0, f1)
        Vs.append(Vj)
        Qs.append(Vj @ QB)
        Ps.append(PB)
        Ts.append(Lj)
        p0s.append(p0)
        p1s.append(p1)
    T = np.zeros((l, l))
    for s0, Lj in zip(starts, Ts):
        T[s0:s0 + Lj.shape[0], s0:s0 + Lj.shape[1]] = Lj
    V = np.hstack(Vs)
    return QLPResult(Q=np.hstack(Qs), T=T, P=np.hstack(Ps), piv0=np.concatenate(p0s),
                     piv1=np.concatenate(p1s), uplo="L", rank0=l, V=V, B=V.T @ A,
                     extra={"blocks": [(s0, min(l, s0 + b)) for s0 in starts]})


# ---------------------------------------------------------------------------
# auto-rank (fixed-accuracy) RQLP (Section 6, with the identity (fixedrank) of
# Section 2)
# ---------------------------------------------------------------------------
def autorank_rqlp(A: np.ndarray, Omega: np.ndarray, b: int, eps: float, q: int = 0,
                  piv0: Optional[Sequence[int]] = None, piv1: Optional[Sequence[int]] = None) -> QLPResult:
    """Block RQLP whose rank is set by an accuracy tolerance.

    The basis grows one block of b columns of Omega at a time (Algorithm 4.1:
    range finder on the original A, reorthogonalisation twice against the
    earlier blocks, B_j = V_j^T A); after each block the error indicator
    ||E||_F^2 = ||A||_F^2 - ||B||_F^2 of Section 6 (the identity (fixedrank):
    it equals ||A - V V^T A||_F^2) is evaluated with B the blocks so far, and
    the loop stops at the first block where it is <= eps, or when the columns
    of Omega (n x lmax) are used up.  The pivoted QLPs of the blocks taken
    then give Q, T = blkdiag(L_j), P as in Algorithm 4.1.  extra["rank"] is
    the number of columns taken, extra["err2"] the indicator there,
    extra["err2_history"] its value after each block, extra["converged"]
    whether it reached eps.  piv0 / piv1 freeze the per-block pivots."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    lmax = Omega.shape[1]
    normA2 = float(np.sum(A * A))
    normB2 = 0.0
    Vs, Bs, hist = [], [], []
    s0 = 0
    while s0 < lmax:
        s1 = min(lmax, s0 + b)
        Vj = range_finder(A, Omega[:, s0:s1], q)
        for _ in range(2):
            if Vs:
                Vprev = np.hstack(Vs)
                Vj = Vj - Vprev @ (Vprev.T @ Vj)
            Vj = orthonormal_basis(Vj)
        Bj = Vj.T @ A
        Vs.append(Vj)
        Bs.append(Bj)
        normB2 += float(np.sum(Bj * Bj))
        hist.append(normA2 - normB2)
        s0 = s1
        if hist[-1] <= eps:
            break
    l = s0
    Qs, Ps, Ts, p0s, p1s = [], [], [], [], []
    for j, (Vj, Bj) in enumerate(zip(Vs, Bs)):
        a, e = j * b, j * b + Bj.shape[0]
        f0 = None if piv0 is None else np.asarray(piv0)[a:e]
        f1 = None if piv1 is None else np.asarray(piv1)[a:e]
        QB, Lj, PB, p0, p1, _, _ = qlp_reduced(Bj, 0, f0, f1)
        Qs.append(Vj @ QB)
        Ps.append(PB)
        Ts.append(Lj)
        p0s.append(p0)
        p1s.append(p1)
    T = np.zeros((l, l))
    for j, Lj in enumerate(Ts):
        T[j * b:j * b + Lj.shape[0], j * b:j * b + Lj.shape[1]] = Lj
    V = np.hstack(Vs)
    return QLPResult(Q=np.hstack(Qs), T=T, P=np.hstack(Ps), piv0=np.concatenate(p0s),
                     piv1=np.concatenate(p1s), uplo="L", rank0=l, V=V, B=np.vstack(Bs),
                     extra={"rank": l, "err2": hist[-1], "err2_history": hist, "normA2": normA2,
                            "converged": hist[-1] <= eps})


# ---------------------------------------------------------------------------
# deterministic pivoted QLP (Stewart; eq. (1.2))
# ---------------------------------------------------------------------------
def stewart_qlp(A: np.ndarray, kt: Optional[int] = None):
    """A Pi0 = Qhat R, R^T Pi1 = Phat L^T; returns (Q, L, P, piv0, piv1) with
    A = Q L P^T.  ``kt`` (optional): the truncated pivoted QLP, the first CPQR
    stopped after kt steps (R is kt x n) and the second one on its kt x n R;
    then Q L P^T = Qhat_kt R Pi0^T, A's projection on the first kt columns of
    Qhat."""
    A = np.asarray(A, dtype=np.float64)
    f0 = cpqr(A, steps=kt)
    f1 = cpqr(f0.R.T)
    Q = f0.Q[:, f1.perm]
    P = _rows_by_perm(f0.perm, f1.Q)
    return Q, f1.R.T, P, f0.perm, f1.perm


# ---------------------------------------------------------------------------
# error measures
# ---------------------------------------------------------------------------
def lvalue_abs_err(lvals: np.ndarray, sigma: np.ndarray, k: int) -> float:
    """Section 5: err = max_{j<=k} |sigma_j(A) - |L_jj||."""
    return float(np.max(np.abs(sigma[:k] - np.abs(lvals[:k]))))


def reconstruction_rel_err(A: np.ndarray, r: QLPResult) -> float:
    """||A - Q T P^T||_F / ||A||_F."""
    return float(np.linalg.norm(A - r.Q @ r.T @ r.P.T) / np.linalg.norm(A))
