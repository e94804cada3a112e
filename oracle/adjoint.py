"""Reference gradient of the randomized QLP L-values with frozen pivots.

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.

The L-values are differentiable functions of A once the pivot sequences of
the two column-pivoted QRs are frozen (any fixed pivot order still gives a
valid QLP, Section 1, and the method is piecewise smooth between pivot
changes).  This module rebuilds the whole pipeline of Algorithm 2.1 / 2.2 --
range finder with q subspace iterations, B = V^T A, the QR of B Pi0, the
second factorisation of R0^T -- from PyTorch CPU operations in FP64, each QR
with a non-negative diagonal (torch.linalg.qr, reduced mode, signs fixed
afterwards), and differentiates it with autograd.  The cotangent is a
triangular dT (the loss <dT, T>); the weighted L-value loss
sum_{j < k} w_j T_jj is dT = diag(w, 0).

Pinned by central finite differences of the NumPy oracle (oracle.rqlp,
Householder QR written out by hand), which shares no code with this module.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np


def _torch():
    import torch
    return torch


def _qr_pos(X):
    """Thin QR with diag(R) >= 0 (the unique factorisation for full rank)."""
    torch = _torch()
    Q, R = torch.linalg.qr(X, mode="reduced")
    s = torch.sign(torch.diagonal(R))
    s = torch.where(s == 0, torch.ones_like(s), s)
    return Q * s[None, :], R * s[:, None]


def _full_perm(piv: Sequence[int], n: int) -> np.ndarray:
    """The given leading pivots followed by the remaining indices in order (the
    order of the non-pivot columns does not change any triangular factor)."""
    piv = np.asarray(piv, dtype=np.int64)
    rest = np.setdiff1d(np.arange(n), piv, assume_unique=False)
    return np.concatenate([piv, rest])


def t_factor_torch(A, Omega, k: int, p: int, q: int, d: int, piv0: Sequence[int],
                   piv1: Optional[Sequence[int]] = None):
    """The triangular factor T of RQLP (d = 0) / ERQLP (d >= 1) as a torch
    function of A (FP64 tensors), with the pivots frozen.  Returns (T, uplo)."""
    torch = _torch()
    l = k + p
    m, n = A.shape
    Y = A @ Omega
    V, _ = _qr_pos(Y)
    for _ in range(q):
        Z = A.transpose(0, 1) @ V
        W, _ = _qr_pos(Z)
        Y = A @ W
        V, _ = _qr_pos(Y)
    B = V.transpose(0, 1) @ A                       # l x n
    perm0 = torch.as_tensor(_full_perm(piv0, n))
    _, R0 = _qr_pos(B[:, perm0])                    # B Pi0 = Q0 R0 (wide)
    if d == 0:
        perm1 = torch.as_tensor(np.asarray(piv1, dtype=np.int64))
        _, Lt = _qr_pos(R0.transpose(0, 1)[:, perm1])  # R0^T Pi1 = Q1 L^T
        return Lt.transpose(0, 1), "L"
    Rprev = R0
    for _ in range(d):
        _, Rprev = _qr_pos(Rprev.transpose(0, 1))   # R(i-1)^T = Q(i) R(i)
    if d % 2 == 1:
        return Rprev.transpose(0, 1), "L"
    return Rprev, "U"


def weights_cotangent(w: np.ndarray, l: int) -> np.ndarray:
    """dT for the loss sum_{j < k} w_j T_jj (k = len(w))."""
    dT = np.zeros((l, l))
    dT[np.arange(len(w)), np.arange(len(w))] = w
    return dT


def vjp(A: np.ndarray, Omega: np.ndarray, k: int, p: int, q: int, d: int, piv0: Sequence[int],
        piv1: Optional[Sequence[int]], dT: np.ndarray):
    """dA = d <dT, T(A)> / dA (FP64, CPU autograd).  Returns (dA, T)."""
    torch = _torch()
    At = torch.tensor(np.asarray(A, dtype=np.float64), requires_grad=True)
    Om = torch.tensor(np.asarray(Omega, dtype=np.float64))
    T, _ = t_factor_torch(At, Om, k, p, q, d, piv0, piv1)
    loss = (torch.tensor(np.asarray(dT, dtype=np.float64)) * T).sum()
    loss.backward()
    return At.grad.numpy().copy(), T.detach().numpy().copy()


def directional_fd(A: np.ndarray, Omega: np.ndarray, k: int, p: int, q: int, d: int, piv0: Sequence[int],
                   piv1: Optional[Sequence[int]], dT: np.ndarray, E: np.ndarray, h: float) -> float:
    """Central difference (f(A + h E) - f(A - h E)) / (2 h) of f = <dT, T>,
    with T from the NumPy oracle run on the frozen pivots."""
    from .rqlp import rqlp

    def f(X):
        r = rqlp(X, Omega, k, p, q=q, d=d, piv0=piv0, piv1=piv1 if d == 0 else None)
        return float(np.sum(dT * r.T))

    return (f(A + h * E) - f(A - h * E)) / (2.0 * h)
