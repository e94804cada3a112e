"""Shared helpers for the GPU parity tests (host <-> device copies and the
pivot-separation rule)."""
import numpy as np

from oracle.qr import cpqr as oracle_cpqr

PIVOT_SEPARATION = 1e-8   # pivots must agree where the top two residual norms differ by more


def to_dev(a, dtype=None):
    """NumPy (any order) -> column-major torch tensor on cuda:0."""
    import torch
    a = np.asarray(a)
    t = torch.from_numpy(np.ascontiguousarray(a.T))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0").t()


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def pivots_valid(M, piv, rel=PIVOT_SEPARATION):
    """Replay the CPQR of M with the given pivots and check each one was a
    maximal residual-norm column up to ``rel``.  Returns (ok, first_bad_step)."""
    f = oracle_cpqr(M, piv=piv, want_q=False, want_trace=True)
    tr = f.trace
    bad = np.flatnonzero(tr[:, 1] < tr[:, 0] * (1.0 - rel))
    return (bad.size == 0, int(bad[0]) if bad.size else -1)


def first_difference(a, b):
    d = np.flatnonzero(np.asarray(a) != np.asarray(b))
    return int(d[0]) if d.size else -1
