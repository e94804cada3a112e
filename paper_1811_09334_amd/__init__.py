"""MI355X-native randomized QLP (RQLP / ERQLP / block RQLP).

``A ~= Q T P^T`` with Q (m x l), P (n x l) column-orthonormal and T (l x l)
triangular whose diagonal are the L-values (Wu & Xiang, Algorithms 2.1, 2.2,
4.1).  Every step runs in the gfx950 kernels of ``librqlp.so``; this module
only allocates device memory with torch, picks the current stream and
forwards pointers through the C ABI (``_lib``).  When the library is missing,
calls raise: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

from . import inputs  # noqa: F401
from ._lib import RQLPError, check, load  # noqa: F401
from . import _lib

PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "fp16": 3, "bf16x3": 4}
INFO_FLAGS = {"cholqr_shifted": 0x1, "rank_deficient": 0x2, "nonfinite": 0x4, "barrier_timeout": 0x8,
              "chol_failed": 0x10, "bad_pivots": 0x20, "not_converged": 0x40}


def _torch():
    import torch
    return torch


def _prec(precision) -> int:
    if isinstance(precision, int):
        return precision
    return PRECISIONS[precision]


def _elem_dtype(prec: int):
    torch = _torch()
    return torch.float64 if prec == 0 else torch.float32


def empty_colmajor(rows: int, cols: int, dtype, device):
    """Uninitialised column-major (rows x cols) tensor: stride (1, rows)."""
    torch = _torch()
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def colmajor(t):
    """``t`` itself when it is already column-major (stride(0) == 1), else a column-major copy."""
    if t.dim() != 2:
        raise ValueError("expected a matrix")
    rows, cols = t.shape
    if t.stride(0) == 1 and (cols <= 1 or t.stride(1) >= max(rows, 1)):
        return t
    return t.t().contiguous().t()


def ld(t) -> int:
    rows, cols = t.shape
    return max(int(t.stride(1)) if cols > 1 else rows, 1)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(device=None) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


@dataclass
class Factorization:
    Q: "object"        # m x l (column-major)
    T: "object"        # l x l, float64
    P: "object"        # n x l
    piv0: "object"     # l int64
    piv1: "object"     # l int64
    lvals: "object"    # l float64
    info: "object"     # 1 int32 (device)
    uplo: str

    def info_flags(self) -> dict:
        v = int(self.info.item())
        return {k: bool(v & b) for k, b in INFO_FLAGS.items()}


def workspace_size(m, n, k, p, q=0, d=0, b=0, precision="f64") -> int:
    return _lib.rqlp_workspace_size(m, n, k, p, q, d, b, _prec(precision))


def factor(A, k: int, p: int, q: int = 0, d: int = 0, b: int = 0, precision="f64", seed: int = 0,
           Omega=None, work=None) -> Factorization:
    """Randomized QLP of the device matrix ``A`` (m x n) through ``rqlp_factor``.

    ``A`` (and ``Omega`` if given, n x (k+p)) must be float64 for 'f64' and
    float32 otherwise; column-major layouts are used as they are, other
    layouts are copied once to column-major."""
    torch = _torch()
    load()
    prec = _prec(precision)
    dt = _elem_dtype(prec)
    if A.dtype != dt:
        raise TypeError(f"A must be {dt} for precision {precision}")
    A = colmajor(A)
    m, n = A.shape
    l = k + p
    dev = A.device
    if Omega is not None:
        if Omega.dtype != dt or tuple(Omega.shape) != (n, l):
            raise ValueError("Omega must be n x (k+p) with the element type of A")
        Omega = colmajor(Omega)
    Q = empty_colmajor(m, l, dt, dev)
    T = empty_colmajor(l, l, torch.float64, dev)
    P = empty_colmajor(n, l, dt, dev)
    piv0 = torch.empty(l, dtype=torch.int64, device=dev)
    piv1 = torch.empty(l, dtype=torch.int64, device=dev)
    lv = torch.empty(l, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = workspace_size(m, n, k, p, q, d, b, prec)
    if work is None or work.numel() < nbytes:
        work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    uplo = ctypes.c_char(b"?")
    st = _lib.rqlp_factor(A.data_ptr(), ld(A), m, n, k, p, q, d, b, prec, seed,
                          _ptr(Omega), ld(Omega) if Omega is not None else max(n, 1),
                          Q.data_ptr(), ld(Q), T.data_ptr(), ld(T), P.data_ptr(), ld(P),
                          piv0.data_ptr(), piv1.data_ptr(), lv.data_ptr(), info.data_ptr(),
                          ctypes.byref(uplo), work.data_ptr(), work.numel(), _stream(dev))
    check("rqlp_factor", st)
    return Factorization(Q=Q, T=T, P=P, piv0=piv0, piv1=piv1, lvals=lv, info=info, uplo=uplo.value.decode())


def factor_autorank(A, lmax: int, b: int, eps: float, q: int = 0, precision="f64", seed: int = 0, Omega=None,
                    work=None):
    """Auto-rank randomized QLP of the device matrix ``A`` through
    ``rqlp_factor_autorank``: returns (Factorization with lmax columns, rank,
    err2); the columns past ``rank`` are zero."""
    torch = _torch()
    load()
    prec = _prec(precision)
    dt = _elem_dtype(prec)
    if A.dtype != dt:
        raise TypeError(f"A must be {dt} for precision {precision}")
    A = colmajor(A)
    m, n = A.shape
    dev = A.device
    if Omega is not None:
        if Omega.dtype != dt or tuple(Omega.shape) != (n, lmax):
            raise ValueError("Omega must be n x lmax with the element type of A")
        Omega = colmajor(Omega)
    Q = empty_colmajor(m, lmax, dt, dev)
    T = empty_colmajor(lmax, lmax, torch.float64, dev)
    P = empty_colmajor(n, lmax, dt, dev)
    piv0 = torch.empty(lmax, dtype=torch.int64, device=dev)
    piv1 = torch.empty(lmax, dtype=torch.int64, device=dev)
    lv = torch.empty(lmax, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = _lib.rqlp_autorank_workspace_size(m, n, lmax, b, q, prec)
    if work is None or work.numel() < nbytes:
        work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    rank = ctypes.c_int64(0)
    err2 = ctypes.c_double(0.0)
    st = _lib.rqlp_factor_autorank(A.data_ptr(), ld(A), m, n, lmax, b, q, float(eps), prec, seed,
                                   _ptr(Omega), ld(Omega) if Omega is not None else max(n, 1),
                                   Q.data_ptr(), ld(Q), T.data_ptr(), ld(T), P.data_ptr(), ld(P),
                                   piv0.data_ptr(), piv1.data_ptr(), lv.data_ptr(), info.data_ptr(),
                                   ctypes.byref(rank), ctypes.byref(err2), work.data_ptr(), work.numel(),
                                   _stream(dev))
    check("rqlp_factor_autorank", st)
    f = Factorization(Q=Q, T=T, P=P, piv0=piv0, piv1=piv1, lvals=lv, info=info, uplo="L")
    return f, rank.value, err2.value


def pivoted_qlp(A, kt: int, work=None) -> Factorization:
    """Deterministic truncated pivoted QLP (kt steps) of the FP64 device
    matrix ``A`` through ``rqlp_qlp``."""
    torch = _torch()
    load()
    if A.dtype != torch.float64:
        raise TypeError("A must be float64")
    A = colmajor(A)
    m, n = A.shape
    dev = A.device
    Q = empty_colmajor(m, kt, torch.float64, dev)
    T = empty_colmajor(kt, kt, torch.float64, dev)
    P = empty_colmajor(n, kt, torch.float64, dev)
    piv0 = torch.empty(kt, dtype=torch.int64, device=dev)
    piv1 = torch.empty(kt, dtype=torch.int64, device=dev)
    lv = torch.empty(kt, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = _lib.rqlp_qlp_workspace_size(m, n, kt)
    if work is None or work.numel() < nbytes:
        work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    st = _lib.rqlp_qlp(A.data_ptr(), ld(A), m, n, kt, Q.data_ptr(), ld(Q), T.data_ptr(), ld(T), P.data_ptr(), ld(P),
                       piv0.data_ptr(), piv1.data_ptr(), lv.data_ptr(), info.data_ptr(), work.data_ptr(),
                       work.numel(), _stream(dev))
    check("rqlp_qlp", st)
    return Factorization(Q=Q, T=T, P=P, piv0=piv0, piv1=piv1, lvals=lv, info=info, uplo="L")


def backward(A, k: int, p: int, piv0, piv1, dT, q: int = 0, d: int = 0, b: int = 0, precision=None, seed: int = 0,
             Omega=None, work=None):
    """dA = d<dT, T>/dA with the pivots frozen, through ``rqlp_backward``.

    ``A``, ``q``, ``d``, ``b``, ``precision``, ``seed`` and ``Omega`` as in the
    forward ``factor`` call that produced ``piv0`` / ``piv1``; ``dT`` is an
    l x l float64 device tensor.  Returns (dA, info)."""
    torch = _torch()
    load()
    if precision is None:
        precision = "f64" if A.dtype == torch.float64 else "f32"
    prec = _prec(precision)
    A = colmajor(A)
    m, n = A.shape
    l = k + p
    dev = A.device
    dT = colmajor(dT.to(torch.float64))
    if Omega is not None:
        Omega = colmajor(Omega)
    dA = empty_colmajor(m, n, A.dtype, dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = _lib.rqlp_backward_workspace_size(m, n, k, p, q, d, b, prec)
    if work is None or work.numel() < nbytes:
        work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    piv0 = piv0.to(torch.int64).contiguous()
    piv1 = piv1.to(torch.int64).contiguous()
    st = _lib.rqlp_backward(A.data_ptr(), ld(A), m, n, k, p, q, d, b, prec, seed, _ptr(Omega),
                            ld(Omega) if Omega is not None else max(n, 1), piv0.data_ptr(), piv1.data_ptr(),
                            dT.data_ptr(), ld(dT), None, max(m, 1), None, max(n, 1), None, dA.data_ptr(), ld(dA),
                            info.data_ptr(), work.data_ptr(), work.numel(), _stream(dev))
    check("rqlp_backward", st)
    return dA, info


def _autograd_function():
    torch = _torch()

    class RQLPFunction(torch.autograd.Function):
        """T (differentiable), Q, P of the randomized QLP; the backward calls
        rqlp_backward with the forward's pivots frozen (Q and P carry no
        gradient)."""

        @staticmethod
        def forward(ctx, A, k, p, q, d, precision, seed, Omega):
            f = factor(A.detach(), k, p, q=q, d=d, precision=precision, seed=seed, Omega=Omega)
            ctx.save_for_backward(A, f.piv0, f.piv1)
            ctx.args = (k, p, q, d, precision, seed, Omega)
            ctx.mark_non_differentiable(f.Q, f.P)
            return f.T, f.Q, f.P

        @staticmethod
        def backward(ctx, dT, dQ, dP):
            A, piv0, piv1 = ctx.saved_tensors
            k, p, q, d, precision, seed, Omega = ctx.args
            if dT is None:
                return (None,) * 8
            dA, _ = backward(A.detach(), k, p, piv0, piv1, dT, q=q, d=d, precision=precision, seed=seed,
                             Omega=Omega)
            return dA, None, None, None, None, None, None, None

    return RQLPFunction


_RQLP_FN = None


def rqlp(A, k: int, p: int, q: int = 0, d: int = 0, precision=None, seed: int = 0, Omega=None):
    """Differentiable randomized QLP: returns (T, Q, P) with T differentiable
    with respect to A (pivots frozen at the forward's choice)."""
    global _RQLP_FN
    torch = _torch()
    if _RQLP_FN is None:
        _RQLP_FN = _autograd_function()
    if precision is None:
        precision = "f64" if A.dtype == torch.float64 else "f32"
    return _RQLP_FN.apply(A, k, p, q, d, precision, seed, Omega)


def generate_omega(n: int, l: int, seed: int, precision="f64", device="cuda"):
    """The library's Philox4x32-10 / Box-Muller test matrix (n x l, column-major)."""
    prec = _prec(precision)
    out = empty_colmajor(n, l, _elem_dtype(prec), device)
    check("rqlp_generate_omega", _lib.rqlp_generate_omega(n, l, seed, prec, out.data_ptr(), ld(out),
                                                          _stream(out.device)))
    return out


def sketch(A, X, precision=None):
    """Y = A X through ``rqlp_sketch``."""
    torch = _torch()
    prec = _prec(precision if precision is not None else ("f64" if A.dtype == torch.float64 else "f32"))
    A, X = colmajor(A), colmajor(X)
    m, n = A.shape
    c = X.shape[1]
    Y = empty_colmajor(m, c, A.dtype, A.device)
    nb = _lib.rqlp_gemm_workspace(m, n, c, prec)
    work = torch.empty(nb, dtype=torch.uint8, device=A.device)
    check("rqlp_sketch", _lib.rqlp_sketch(A.data_ptr(), ld(A), m, n, X.data_ptr(), ld(X), c, Y.data_ptr(), ld(Y),
                                          prec, work.data_ptr(), nb, _stream(A.device)))
    return Y


def project(A, V, precision=None):
    """B = V^T A through ``rqlp_project``."""
    torch = _torch()
    prec = _prec(precision if precision is not None else ("f64" if A.dtype == torch.float64 else "f32"))
    A, V = colmajor(A), colmajor(V)
    m, n = A.shape
    c = V.shape[1]
    B = empty_colmajor(c, n, A.dtype, A.device)
    nb = _lib.rqlp_gemm_workspace(m, n, c, prec)
    work = torch.empty(nb, dtype=torch.uint8, device=A.device)
    check("rqlp_project", _lib.rqlp_project(A.data_ptr(), ld(A), m, n, V.data_ptr(), ld(V), c, B.data_ptr(),
                                            ld(B), prec, work.data_ptr(), nb, _stream(A.device)))
    return B


ENC_FORMS = {"cols": 0, "rows": 1}


@dataclass
class Encoded:
    """A encoded for the 16-bit MFMA products (``rqlp_encode``): flat fragment-tiled
    copies (form "cols": the operand A^T of B = V^T A; "rows": the operand A of Y = A X)."""
    hi: "object"          # uint16 bit patterns as int16, rqlp_encoded_elems entries
    lo: "object"          # bf16x3 remainders or None
    colexp: "object"      # int32 per-column exponents (FP16) or None
    gexp: "object"        # int32 max exponent (FP16) or None
    m: int
    n: int
    precision: int
    form: str


def encode(A, precision="bf16", form: str = "cols") -> Encoded:
    """16-bit encoding of the FP32 device matrix A through ``rqlp_encode``."""
    torch = _torch()
    prec = _prec(precision)
    A = colmajor(A)
    m, n = A.shape
    f = ENC_FORMS[form]
    ne = _lib.rqlp_encoded_elems(m, n, f)
    hi = torch.empty(max(ne, 1), dtype=torch.int16, device=A.device)
    lo = torch.empty(max(ne, 1), dtype=torch.int16, device=A.device) if prec == PRECISIONS["bf16x3"] else None
    fp16 = prec == PRECISIONS["fp16"]
    colexp = torch.empty(max(n, 1), dtype=torch.int32, device=A.device) if fp16 else None
    gexp = torch.empty(1, dtype=torch.int32, device=A.device) if fp16 else None
    check("rqlp_encode", _lib.rqlp_encode(A.data_ptr(), ld(A), m, n, prec, f, hi.data_ptr(), _ptr(lo),
                                          _ptr(colexp), _ptr(gexp), _stream(A.device)))
    return Encoded(hi[:ne], None if lo is None else lo[:ne], colexp, gexp, m, n, prec, form)


def project_encoded(E: Encoded, V, B=None, work=None):
    """B = V^T A through ``rqlp_project_encoded`` with A pre-encoded (form "cols")."""
    torch = _torch()
    if E.form != "cols":
        raise ValueError("project_encoded needs the encoding of form 'cols'")
    V = colmajor(V)
    c = V.shape[1]
    if B is None:
        B = empty_colmajor(c, E.n, torch.float32, V.device)
    nb = _lib.rqlp_gemm_workspace(E.m, E.n, c, E.precision)
    if work is None or work.numel() < nb:
        work = torch.empty(nb, dtype=torch.uint8, device=V.device)
    check("rqlp_project_encoded", _lib.rqlp_project_encoded(E.hi.data_ptr(), _ptr(E.lo), _ptr(E.colexp),
                                                            _ptr(E.gexp), E.m, E.n, V.data_ptr(), ld(V), c,
                                                            B.data_ptr(), ld(B), E.precision, work.data_ptr(),
                                                            work.numel(), _stream(V.device)))
    return B


def sketch_encoded(E: Encoded, X, Y=None, work=None):
    """Y = A X through ``rqlp_sketch_encoded`` with A pre-encoded (form "rows")."""
    torch = _torch()
    if E.form != "rows":
        raise ValueError("sketch_encoded needs the encoding of form 'rows'")
    X = colmajor(X)
    c = X.shape[1]
    if Y is None:
        Y = empty_colmajor(E.m, c, torch.float32, X.device)
    nb = _lib.rqlp_gemm_workspace(E.m, E.n, c, E.precision)
    if work is None or work.numel() < nb:
        work = torch.empty(nb, dtype=torch.uint8, device=X.device)
    check("rqlp_sketch_encoded", _lib.rqlp_sketch_encoded(E.hi.data_ptr(), _ptr(E.lo), _ptr(E.colexp),
                                                          _ptr(E.gexp), E.m, E.n, X.data_ptr(), ld(X), c,
                                                          Y.data_ptr(), ld(Y), E.precision, work.data_ptr(),
                                                          work.numel(), _stream(X.device)))
    return Y


def orthonormalize(Y, want_r: bool = False):
    """Y = V R with V orthonormal, R upper triangular, by CholeskyQR2 through ``rqlp_orthonormalize`` (FP64)."""
    torch = _torch()
    Y = colmajor(Y)
    m, c = Y.shape
    V = empty_colmajor(m, c, torch.float64, Y.device)
    R = empty_colmajor(c, c, torch.float64, Y.device) if want_r else None
    info = torch.zeros(1, dtype=torch.int32, device=Y.device)
    nb = _lib.rqlp_orthonormalize_workspace(m, c)
    work = torch.empty(nb, dtype=torch.uint8, device=Y.device)
    check("rqlp_orthonormalize", _lib.rqlp_orthonormalize(Y.data_ptr(), ld(Y), m, c, V.data_ptr(), ld(V),
                                                          _ptr(R), ld(R) if R is not None else 1, info.data_ptr(),
                                                          work.data_ptr(), nb, _stream(Y.device)))
    return (V, R, info) if want_r else (V, info)


def cpqr(M):
    """Column-pivoted QR through ``rqlp_cpqr``: returns (piv, R11, Rt, Q, info)."""
    torch = _torch()
    M = colmajor(M)
    rows, cols = M.shape
    kmax = min(rows, cols)
    piv = torch.empty(kmax, dtype=torch.int64, device=M.device)
    R = empty_colmajor(rows, kmax, torch.float64, M.device)
    Rt = empty_colmajor(cols, rows, torch.float64, M.device)
    Q = empty_colmajor(rows, kmax, torch.float64, M.device)
    info = torch.zeros(1, dtype=torch.int32, device=M.device)
    nb = _lib.rqlp_cpqr_workspace(rows, cols)
    work = torch.empty(nb, dtype=torch.uint8, device=M.device)
    check("rqlp_cpqr", _lib.rqlp_cpqr(M.data_ptr(), ld(M), rows, cols, piv.data_ptr(), R.data_ptr(), ld(R),
                                      Rt.data_ptr(), ld(Rt), Q.data_ptr(), ld(Q), info.data_ptr(),
                                      work.data_ptr(), nb, _stream(M.device)))
    return piv, R, Rt, Q, info
