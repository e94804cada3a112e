"""ctypes binding of ``librqlp.so`` (the C ABI declared in include/rqlp.h).

Marshalling only: every function here forwards integers and device pointers
to the library of the same name; no arithmetic of the method happens in
Python.  ``load()`` raises when the library is missing: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librqlp.so")

# names and signatures exported by include/rqlp.h
SIGNATURES = {
    "rqlp_version": (c_char_p, []),
    "rqlp_status_string": (c_char_p, [c_int]),
    "rqlp_workspace_size": (c_int, [c_int64, c_int64, c_int64, c_int64, c_int, c_int, c_int, c_int,
                                    POINTER(c_size_t)]),
    "rqlp_generate_omega": (c_int, [c_int64, c_int64, c_uint64, c_int, c_void_p, c_int64, c_void_p]),
    "rqlp_factor": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_int64, c_int64, c_int, c_int, c_int, c_int,
                            c_uint64, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                            c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_char), c_void_p, c_size_t,
                            c_void_p]),
    "rqlp_factor_noalloc": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_int64, c_int64, c_int, c_int, c_int,
                                    c_int, c_uint64, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                                    c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_char),
                                    c_void_p]),
    "rqlp_autorank_workspace_size": (c_int, [c_int64, c_int64, c_int64, c_int64, c_int, c_int, POINTER(c_size_t)]),
    "rqlp_factor_autorank": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_int64, c_int64, c_int, c_double, c_int,
                                     c_uint64, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                     c_int64, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_int64),
                                     POINTER(c_double), c_void_p, c_size_t, c_void_p]),
    "rqlp_qlp_workspace_size": (c_int, [c_int64, c_int64, c_int64, POINTER(c_size_t)]),
    "rqlp_qlp": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                         c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "rqlp_backward": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_int64, c_int64, c_int, c_int, c_int, c_int,
                              c_uint64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_int64,
                              c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_size_t,
                              c_void_p]),
    "rqlp_backward_workspace_size": (c_int, [c_int64, c_int64, c_int64, c_int64, c_int, c_int, c_int, c_int,
                                             POINTER(c_size_t)]),
    "rqlp_sketch": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64, c_int64, c_void_p, c_int64,
                            c_int, c_void_p, c_size_t, c_void_p]),
    "rqlp_project": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64, c_int64, c_void_p, c_int64,
                             c_int, c_void_p, c_size_t, c_void_p]),
    "rqlp_gemm_workspace": (c_int, [c_int64, c_int64, c_int64, c_int, POINTER(c_size_t)]),
    "rqlp_encoded_elems": (c_int, [c_int64, c_int64, c_int, POINTER(c_size_t)]),
    "rqlp_encode": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_int, c_int, c_void_p, c_void_p, c_void_p,
                            c_void_p, c_void_p]),
    "rqlp_project_encoded": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_int64,
                                     c_int64, c_void_p, c_int64, c_int, c_void_p, c_size_t, c_void_p]),
    "rqlp_sketch_encoded": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_int64,
                                    c_int64, c_void_p, c_int64, c_int, c_void_p, c_size_t, c_void_p]),
    "rqlp_orthonormalize": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                                    c_void_p, c_void_p, c_size_t, c_void_p]),
    "rqlp_orthonormalize_workspace": (c_int, [c_int64, c_int64, POINTER(c_size_t)]),
    "rqlp_cpqr": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p, c_int64, c_void_p, c_int64,
                          c_void_p, c_int64, c_void_p, c_void_p, c_size_t, c_void_p]),
    "rqlp_cpqr_workspace": (c_int, [c_int64, c_int64, POINTER(c_size_t)]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (once).  Raises RuntimeError when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it first (python -m paper_1811_09334_amd.build_lib)")
    # torch first, so that the library binds to the HIP runtime torch has
    # already brought into the process (the one that owns the tensors it is
    # given): loaded before torch, a factorisation returned RQLP_E_UNSUPPORTED
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class RQLPError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = load().rqlp_status_string(status).decode()
        super().__init__(f"{fn} returned {status}: {msg}")
        self.status = status


def check(fn: str, status: int) -> None:
    if status != 0:
        raise RQLPError(fn, status)


def _call(name, *args):
    return getattr(load(), name)(*args)


def rqlp_version() -> str:
    return _call("rqlp_version").decode()


def rqlp_status_string(status: int) -> str:
    return _call("rqlp_status_string", status).decode()


def rqlp_workspace_size(m, n, k, p, q, d, b, precision) -> int:
    out = c_size_t(0)
    check("rqlp_workspace_size", _call("rqlp_workspace_size", m, n, k, p, q, d, b, precision, ctypes.byref(out)))
    return out.value


def rqlp_generate_omega(n, l, seed, precision, omega_ptr, ldo, stream) -> int:
    return _call("rqlp_generate_omega", n, l, seed, precision, omega_ptr, ldo, stream)


def rqlp_factor(A, lda, m, n, k, p, q, d, b, precision, seed, Omega, ldo, Q, ldq, T, ldt, P, ldp,
                piv0, piv1, lvals, info, uplo, work, work_bytes, stream) -> int:
    return _call("rqlp_factor", A, lda, m, n, k, p, q, d, b, precision, seed, Omega, ldo, Q, ldq, T, ldt, P, ldp,
                 piv0, piv1, lvals, info, uplo, work, work_bytes, stream)


def rqlp_factor_noalloc(A, lda, m, n, k, p, q, d, b, precision, seed, Omega, ldo, Q, ldq, T, ldt, P, ldp,
                        piv0, piv1, lvals, info, uplo, stream) -> int:
    return _call("rqlp_factor_noalloc", A, lda, m, n, k, p, q, d, b, precision, seed, Omega, ldo, Q, ldq, T, ldt,
                 P, ldp, piv0, piv1, lvals, info, uplo, stream)


def rqlp_autorank_workspace_size(m, n, lmax, b, q, precision) -> int:
    out = c_size_t(0)
    check("rqlp_autorank_workspace_size", _call("rqlp_autorank_workspace_size", m, n, lmax, b, q, precision,
                                                ctypes.byref(out)))
    return out.value


def rqlp_factor_autorank(A, lda, m, n, lmax, b, q, eps, precision, seed, Omega, ldo, Q, ldq, T, ldt, P, ldp, piv0,
                         piv1, lvals, info, rank, err2, work, work_bytes, stream) -> int:
    return _call("rqlp_factor_autorank", A, lda, m, n, lmax, b, q, eps, precision, seed, Omega, ldo, Q, ldq, T, ldt,
                 P, ldp, piv0, piv1, lvals, info, rank, err2, work, work_bytes, stream)


def rqlp_qlp_workspace_size(m, n, kt) -> int:
    out = c_size_t(0)
    check("rqlp_qlp_workspace_size", _call("rqlp_qlp_workspace_size", m, n, kt, ctypes.byref(out)))
    return out.value


def rqlp_qlp(A, lda, m, n, kt, Q, ldq, T, ldt, P, ldp, piv0, piv1, lvals, info, work, work_bytes, stream) -> int:
    return _call("rqlp_qlp", A, lda, m, n, kt, Q, ldq, T, ldt, P, ldp, piv0, piv1, lvals, info, work, work_bytes,
                 stream)


def rqlp_backward(A, lda, m, n, k, p, q, d, b, precision, seed, Omega, ldo, piv0, piv1, dT, lddt, dQ, lddq, dP,
                  lddp, saved, dA, ldda, info, work, work_bytes, stream) -> int:
    return _call("rqlp_backward", A, lda, m, n, k, p, q, d, b, precision, seed, Omega, ldo, piv0, piv1, dT, lddt,
                 dQ, lddq, dP, lddp, saved, dA, ldda, info, work, work_bytes, stream)


def rqlp_backward_workspace_size(m, n, k, p, q, d, b, precision) -> int:
    out = c_size_t(0)
    check("rqlp_backward_workspace_size", _call("rqlp_backward_workspace_size", m, n, k, p, q, d, b, precision,
                                                ctypes.byref(out)))
    return out.value


def rqlp_sketch(A, lda, m, n, X, ldx, c, Y, ldy, precision, work, work_bytes, stream) -> int:
    return _call("rqlp_sketch", A, lda, m, n, X, ldx, c, Y, ldy, precision, work, work_bytes, stream)


def rqlp_project(A, lda, m, n, V, ldv, c, B, ldb, precision, work, work_bytes, stream) -> int:
    return _call("rqlp_project", A, lda, m, n, V, ldv, c, B, ldb, precision, work, work_bytes, stream)


def rqlp_gemm_workspace(m, n, c, precision) -> int:
    out = c_size_t(0)
    check("rqlp_gemm_workspace", _call("rqlp_gemm_workspace", m, n, c, precision, ctypes.byref(out)))
    return out.value


def rqlp_encoded_elems(m, n, form) -> int:
    out = c_size_t(0)
    check("rqlp_encoded_elems", _call("rqlp_encoded_elems", m, n, form, ctypes.byref(out)))
    return out.value


def rqlp_encode(A, lda, m, n, precision, form, Ahi, Alo, colexp, gexp, stream) -> int:
    return _call("rqlp_encode", A, lda, m, n, precision, form, Ahi, Alo, colexp, gexp, stream)


def rqlp_project_encoded(Ahi, Alo, colexp, gexp, m, n, V, ldv, c, B, ldb, precision, work, work_bytes,
                         stream) -> int:
    return _call("rqlp_project_encoded", Ahi, Alo, colexp, gexp, m, n, V, ldv, c, B, ldb, precision, work,
                 work_bytes, stream)


def rqlp_sketch_encoded(Ahi, Alo, colexp, gexp, m, n, X, ldx, c, Y, ldy, precision, work, work_bytes,
                        stream) -> int:
    return _call("rqlp_sketch_encoded", Ahi, Alo, colexp, gexp, m, n, X, ldx, c, Y, ldy, precision, work,
                 work_bytes, stream)


def rqlp_orthonormalize(Y, ldy, m, c, V, ldv, R, ldr, info, work, work_bytes, stream) -> int:
    return _call("rqlp_orthonormalize", Y, ldy, m, c, V, ldv, R, ldr, info, work, work_bytes, stream)


def rqlp_orthonormalize_workspace(m, c) -> int:
    out = c_size_t(0)
    check("rqlp_orthonormalize_workspace", _call("rqlp_orthonormalize_workspace", m, c, ctypes.byref(out)))
    return out.value


def rqlp_cpqr(M, ldm, rows, cols, piv, R, ldr, Rt, ldrt, Qm, ldq, info, work, work_bytes, stream) -> int:
    return _call("rqlp_cpqr", M, ldm, rows, cols, piv, R, ldr, Rt, ldrt, Qm, ldq, info, work, work_bytes, stream)


def rqlp_cpqr_workspace(rows, cols) -> int:
    out = c_size_t(0)
    check("rqlp_cpqr_workspace", _call("rqlp_cpqr_workspace", rows, cols, ctypes.byref(out)))
    return out.value
