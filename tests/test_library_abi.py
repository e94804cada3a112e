"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/rqlp.h declares, and rejects invalid arguments
with LAPACK-style negative indices before touching the device."""
import ctypes
import os
import re

import pytest

import paper_1811_09334_amd as rq
from paper_1811_09334_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rqlp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rqlp_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("librqlp.so is not built (run __graft_entry__.build())")
    return rq.load()


def test_every_declared_symbol_is_exported_and_bound(lib):
    names = _declared()
    assert "rqlp_factor" in names and "rqlp_cpqr" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} has no Python binding"
    assert set(_lib.SIGNATURES) == set(names)


def test_version_and_status_strings(lib):
    assert _lib.rqlp_version().startswith("rqlp-gfx950")
    assert _lib.rqlp_status_string(0) == "success"
    assert "workspace" in _lib.rqlp_status_string(-1000)
    assert "invalid argument" in _lib.rqlp_status_string(-4)


def _factor_status(**kw):
    a = dict(A=1, lda=100, m=100, n=50, k=5, p=3, q=0, d=0, b=0, precision=0, seed=0, Omega=None, ldo=50,
             Q=1, ldq=100, T=1, ldt=8, P=1, ldp=50, piv0=None, piv1=None, lvals=None, info=None, uplo=None,
             work=1, work_bytes=0, stream=None)
    a.update(kw)
    return _lib.rqlp_factor(*a.values())


@pytest.mark.parametrize("kw,code", [
    (dict(A=None), -1), (dict(lda=99), -2), (dict(m=0), -3), (dict(n=101), -4), (dict(n=0), -4),
    (dict(k=1), -5), (dict(p=1), -6), (dict(k=48, p=3), -6), (dict(q=-1), -7), (dict(d=-1), -8),
    (dict(b=-1), -9), (dict(b=4, d=2), -9), (dict(precision=7), -10), (dict(Omega=1, ldo=49), -13),
    (dict(Q=None), -14), (dict(ldq=99), -15), (dict(T=None), -16), (dict(ldt=7), -17), (dict(P=None), -18),
    (dict(ldp=49), -19), (dict(work=None), -25),
])
def test_factor_rejects_invalid_arguments(lib, kw, code):
    assert _factor_status(**kw) == code


def test_workspace_too_small_is_reported(lib):
    assert _factor_status(work_bytes=16) == -1000


def test_workspace_size_query(lib):
    b1 = rq.workspace_size(1000, 500, 20, 5)
    b2 = rq.workspace_size(20000, 10000, 200, 10, 1, 2)
    assert 0 < b1 < b2
    # dominated by the m x l panels, the reduced matrix and the split-K partial sums
    assert b2 >= 8 * (2 * 20000 * 210 + 3 * 10000 * 210)
    with pytest.raises(rq.RQLPError):
        rq.workspace_size(10, 20, 2, 2)


def test_building_block_argument_checks(lib):
    assert _lib.rqlp_sketch(None, 10, 10, 5, 1, 5, 3, 1, 10, 0, None, 0, None) == -1
    assert _lib.rqlp_sketch(1, 9, 10, 5, 1, 5, 3, 1, 10, 0, None, 0, None) == -2
    assert _lib.rqlp_project(1, 10, 10, 5, 1, 10, 3, 1, 2, 0, None, 0, None) == -9
    assert _lib.rqlp_cpqr(1, 3, 4, 6, None, None, 0, None, 0, None, 0, None, None, 0, None) == -2
    assert _lib.rqlp_orthonormalize(1, 10, 10, 11, 1, 10, None, 0, None, None, 0, None) == -4
    assert _lib.rqlp_generate_omega(10, 3, 0, 9, 1, 10, None) == -4


def test_encode_argument_checks(lib):
    # (A, lda, m, n, precision, form, Ahi, Alo, colexp, gexp, stream)
    assert _lib.rqlp_encode(1, 9, 10, 5, 2, 0, 1, None, None, None, None) == -2
    assert _lib.rqlp_encode(1, 10, 10, 5, 0, 0, 1, None, None, None, None) == -5     # not a mixed type
    assert _lib.rqlp_encode(1, 10, 10, 5, 2, 2, 1, None, None, None, None) == -6     # unknown form
    assert _lib.rqlp_encode(None, 10, 10, 5, 2, 0, 1, None, None, None, None) == -1
    assert _lib.rqlp_encode(1, 10, 10, 5, 2, 0, None, None, None, None, None) == -7
    assert _lib.rqlp_encode(1, 10, 10, 5, 2, 0, 1, 1, None, None, None) == -8        # lo only for bf16x3
    assert _lib.rqlp_encode(1, 10, 10, 5, 4, 1, 1, None, None, None, None) == -8
    assert _lib.rqlp_encode(1, 10, 10, 5, 3, 0, 1, None, None, 1, None) == -9        # fp16 needs colexp
    assert _lib.rqlp_encode(1, 10, 10, 5, 3, 0, 1, None, 1, None, None) == -10       # ... and gexp
    assert _lib.rqlp_encode(1, 10, 0, 5, 2, 0, None, None, None, None, None) == 0    # empty: nothing to do
    # (Ahi, Alo, colexp, gexp, m, n, V, ldv, c, B, ldb, precision, work, bytes, stream)
    assert _lib.rqlp_project_encoded(1, None, None, None, 10, 5, 1, 9, 3, 1, 3, 2, None, 0, None) == -8
    assert _lib.rqlp_project_encoded(1, None, None, None, 10, 5, 1, 10, 3, 1, 2, 2, None, 0, None) == -11
    assert _lib.rqlp_project_encoded(1, None, None, None, 10, 5, 1, 10, 3, 1, 3, 1, None, 0, None) == -12
    assert _lib.rqlp_project_encoded(1, None, None, None, 10, 5, 1, 10, 3, 1, 3, 3, None, 0, None) == -3
    assert _lib.rqlp_project_encoded(1, 1, None, None, 10, 5, 1, 10, 3, 1, 3, 2, None, 0, None) == -2
    assert _lib.rqlp_project_encoded(1, None, None, None, 10, 5, None, 10, 3, 1, 3, 2, None, 0, None) == -7
    assert _lib.rqlp_project_encoded(1, None, None, None, 10, 5, 1, 10, 3, None, 3, 2, None, 0, None) == -10
    assert _lib.rqlp_project_encoded(1, None, None, None, 10, 0, 1, 10, 3, None, 3, 2, None, 0, None) == 0
    assert _lib.rqlp_project_encoded(1, None, None, None, 10, 5, 1, 10, 3, 1, 3, 2, None, 0, None) == -1000
    # (Ahi, Alo, colexp, gexp, m, n, X, ldx, c, Y, ldy, precision, work, bytes, stream)
    assert _lib.rqlp_sketch_encoded(1, None, None, None, 10, 5, 1, 4, 3, 1, 10, 2, None, 0, None) == -8
    assert _lib.rqlp_sketch_encoded(1, None, None, None, 10, 5, 1, 5, 3, 1, 9, 2, None, 0, None) == -11
    assert _lib.rqlp_sketch_encoded(1, None, 1, None, 10, 5, 1, 5, 3, 1, 10, 3, None, 0, None) == -4
    assert _lib.rqlp_sketch_encoded(1, None, None, None, 10, 5, 1, 5, 3, 1, 10, 2, None, 0, None) == -1000


def test_encoded_sizes(lib):
    # whole 16 x 32 blocks: rows padded to 16, k to 32
    assert _lib.rqlp_encoded_elems(100, 40, 0) == 48 * 128          # A^T: 40 rows, k = 100
    assert _lib.rqlp_encoded_elems(100, 40, 1) == 112 * 64          # A: 100 rows, k = 40
    assert _lib.rqlp_encoded_elems(0, 40, 1) == 0
    with pytest.raises(rq.RQLPError):
        _lib.rqlp_encoded_elems(10, 10, 5)


def test_mixed_workspace_holds_the_16bit_copies(lib):
    m, n, k, p = 32768, 16384, 256, 16
    b = rq.workspace_size(m, n, k, p, 2, 2, 0, "bf16")
    assert b >= 2 * 2 * m * n                       # column- and row-major bfloat16 copies of A
    assert rq.workspace_size(m, n, k, p, 2, 2, 0, "bf16x3") >= b + 2 * 2 * m * n


def test_unsupported_combinations_are_reported(lib):
    assert _factor_status(b=4) == -1000              # block RQLP is supported: only the workspace is short


def _backward_status(**kw):
    a = dict(A=1, lda=100, m=100, n=50, k=5, p=3, q=0, d=0, b=0, precision=0, seed=0, Omega=None, ldo=50,
             piv0=1, piv1=1, dT=1, lddt=8, dQ=None, lddq=100, dP=None, lddp=50, saved=None, dA=1, ldda=100,
             info=None, work=1, work_bytes=0, stream=None)
    a.update(kw)
    return _lib.rqlp_backward(*a.values())


@pytest.mark.parametrize("kw,code", [
    (dict(A=None), -1), (dict(lda=99), -2), (dict(m=0), -3), (dict(n=101), -4), (dict(k=1), -5), (dict(p=1), -6),
    (dict(q=-1), -7), (dict(d=-1), -8), (dict(b=-1), -9), (dict(precision=9), -10), (dict(Omega=1, ldo=49), -13),
    (dict(piv0=None), -14), (dict(piv1=None), -15), (dict(dT=None), -16), (dict(lddt=7), -17),
    (dict(dQ=1, lddq=99), -19), (dict(dP=1, lddp=49), -21), (dict(dA=None), -23), (dict(ldda=99), -24),
    (dict(work=None), -26),
    (dict(d=1), -1002), (dict(b=4), -1002), (dict(precision=2), -1002), (dict(dQ=1), -1002), (dict(saved=1), -1002),
    (dict(work_bytes=16), -1000),
])
def test_backward_rejects_invalid_or_unsupported_arguments(lib, kw, code):
    assert _backward_status(**kw) == code


def test_backward_workspace_query(lib):
    b = rq._lib.rqlp_backward_workspace_size(16384, 4096, 128, 8, 1, 0, 0, 1)
    assert b >= 4 * (16384 + 4096) * 4 * 136          # the two (2q + 2) l panels
    with pytest.raises(rq.RQLPError):
        rq._lib.rqlp_backward_workspace_size(100, 50, 5, 3, 0, 1, 0, 0)


def _autorank_status(**kw):
    import ctypes as ct
    a = dict(A=1, lda=100, m=100, n=50, lmax=20, b=8, q=0, eps=1e-3, precision=0, seed=0, Omega=None, ldo=50,
             Q=1, ldq=100, T=1, ldt=20, P=1, ldp=50, piv0=None, piv1=None, lvals=None, info=None,
             rank=ct.byref(ct.c_int64(0)), err2=None, work=1, work_bytes=0, stream=None)
    a.update(kw)
    return _lib.rqlp_factor_autorank(*a.values())


@pytest.mark.parametrize("kw,code", [
    (dict(A=None), -1), (dict(lda=99), -2), (dict(m=0), -3), (dict(n=101), -4), (dict(lmax=0), -5),
    (dict(lmax=51), -5), (dict(b=0), -6), (dict(q=-1), -7), (dict(eps=-1.0), -8), (dict(eps=float("nan")), -8),
    (dict(precision=9), -9), (dict(Omega=1, ldo=49), -12), (dict(Q=None), -13), (dict(ldq=99), -14),
    (dict(T=None), -15), (dict(ldt=19), -16), (dict(P=None), -17), (dict(ldp=49), -18), (dict(rank=None), -23),
    (dict(work=None), -25),
])
def test_autorank_argument_errors(lib, kw, code):
    assert _autorank_status(**kw) == code


def test_autorank_workspace_query(lib):
    assert _lib.rqlp_autorank_workspace_size(1000, 500, 64, 16, 1, 0) > 0
    with pytest.raises(_lib.RQLPError):
        _lib.rqlp_autorank_workspace_size(1000, 500, 501, 16, 1, 0)


@pytest.mark.parametrize("kw,code", [
    (dict(A=None), -1), (dict(lda=99), -2), (dict(m=0), -3), (dict(n=0), -4), (dict(kt=0), -5), (dict(kt=51), -5),
    (dict(Q=None), -6), (dict(ldq=99), -7), (dict(T=None), -8), (dict(ldt=19), -9), (dict(P=None), -10),
    (dict(ldp=49), -11), (dict(work=None), -16), (dict(m=7000, lda=7000, ldq=7000), -1002),
])
def test_qlp_argument_errors(lib, kw, code):
    a = dict(A=1, lda=100, m=100, n=50, kt=20, Q=1, ldq=100, T=1, ldt=20, P=1, ldp=50, piv0=None, piv1=None,
             lvals=None, info=None, work=1, work_bytes=0, stream=None)
    a.update(kw)
    assert _lib.rqlp_qlp(*a.values()) == code
