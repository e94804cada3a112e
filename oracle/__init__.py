"""CPU oracle for randomized QLP (FP64, NumPy).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import anything from here.  The
product path (the HIP library and its Python binding) never calls it, and
this package imports nothing from the product.

Contents
  qr.py      hand-written Householder QR / column-pivoted QR (Businger-Golub)
  rqlp.py    RQLP (Alg. 2.1), ERQLP (Alg. 2.2), block RQLP (Alg. 4.1),
             auto-rank RQLP (Section 6), Stewart's pivoted QLP (eq. 1.2),
             error measures
  philox.py  Philox4x32-10 + Box-Muller reference for the library's Omega
  adjoint.py reference gradient of sum_j w_j L_jj (frozen pivots) and finite
             differences

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
to closed forms, library routines, invariants, brute force or published
values; none is "parity unpinned" except the absolute values of the paper's
Tables 1-4, whose random matrices are not specified (orderings only).
"""
from .qr import QRResult, cpqr, householder_qr  # noqa: F401
from .rqlp import (QLPResult, autorank_rqlp, brqlp, lvalue_abs_err, orthonormal_basis,  # noqa: F401
                   qlp_reduced, range_finder, reconstruction_rel_err, rqlp, stewart_qlp)
