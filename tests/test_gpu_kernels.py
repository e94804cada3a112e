"""GPU parity of the building blocks (through the C ABI) against the FP64
oracle or plain NumPy products: the Gaussian generator, the skinny MFMA
products, CholeskyQR2 and the column-pivoted QR."""
import numpy as np
import pytest

from oracle.philox import omega_gaussian
from oracle.qr import cpqr as oracle_cpqr
from paper_1811_09334_amd import inputs

from _helpers import first_difference, pivots_valid, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_omega_generator_matches_reference(gpu):
    for n, l, seed in [(500, 25, 2000), (1031, 47, 2**40 + 7), (7, 3, 0)]:
        g = to_np(gpu.generate_omega(n, l, seed, "f64"))
        ref = omega_gaussian(n, l, seed)
        assert g.shape == (n, l)
        assert np.max(np.abs(g - ref)) < 1e-13 * max(1.0, np.abs(ref).max())
    g32 = to_np(gpu.generate_omega(300, 20, 5, "bf16"))
    ref = inputs.round_to_bf16(omega_gaussian(300, 20, 5))
    # same bfloat16 value except where the double sits on a rounding boundary
    assert np.mean(g32 == ref) > 0.999


@pytest.mark.parametrize("m,n,c", [(1000, 500, 25), (777, 333, 47), (4096, 2048, 210), (64, 16, 16),
                                   (130, 70, 3), (5000, 300, 272), (2000, 4000, 120)])
def test_sketch_and_projection_f64(gpu, m, n, c):
    rng = np.random.default_rng(m + n + c)
    A = rng.standard_normal((m, n))
    X = rng.standard_normal((n, c))
    V = rng.standard_normal((m, c))
    Y = to_np(gpu.sketch(to_dev(A), to_dev(X)))
    ref = A @ X
    assert np.max(np.abs(Y - ref)) < 1e-13 * np.sqrt(n) * np.abs(ref).max() + 1e-13
    B = to_np(gpu.project(to_dev(A), to_dev(V)))
    ref = V.T @ A
    assert B.shape == (c, n)
    assert np.max(np.abs(B - ref)) < 1e-13 * np.sqrt(m) * np.abs(ref).max() + 1e-13


@pytest.mark.parametrize("m,n,c", [(1000, 500, 25), (777, 333, 47), (3000, 1000, 136)])
def test_sketch_and_projection_f32(gpu, m, n, c):
    import torch
    rng = np.random.default_rng(7 * m + c)
    A = rng.standard_normal((m, n)).astype(np.float32)
    X = rng.standard_normal((n, c)).astype(np.float32)
    Y = to_np(gpu.sketch(to_dev(A), to_dev(X))).astype(np.float64)
    ref = A.astype(np.float64) @ X.astype(np.float64)
    assert np.max(np.abs(Y - ref)) < 2e-6 * np.sqrt(n) * np.abs(ref).max()
    B = to_np(gpu.project(to_dev(A), to_dev(Y.astype(np.float32)))).astype(np.float64)
    refB = Y.astype(np.float32).astype(np.float64).T @ A.astype(np.float64)
    assert np.max(np.abs(B - refB)) < 2e-6 * np.sqrt(m) * np.abs(refB).max()
    assert torch.cuda.is_available()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_products_on_padded_offset_views(gpu, dtype):
    """Sketch and projection on operands that are views into larger column-major
    arrays (leading dimension above the row count, first element not at the start
    of the allocation), with M, N and K ragged against the 64 x 112 tiles and the
    K stages: interior tiles take the unchecked loads, the edges the checked ones."""
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    tol = 1e-13 if dtype == "f64" else 2e-6
    rng = np.random.default_rng(11)
    for m, n, c, pad, off in [(1000, 517, 130, 7, 3), (2311, 1033, 210, 1, 1), (640, 4101, 47, 64, 5)]:
        A = rng.standard_normal((m, n)).astype(np.float32 if dtype == "f32" else np.float64)
        X = rng.standard_normal((n, c)).astype(A.dtype)
        V = rng.standard_normal((m, c)).astype(A.dtype)
        big = torch.zeros((n, m + pad + off), dtype=tdt, device="cuda:0")
        big[:, off:off + m] = torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda:0")
        Ad = big.t()[off:off + m, :]                    # column-major view, lda = m + pad + off
        assert Ad.stride() == (1, m + pad + off) and Ad.storage_offset() == off
        bigx = torch.zeros((c, n + pad), dtype=tdt, device="cuda:0")
        bigx[:, :n] = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda:0")
        Xd = bigx.t()[:n, :]
        Y = to_np(gpu.sketch(Ad, Xd)).astype(np.float64)
        ref = A.astype(np.float64) @ X.astype(np.float64)
        assert np.max(np.abs(Y - ref)) < tol * np.sqrt(n) * np.abs(ref).max() + tol
        B = to_np(gpu.project(Ad, to_dev(V))).astype(np.float64)
        refB = V.astype(np.float64).T @ A.astype(np.float64)
        assert B.shape == (c, n)
        assert np.max(np.abs(B - refB)) < tol * np.sqrt(m) * np.abs(refB).max() + tol


@pytest.mark.parametrize("m,c,cond", [(2000, 25, 1e2), (5000, 210, 1e6), (333, 333, 1e3), (4096, 272, 1e4),
                                      (100, 7, 1.0)])
def test_cholqr2_orthonormalizes(gpu, m, c, cond):
    rng = np.random.default_rng(c)
    U = inputs.haar_columns(rng, m, c)
    Vr = inputs.haar_columns(rng, c, c)
    Y = (U * np.logspace(0, -np.log10(cond), c)) @ Vr.T
    V, R, info = gpu.orthonormalize(to_dev(Y), want_r=True)
    V, R = to_np(V), to_np(R)
    assert int(to_np(info)[0]) == 0
    assert np.abs(V.T @ V - np.eye(c)).max() < 1e-13 * max(10, c)
    assert np.allclose(np.tril(R, -1), 0.0) and np.all(np.diag(R) > 0)
    assert np.linalg.norm(Y - V @ R) < 1e-14 * cond * np.linalg.norm(Y) * c
    # unique QR with positive diagonal: compare with the oracle's Householder QR
    q, r = np.linalg.qr(Y)
    s = np.sign(np.diag(r))
    assert np.allclose(V[:, :min(c, 10)], (q * s)[:, :min(c, 10)], atol=1e-9 * cond)


@pytest.mark.parametrize("rows,cols,seed", [(25, 500, 0), (210, 2000, 1), (47, 333, 2), (64, 64, 3),
                                            (136, 136, 4), (200, 200, 5), (272, 4000, 6), (30, 12, 7),
                                            # the reduced-matrix shapes of the benchmark workloads: 157, 256
                                            # and 128 workgroups of 64 columns (pivot agreement over more
                                            # than 64 key slots, i.e. several slots per polling lane)
                                            (210, 10000, 8), (272, 16384, 9), (64, 8192, 10), (17, 4097, 12),
                                            # one workgroup holding the whole matrix in registers (rows <= 192,
                                            # cols <= 192): the l x l second factorisation
                                            (125, 125, 13), (192, 192, 14), (150, 40, 15), (20, 180, 16),
                                            (100, 190, 17),
                                            # more than 256 workgroups (313): the decider polls its key
                                            # slots in two chunks of 256
                                            (24, 20000, 18)])
def test_cpqr_matches_oracle(gpu, rows, cols, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((rows, cols)) * np.exp(rng.uniform(-6, 0, cols))[None, :]
    piv, R, Rt, Q, info = gpu.cpqr(to_dev(M))
    piv, R, Rt, Q = to_np(piv), to_np(R), to_np(Rt), to_np(Q)
    kmax = min(rows, cols)
    ok, bad = pivots_valid(M, piv)
    assert ok, f"pivot {bad} was not a maximal column"
    ref = oracle_cpqr(M)
    if first_difference(piv, ref.perm[:kmax]) >= 0:
        ref = oracle_cpqr(M, piv=piv)      # a near-tie was broken the other way: compare on its pivots
    scale = np.abs(ref.R).max()
    assert np.max(np.abs(R[:kmax] - ref.R[:, :kmax])) < 1e-12 * scale
    assert np.all(R[kmax:] == 0.0)
    # Rt holds R in the original column order (transposed)
    Rorig = np.zeros((kmax, cols))
    Rorig[:, ref.perm] = ref.R
    assert np.max(np.abs(Rt[:, :kmax].T - Rorig)) < 1e-12 * scale
    assert np.max(np.abs(Q - ref.Q)) < 1e-10
    assert int(to_np(info)[0]) == 0


@pytest.mark.parametrize("rows,cols", [(40, 300), (40, 150), (60, 60)])
def test_cpqr_rank_deficient_stop(gpu, rows, cols):
    rng = np.random.default_rng(11)
    M = rng.standard_normal((rows, 6)) @ rng.standard_normal((6, cols))
    piv, R, Rt, Q, info = gpu.cpqr(to_dev(M))
    piv, R = to_np(piv), to_np(R)
    ref = oracle_cpqr(M)
    assert ref.rank == 6
    assert int(to_np(info)[0]) & 0x2
    assert np.array_equal(piv[:6], ref.perm[:6])
    assert np.allclose(R[6:, :], 0.0)
    # after the stop the remaining pivots are the smallest unused indices
    kmax = min(rows, cols)
    assert np.array_equal(piv[6:], ref.perm[6:kmax])


def test_cholqr2_shifted_retry_on_singular_gram(gpu):
    """A zero column makes a pivot of the Gram's Cholesky exactly 0: the
    first attempt breaks down, the shifted retry runs (flag 0x1, not 0x10)
    and the result is a finite basis whose range still contains Y."""
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((500, 40))
    Y[:, 17] = 0.0
    V, R, info = gpu.orthonormalize(to_dev(Y), want_r=True)
    V, info = to_np(V), int(to_np(info)[0])
    assert info & 0x1 and not info & 0x10
    assert np.all(np.isfinite(V))
    resid = Y - V @ np.linalg.lstsq(V, Y, rcond=None)[0]
    assert np.linalg.norm(resid) < 1e-8 * np.linalg.norm(Y)


@pytest.mark.parametrize("c", [1, 15, 16, 17, 100, 256, 257, 511, 512, 513, 700])
def test_cholqr2_panel_widths(gpu, c):
    """Panel widths around the 16-column blocks and the multi-workgroup limit."""
    rng = np.random.default_rng(c)
    m = max(2 * c, 64)
    Y = rng.standard_normal((m, c)) * np.logspace(0, -2, c)[None, :]
    V, R, info = gpu.orthonormalize(to_dev(Y), want_r=True)
    V, R = to_np(V), to_np(R)
    assert int(to_np(info)[0]) == 0
    assert np.abs(V.T @ V - np.eye(c)).max() < 1e-12 * max(10, c)
    assert np.linalg.norm(Y - V @ R) < 1e-13 * np.linalg.norm(Y) * max(10, c)
    assert np.allclose(np.tril(R, -1), 0.0) and np.all(np.diag(R) > 0)


@pytest.mark.parametrize("m,c", [(7, 5), (13, 13), (1001, 33), (4099, 272), (4100, 272), (2052, 130)])
def test_cholqr2_row_counts(gpu, m, c):
    """Row counts that leave a tail past the last whole fragment of the Gram
    product, or are odd (the update then takes the general product)."""
    rng = np.random.default_rng(m + c)
    Y = rng.standard_normal((m, c)) * np.logspace(0, -3, c)[None, :]
    V, R, info = gpu.orthonormalize(to_dev(Y), want_r=True)
    V, R = to_np(V), to_np(R)
    assert int(to_np(info)[0]) == 0
    assert np.abs(V.T @ V - np.eye(c)).max() < 1e-12 * max(10, c)
    assert np.linalg.norm(Y - V @ R) < 1e-13 * np.linalg.norm(Y) * max(10, c)
    q, r = np.linalg.qr(Y)
    s = np.sign(np.diag(r))
    assert np.allclose(R, s[:, None] * r, atol=1e-10 * np.abs(r).max())
