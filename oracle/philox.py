"""Reference Philox4x32-10 counter-based generator and Box-Muller Gaussians.

TEST INFRASTRUCTURE: the library's own Gaussian test-matrix generator is
checked against this module.  Definitions: Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11), Philox-4x32 with 10
rounds; Box & Muller (1958).

Stream layout shared by contract with the library (documented in
include/rqlp.h): for the n x l matrix Omega and 64-bit seed s, element
(i, j) is produced by the block with counter (i, j, 0, 0) and key
(lo32(s), hi32(s)); its first two 32-bit outputs u0, u1 give
    U1 = (u0 + 1) * 2^-32 in (0, 1],  U2 = u1 * 2^-32 in [0, 1),
    Omega[i, j] = sqrt(-2 ln U1) * cos(2 pi U2).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """ctr: (..., 4) uint32, key: (..., 2) uint32 -> (..., 4) uint32."""
    c = [np.asarray(ctr[..., i], dtype=np.uint32).copy() for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint32).copy()
    k1 = np.asarray(key[..., 1], dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = (k0 + W0).astype(np.uint32)
                k1 = (k1 + W1).astype(np.uint32)
            p0 = M0 * c[0].astype(np.uint64)
            p1 = M1 * c[2].astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK).astype(np.uint32)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def omega_bits(n: int, l: int, seed: int) -> np.ndarray:
    """(n, l, 2) uint32 raw words u0, u1 for every element."""
    i, j = np.meshgrid(np.arange(n, dtype=np.uint32), np.arange(l, dtype=np.uint32), indexing="ij")
    ctr = np.stack([i, j, np.zeros_like(i), np.zeros_like(i)], axis=-1)
    key = np.empty(i.shape + (2,), dtype=np.uint32)
    key[..., 0] = np.uint32(seed & 0xFFFFFFFF)
    key[..., 1] = np.uint32((seed >> 32) & 0xFFFFFFFF)
    out = philox4x32_10(ctr, key)
    return out[..., :2]


def omega_gaussian(n: int, l: int, seed: int) -> np.ndarray:
    """n x l N(0,1) matrix (Fortran order) from the stream layout above."""
    u = omega_bits(n, l, seed).astype(np.float64)
    u1 = (u[..., 0] + 1.0) * 2.0 ** -32
    u2 = u[..., 1] * 2.0 ** -32
    return np.asfortranarray(np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2))
