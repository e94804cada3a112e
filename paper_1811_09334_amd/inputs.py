"""Seeded synthetic inputs for randomized QLP workloads.

This module only *builds inputs*: matrices with prescribed singular spectra,
Gaussian test matrices and loss weights.  It contains none of the
factorisation's arithmetic and is shared by the CPU oracle tests and the GPU
tests/benchmark so that both sides see bit-identical data.

Constructions follow the paper's synthetic examples (Section 5, Example 5.1:
A = U diag(s) V^T with random orthogonal U, V and the polynomially /
exponentially decaying spectra "pds" / "eds") and the benchmark workloads
listed in ``WORKLOADS`` (two-level log-linear spectrum, low rank plus noise,
exponential decay, noise plus spikes).

Two back ends:
  * NumPy (PCG64), FP64, for sizes the CPU handles in seconds;
  * torch on a device (for the full-size workloads), same recipe, its own
    seeded generator.  Values differ between back ends; a test always feeds
    the same array to both sides it compares.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np


# ----------------------------------------------------------------------------
# spectra
# ----------------------------------------------------------------------------
def spectrum_poly(n: int, power: float = 2.0) -> np.ndarray:
    """s_j = j^(-power), j = 1..n."""
    j = np.arange(1, n + 1, dtype=np.float64)
    return j ** (-power)


def spectrum_two_level(n: int, head: int = 200, lo: float = 1e-4, tail: float = 1e-6) -> np.ndarray:
    """s_j = lo^((j-1)/(head-1)) for j <= head (log-linear 1 -> lo), ``tail`` beyond."""
    s = np.full(n, tail, dtype=np.float64)
    h = min(head, n)
    j = np.arange(h, dtype=np.float64)
    s[:h] = 10.0 ** (math.log10(lo) * j / max(head - 1, 1))
    return s


def spectrum_exp(n: int, scale: float = 300.0) -> np.ndarray:
    """s_j = exp(-j / scale), j = 1..n."""
    j = np.arange(1, n + 1, dtype=np.float64)
    return np.exp(-j / scale)


def spectrum_pds(n: int, t: int = 30, s: float = 2.0) -> np.ndarray:
    """Example 5.1 (I): diag(1,...,1, 2^-s, 3^-s, ..., (n-t+1)^-s) with t ones."""
    out = np.ones(n, dtype=np.float64)
    j = np.arange(2, n - t + 2, dtype=np.float64)
    out[t:] = j ** (-s)
    return out


def spectrum_eds(n: int, t: int = 30, s: float = 1.0 / 20.0) -> np.ndarray:
    """Example 5.1 (II): diag(1,...,1, 2^-s, 2^-2s, ..., 2^-(n-t)s) with t ones."""
    out = np.ones(n, dtype=np.float64)
    j = np.arange(1, n - t + 1, dtype=np.float64)
    out[t:] = 2.0 ** (-s * j)
    return out


# ----------------------------------------------------------------------------
# NumPy back end
# ----------------------------------------------------------------------------
def haar_columns(rng: np.random.Generator, m: int, r: int) -> np.ndarray:
    """m x r matrix with orthonormal columns: Q factor of an N(0,1) matrix,
    column signs fixed so that diag(R) > 0 (Haar distributed)."""
    g = rng.standard_normal((m, r))
    q, rr = np.linalg.qr(g)
    sgn = np.sign(np.diag(rr))
    sgn[sgn == 0] = 1.0
    return q * sgn


def svd_matrix(m: int, n: int, s: np.ndarray, seed: int) -> np.ndarray:
    """A = U diag(s) V^T, U (m x r), V (n x r) Haar, r = len(s).  Fortran order."""
    rng = np.random.default_rng(seed)
    r = len(s)
    u = haar_columns(rng, m, r)
    v = haar_columns(rng, n, r)
    return np.asfortranarray((u * s) @ v.T)


def lowrank_plus_noise(m: int, n: int, s: np.ndarray, noise: float, seed: int,
                       noise_first: bool = False) -> np.ndarray:
    """A = U_r diag(s) V_r^T + noise * N(0,1)  (or N(0,1)*noise + signal)."""
    rng = np.random.default_rng(seed)
    r = len(s)
    if noise_first:
        e = rng.standard_normal((m, n)) * noise
        u = haar_columns(rng, m, r)
        v = haar_columns(rng, n, r)
    else:
        u = haar_columns(rng, m, r)
        v = haar_columns(rng, n, r)
        e = rng.standard_normal((m, n)) * noise
    return np.asfortranarray((u * s) @ v.T + e)


def gaussian(rows: int, cols: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) matrix (Fortran order), e.g. the test matrix Omega."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((rows, cols)))


def uniform_weights(k: int, seed: int) -> np.ndarray:
    """Seeded U(0,1) loss weights w_1..w_k."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=k)


def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even); returned as float64.

    Used to make the exact 16-bit test matrix that a mixed-precision run feeds
    to its GEMMs, so that both sides of a comparison share it."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) >> 16
    out = (b.astype(np.uint32) << 16).view(np.float32)
    return np.asfortranarray(out.astype(np.float64))


def round_to_fp16(x: np.ndarray) -> np.ndarray:
    """Round to IEEE half (ties to even), returned as float64."""
    return np.asfortranarray(np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    m: int
    n: int
    k: int
    p: int
    q: int
    d: int
    b: int
    precision: str          # 'f64' | 'f32' | 'bf16' | 'fp16' | 'bf16x3'
    storage: str            # dtype A is stored in: 'f64' | 'f32'
    kind: str               # 'svd' | 'lowrank_noise' | 'noise_spikes'
    spectrum: Callable[[int], np.ndarray]
    rank: Optional[int] = None      # number of singular values in the construction
    noise: float = 0.0
    seed_a: int = 0
    seed_omega: int = 0

    @property
    def l(self) -> int:
        return self.k + self.p

    def spectrum_values(self) -> np.ndarray:
        r = self.rank if self.rank is not None else self.n
        return self.spectrum(r)

    def scaled(self, m: int, n: int, k: Optional[int] = None, p: Optional[int] = None,
               rank: Optional[int] = None, name: Optional[str] = None) -> "Workload":
        return dataclasses.replace(
            self, name=name or f"{self.name}@{m}x{n}", m=m, n=n,
            k=self.k if k is None else k, p=self.p if p is None else p,
            rank=self.rank if rank is None else rank)


WORKLOADS = {
    # plain RQLP, FP64, s_j = j^-2
    "rqlp_f64_1000x500": Workload("rqlp_f64_1000x500", 1000, 500, 20, 5, 0, 0, 0, "f64", "f64",
                                  "svd", lambda r: spectrum_poly(r, 2.0), None, 0.0, 1000, 2000),
    # ERQLP with one power iteration, FP64, two-level log-linear spectrum
    "erqlp_f64_20000x10000": Workload("erqlp_f64_20000x10000", 20000, 10000, 200, 10, 1, 2, 0, "f64",
                                      "f64", "svd", lambda r: spectrum_two_level(r), None, 0.0, 1001, 2001),
    # mixed precision ERQLP: rank-256 (s_j = 1/j) + 1e-3 noise, stored FP32
    "erqlp_bf16_32768x16384": Workload("erqlp_bf16_32768x16384", 32768, 16384, 256, 16, 2, 2, 0, "bf16",
                                       "f32", "lowrank_noise", lambda r: spectrum_poly(r, 1.0), 256, 1e-3,
                                       1002, 2002),
    # block RQLP, FP16 GEMMs, s_j = exp(-j/300)
    "brqlp_fp16_65536x8192": Workload("brqlp_fp16_65536x8192", 65536, 8192, 1024, 32, 1, 0, 64, "fp16",
                                      "f32", "svd", lambda r: spectrum_exp(r, 300.0), None, 0.0, 1003, 2003),
    # differentiable RQLP, FP32: N(0,1)/sqrt(n) + rank-64 signal s_j = 10/j
    "drqlp_f32_16384x4096": Workload("drqlp_f32_16384x4096", 16384, 4096, 128, 8, 1, 0, 0, "f32", "f32",
                                     "noise_spikes", lambda r: 10.0 * spectrum_poly(r, 1.0), 64, None,
                                     1004, 2004),
}


# Example 5.1 of Section 5 (Tables 1-2): m = n, k = 120, p = 5, q = 0, the
# pds (t = 30, s = 2) and eds (t = 30, s = 1/20) spectra with Haar factors
# (the paper's random orthogonal factors are not specified), FP64.
PAPER_EXAMPLE_SIZES = (2000, 4000, 6000)


def paper_example(example: str, n: int, d: int = 0) -> Workload:
    """The Section 5 replica workload ``example`` ('pds' or 'eds') at m = n."""
    if example not in ("pds", "eds"):
        raise ValueError(example)
    spec = spectrum_pds if example == "pds" else spectrum_eds
    idx = PAPER_EXAMPLE_SIZES.index(n) if n in PAPER_EXAMPLE_SIZES else 9
    base = 1100 if example == "pds" else 1200
    return Workload(f"{example}_{n}", n, n, 120, 5, 0, d, 0, "f64", "f64", "svd", spec, None, 0.0,
                    base + idx, base + 50 + idx)


def make_matrix(w: Workload) -> np.ndarray:
    """Build A for workload ``w`` with NumPy (FP64 values, Fortran order).

    FP32-stored workloads are rounded to float32 and widened back, so the
    returned FP64 array holds exactly the values the FP32 path reads."""
    s = w.spectrum_values()
    if w.kind == "svd":
        a = svd_matrix(w.m, w.n, s, w.seed_a)
    elif w.kind == "lowrank_noise":
        a = lowrank_plus_noise(w.m, w.n, s, w.noise, w.seed_a)
    elif w.kind == "noise_spikes":
        a = lowrank_plus_noise(w.m, w.n, s, 1.0 / math.sqrt(w.n), w.seed_a, noise_first=True)
    else:
        raise ValueError(w.kind)
    if w.storage == "f32":
        a = np.asfortranarray(a.astype(np.float32).astype(np.float64))
    return a


def make_omega(w: Workload) -> np.ndarray:
    """N(0,1) test matrix Omega (n x l), rounded to the GEMM input type of a
    mixed-precision workload so that both sides share the exact values."""
    om = gaussian(w.n, w.l, w.seed_omega)
    if w.precision in ("bf16", "bf16x3"):
        om = round_to_bf16(om)
    elif w.precision == "fp16":
        om = round_to_fp16(om)
    elif w.precision == "f32":
        om = np.asfortranarray(om.astype(np.float32).astype(np.float64))
    return om


# ----------------------------------------------------------------------------
# torch back end (device generation for full-size workloads)
# ----------------------------------------------------------------------------
def make_matrix_torch(w: Workload, device, dtype=None):
    """Same recipe as ``make_matrix`` on a torch device (seeded generator).

    Returns a column-major (Fortran-ordered) tensor view of shape (m, n):
    ``A.stride() == (1, m)``.  ``dtype`` defaults to the workload's storage type."""
    import torch

    if dtype is None:
        dtype = torch.float64 if w.storage == "f64" else torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(w.seed_a)
    s = torch.as_tensor(w.spectrum_values(), dtype=torch.float64, device=device)
    r = s.numel()

    def haar(rows, cols):
        x = torch.randn(rows, cols, generator=g, dtype=torch.float64, device=device)
        qm, rm = torch.linalg.qr(x)
        sg = torch.sign(torch.diagonal(rm))
        sg[sg == 0] = 1.0
        return qm * sg

    if w.kind == "svd":
        u = haar(w.m, r)
        v = haar(w.n, r)
        at = (v * s) @ u.T                       # (n, m) row-major == A col-major
    elif w.kind == "lowrank_noise":
        u = haar(w.m, r)
        v = haar(w.n, r)
        at = (v * s) @ u.T
        at += w.noise * torch.randn(w.n, w.m, generator=g, dtype=torch.float64, device=device)
    elif w.kind == "noise_spikes":
        at = torch.randn(w.n, w.m, generator=g, dtype=torch.float64, device=device) / math.sqrt(w.n)
        u = haar(w.m, r)
        v = haar(w.n, r)
        at += (v * s) @ u.T
    else:
        raise ValueError(w.kind)
    at = at.to(dtype).contiguous()
    return at.T


def make_omega_torch(w: Workload, device, dtype=None):
    """Omega from the NumPy recipe, copied to ``device`` column-major (n, l)."""
    import torch

    om = make_omega(w)
    if dtype is None:
        dtype = torch.float64
    t = torch.from_numpy(np.ascontiguousarray(om.T)).to(device=device, dtype=dtype)
    return t.T
