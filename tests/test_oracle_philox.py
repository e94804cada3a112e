"""Pins for the oracle's Philox4x32-10 / Box-Muller reference: the published
known-answer vectors and the first two moments of the Gaussian stream."""
import os

import numpy as np

from oracle.philox import omega_gaussian, philox4x32_10

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_known_answer_vectors():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [line.split() for line in f if line.strip() and not line.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x32_10(np.array(v[0:4], dtype=np.uint32), np.array(v[4:6], dtype=np.uint32))
        assert [int(x) for x in out] == v[6:10]


def test_gaussian_stream_moments_and_layout():
    om = omega_gaussian(4000, 50, seed=123)
    assert om.shape == (4000, 50) and om.flags.f_contiguous
    assert abs(om.mean()) < 0.01 and abs(om.var() - 1.0) < 0.01
    # distinct seeds and distinct elements give distinct streams
    om2 = omega_gaussian(4000, 50, seed=124)
    assert np.abs(om - om2).max() > 1.0
    assert np.unique(om).size == om.size
