"""Pins of oracle.philox: published known-answer vectors and Gaussian moments."""
import os

import numpy as np

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.txt")


def test_known_answer_vectors():
    n = 0
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        assert int(f[0]) == 10
        ctr = np.array([int(v, 16) for v in f[1:5]], dtype=np.uint64)
        key = (int(f[5], 16), int(f[6], 16))
        out = philox.philox4x32_10(ctr, key)
        assert [int(v) for v in out] == [int(v, 16) for v in f[7:11]]
        n += 1
    assert n == 3


def test_gaussian_moments_and_independence():
    V = 20000
    a = philox.gaussian_test_vector(42, 0, V).ravel()
    b = philox.gaussian_test_vector(42, 1, V).ravel()
    for z in (a, b):
        assert abs(z.real.mean()) < 0.02 and abs(z.imag.mean()) < 0.02
        assert abs(z.real.var() - 1) < 0.03 and abs(z.imag.var() - 1) < 0.03
    assert abs(np.vdot(a, b)) / len(a) < 0.03
    c = philox.gaussian_test_vector(43, 0, V).ravel()
    assert abs(np.vdot(a, c)) / len(a) < 0.03
