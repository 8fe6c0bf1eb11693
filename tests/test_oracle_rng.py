"""Pins of the counter-based white noise.

P12 (CPU side):
* Philox4x64-10 words equal NumPy's independent Philox bit generator
  (which pre-increments its 256-bit counter before each block);
* the binary64 ln and cos sequences agree with the C library to a few ulp
  over the whole input range the generator can produce;
* the uniforms are exact odd multiples of 2^-53 inside (0, 1);
* the normals have mean 0, variance 1 and a Gaussian CDF (KS test).
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import rng


def _numpy_block(counter: int, key0: int):
    c = counter - 1  # NumPy increments before generating
    words = [(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(counter=np.array(words, dtype=np.uint64),
                          key=np.array([key0, 0], dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("seed", [0, 1, 42, 2 ** 63 + 12345])
def test_philox_matches_numpy(seed):
    sites = np.array([1, 2, 3, 17, 4095, 4096, 2 ** 24 + 5, 2 ** 40 + 3], dtype=np.uint64)
    w = rng.site_words(seed, sites)
    for i, s in enumerate(sites):
        ref = _numpy_block(int(s), seed)
        got = [int(w[k][i]) for k in range(4)]
        assert got == ref
    # counter 0 (the first site) via a 256-bit wrap-around of NumPy's counter
    w0 = rng.site_words(seed, np.array([0], dtype=np.uint64))
    bg = np.random.Philox(counter=np.array([2 ** 64 - 1] * 4, dtype=np.uint64),
                          key=np.array([seed, 0], dtype=np.uint64))
    assert [int(w0[k][0]) for k in range(4)] == [int(x) for x in bg.random_raw(4)]


def test_uniforms_exact_and_open():
    w = np.array([0, 1, 2 ** 12 - 1, 2 ** 12, 2 ** 64 - 1], dtype=np.uint64)
    u = rng.uniform_open(w)
    assert u[0] == 2.0 ** -53 and u[2] == 2.0 ** -53
    assert u[3] == 3 * 2.0 ** -53
    assert u[-1] == 1.0 - 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_ln_and_cos_sequences_are_accurate():
    r = np.random.default_rng(3)
    u = np.concatenate([r.uniform(0, 1, 200000), [2.0 ** -53, 1 - 2.0 ** -53, 0.5, 0.25, 0.75,
                                                   math.sqrt(0.5), 0.999999]])
    ln = rng.ln_spec(u)
    ref = np.log(u)
    ulp = np.abs(ln - ref) / np.spacing(np.abs(ref))
    assert np.max(ulp) <= 4
    c = rng.cos2pi_spec(u)
    assert np.max(np.abs(c - np.cos(2 * np.pi * u))) < 2e-15
    # quadrant boundaries are exact
    np.testing.assert_array_equal(rng.cos2pi_spec(np.array([0.25, 0.5, 0.75])),
                                  [0.0, -1.0, 0.0])


def test_normals_statistics():
    z = rng.white_noise(48, 7).ravel()
    n = z.size
    assert abs(z.mean()) < 4 / math.sqrt(n)
    assert abs(z.var() - 1) < 4 * math.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # independent seeds give uncorrelated fields
    z2 = rng.white_noise(48, 8).ravel()
    assert abs(np.corrcoef(z, z2)[0, 1]) < 4 / math.sqrt(n)
