"""Pins of the degradation oracle (Alg. 1 step 3): the Philox4x32-10 generator against its
published known-answer vectors, and the noise model against its defining properties."""
import os

import numpy as np
import pytest

from oracle import degrade

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        yield v[:4], v[4:6], v[6:]


@pytest.mark.parametrize("ctr,key,expect", list(_kat()))
def test_philox_known_answers(ctr, key, expect):
    out = degrade.philox4x32_10(np.array([ctr], np.uint32), key)[0]
    assert [int(x) for x in out] == expect


def test_no_noise_is_identity():
    x = np.random.default_rng(0).integers(0, 256, size=(40, 70))
    np.testing.assert_array_equal(degrade.degrade(x, 0.0, 0.0, 255, seed=3), x)


def test_gaussian_statistics():
    x = np.full((512, 512), 128)
    g = degrade.degrade(x, 10.0, 0.0, 255, seed=11)
    d = g.astype(np.float64) - 128
    n = d.size
    assert abs(d.mean()) < 5 * 10 / np.sqrt(n)
    # rounding adds 1/12 to the variance
    assert abs(d.var() - (100 + 1 / 12)) < 5 * 100 * np.sqrt(2 / n)
    # fourth moment of a normal: 3 sigma^4 (kurtosis pins the shape, not just the scale)
    k = np.mean(d ** 4) / d.var() ** 2
    assert abs(k - 3.0) < 0.05
    # neighbouring pixels are uncorrelated
    assert abs(np.corrcoef(d[:, :-1].ravel(), d[:, 1:].ravel())[0, 1]) < 0.01


@pytest.mark.parametrize("density", [0.05, 0.3, 1.0])
def test_salt_and_pepper(density):
    x = np.full((300, 300), 100)
    g = degrade.degrade(x, 0.0, density, 4095, seed=5, stream=2)
    imp = (g == 0) | (g == 4095)
    n = g.size
    p = imp.mean()
    assert abs(p - density) <= 5 * np.sqrt(density * (1 - density) / n) + 1e-12
    assert np.all(g[~imp] == 100)
    if density > 0:
        salt = (g == 4095).sum() / imp.sum()
        assert abs(salt - 0.5) < 5 * np.sqrt(0.25 / imp.sum())


def test_clipped_and_streams_differ():
    x = np.full((64, 64), 250)
    g = degrade.degrade(x, 40.0, 0.0, 255, seed=1)
    assert g.min() >= 0 and g.max() == 255
    a = degrade.degrade(x, 40.0, 0.1, 255, seed=1, stream=0)
    b = degrade.degrade(x, 40.0, 0.1, 255, seed=1, stream=1)
    c = degrade.degrade(x, 40.0, 0.1, 255, seed=2, stream=0)
    assert np.mean(a != b) > 0.5 and np.mean(a != c) > 0.5
