"""Pins of the frequency-domain Wiener oracle (Alg. 1 step d, the paper's wnrFn):
the DFT it uses against the DFT's double sum, and the filter against cases whose result
is fixed by the definition."""
import numpy as np
import pytest

from oracle import wiener_fft as wf


@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (8, 8), (6, 10), (15, 4)])
def test_numpy_dft_matches_double_sum(shape):
    x = np.random.default_rng(sum(shape)).normal(size=shape)
    np.testing.assert_allclose(np.fft.fft2(x), wf.dft2_brute(x), atol=1e-9)


def _pair(shape, seed, noise=20.0):
    rng = np.random.default_rng(seed)
    f = rng.integers(0, 256, size=shape).astype(np.float64)
    a = np.clip(f + rng.normal(0, noise, size=shape), 0, 255).round()
    return a, f


def test_clean_input_is_unchanged():
    _, f = _pair((12, 20), 1)
    np.testing.assert_allclose(wf.wiener_fft(f, f, 255), f / 255, atol=1e-12)


def test_zero_original_gives_zero():
    a, _ = _pair((9, 16), 2)
    np.testing.assert_allclose(wf.wiener_fft(a, np.zeros_like(a), 255), 0.0, atol=1e-12)


def test_single_frequency_gain():
    """a = f + noise at one frequency only: every other frequency passes unchanged and that
    one is scaled by |F|^2 / (|F|^2 + |N|^2), written out here in closed form."""
    h, w = 8, 12
    y, x = np.mgrid[0:h, 0:w]
    f = 100 + 40 * np.cos(2 * np.pi * (2 * x / w + y / h))
    n = 10 * np.cos(2 * np.pi * (2 * x / w + y / h))     # noise on the same frequency pair
    out = wf.wiener_fft(f + n, f, 1.0)
    # F at (ky, kx) = (1, 2): 40 * h w / 2; N there: 10 * h w / 2 -> gain 1600 / 1700
    g = 1600 / 1700
    expect = 100 + g * 50 * np.cos(2 * np.pi * (2 * x / w + y / h))
    np.testing.assert_allclose(out, expect, atol=1e-9)


def test_output_real_and_scale_covariant():
    a, f = _pair((10, 14), 3)
    out = wf.wiener_fft(a, f, 255)
    assert np.isrealobj(out)
    np.testing.assert_allclose(wf.wiener_fft(3 * a, 3 * f, 255), 3 * out, atol=1e-10)
    # the gain is at most 1: the output power never exceeds the input's, frequency by frequency
    A = np.fft.fft2(a)
    O = np.fft.fft2(out * 255)
    assert np.all(np.abs(O) <= np.abs(A) + 1e-6)
