"""Pins for the CPU oracle's adaptive Wiener filter and hybrid pipeline (no GPU).

References other than the oracle itself:
  * scipy.signal.wiener (local mean / variance form of the adaptive Wiener filter) run on
    the image after numpy's 'symmetric' padding, then cropped: with the same noise power
    it must agree everywhere, and the mean of its local variance is the noise estimate;
  * a numpy float64 formulation over sliding_window_view (np.mean / np.var per window);
  * closed forms: nu2 = 0 gives the identity, a huge nu2 gives the box mean
    (scipy.ndimage.uniform_filter), a flat region returns its mean, constants pass.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.signal as sig
from numpy.lib.stride_tricks import sliding_window_view

from phantoms import noisy_phantom, random_image


def scipy_wiener_symmetric(a, win, noise):
    wh, ww = win
    p = np.pad(a.astype(np.float64), ((wh // 2, wh // 2), (ww // 2, ww // 2)), mode="symmetric")
    out = sig.wiener(p, (wh, ww), noise)
    return out[wh // 2:wh // 2 + a.shape[0], ww // 2:ww // 2 + a.shape[1]]


def scipy_local_var_symmetric(a, win):
    wh, ww = win
    p = np.pad(a.astype(np.float64), ((wh // 2, wh // 2), (ww // 2, ww // 2)), mode="symmetric")
    m = sig.correlate(p, np.ones(win), "same") / (wh * ww)
    m2 = sig.correlate(p ** 2, np.ones(win), "same") / (wh * ww)
    v = m2 - m ** 2
    return v[wh // 2:wh // 2 + a.shape[0], ww // 2:ww // 2 + a.shape[1]]


def numpy_windows_wiener(a, win, noise=None):
    wh, ww = win
    p = np.pad(a.astype(np.float64), ((wh // 2, wh // 2), (ww // 2, ww // 2)), mode="symmetric")
    wins = sliding_window_view(p, (wh, ww))
    mu = wins.mean(axis=(2, 3))
    var = wins.var(axis=(2, 3))
    nu2 = var.mean() if noise is None else noise
    den = np.maximum(var, nu2)
    gain = np.where(den > 0, np.maximum(var - nu2, 0) / np.where(den > 0, den, 1), 0.0)
    return mu + (a - mu) * gain, nu2


CASES = [
    (64, 64, (3, 3), 255, 10, 0.0, 1),
    (97, 61, (5, 5), 255, 15, 0.0, 2),
    (50, 70, (7, 7), 4095, 60, 0.0, 3),
    (33, 40, (3, 5), 4095, 40, 0.0, 4),
    (7, 9, (7, 7), 255, 20, 0.0, 5),     # window about the image size
]


@pytest.mark.parametrize("h,w,win,maxv,sigma,dens,seed", CASES)
def test_against_scipy_wiener_given_noise(orc, h, w, win, maxv, sigma, dens, seed):
    a = noisy_phantom(h, w, maxv, sigma, dens, seed)
    for noise in (1.0, sigma ** 2, 7.5 * sigma ** 2):
        ref = scipy_wiener_symmetric(a, win, noise) / maxv
        got = orc.wiener(a, win, maxv, noise)
        # scipy sums windows by FFT / direct correlate in float; agree to fp64 noise
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9)


@pytest.mark.parametrize("h,w,win,maxv,sigma,dens,seed", CASES)
def test_noise_estimate_is_mean_local_variance(orc, h, w, win, maxv, sigma, dens, seed):
    a = noisy_phantom(h, w, maxv, sigma, dens, seed)
    ref = scipy_local_var_symmetric(a, win).mean()
    got = orc.noise_estimate(a, win)
    assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref))
    out, nu2 = orc.wiener(a, win, maxv, -1.0, return_nu2=True)
    assert nu2 == got
    ref_out = scipy_wiener_symmetric(a, win, nu2) / maxv
    np.testing.assert_allclose(out, ref_out, rtol=0, atol=1e-9)


@pytest.mark.parametrize("h,w,win,maxv,sigma,dens,seed", CASES)
def test_against_numpy_window_form(orc, h, w, win, maxv, sigma, dens, seed):
    a = noisy_phantom(h, w, maxv, sigma, dens, seed)
    ref, nu2_ref = numpy_windows_wiener(a, win)
    got, nu2 = orc.wiener(a, win, maxv, -1.0, return_nu2=True)
    assert abs(nu2 - nu2_ref) <= 1e-9 * max(1.0, nu2_ref)
    np.testing.assert_allclose(got, ref / maxv, rtol=0, atol=1e-12)


def test_zero_noise_is_identity(orc):
    a = random_image((40, 45), 4095, 9)
    out = orc.wiener(a, (5, 5), 4095, 0.0)
    np.testing.assert_allclose(out, a / 4095.0, rtol=0, atol=1e-15)


def test_huge_noise_is_box_mean(orc):
    a = random_image((40, 45), 255, 10)
    for win in ((3, 3), (5, 5), (7, 3)):
        out = orc.wiener(a, win, 255, 1e30)
        box = ndi.uniform_filter(a.astype(np.float64), size=win, mode="reflect")
        np.testing.assert_allclose(out, box / 255.0, rtol=0, atol=1e-12)


def test_flat_region_returns_local_mean(orc):
    """Inside a flat region the local variance is 0 and the output is the local mean."""
    a = random_image((30, 30), 255, 11)
    a[8:20, 5:25] = 77
    out = orc.wiener(a, (5, 5), 255, -1.0)
    # pixels whose 5x5 window lies inside the flat block
    assert np.all(out[10:18, 7:23] == 77 / 255.0)


@pytest.mark.parametrize("value", [0, 1, 255, 4095])
def test_constant_image_unchanged(orc, value):
    for shape in [(1, 1), (1, 9), (8, 1), (12, 17)]:
        a = np.full(shape, value, np.int32)
        for noise in (-1.0, 0.0, 25.0):
            out = orc.wiener(a, (5, 5), 4095, noise)
            np.testing.assert_array_equal(out, np.full(shape, value / 4095.0))


def test_hybrid_constant_unchanged(orc):
    g = np.full((20, 23), 300, np.int32)
    out, a, nu2 = orc.hybrid(g, 11, (5, 5), 4095)
    np.testing.assert_array_equal(a, g)
    np.testing.assert_array_equal(out, g / 4095.0)
    assert nu2 == 0.0


def test_hybrid_is_wiener_of_amf(orc):
    g = noisy_phantom(60, 70, 255, 15, 0.2, 12)
    out, a, nu2 = orc.hybrid(g, 9, (5, 5), 255)
    a_ref = orc.amf(g, 9)
    np.testing.assert_array_equal(a, a_ref)
    ref = scipy_wiener_symmetric(a_ref, (5, 5), nu2) / 255
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-9)


def test_bad_window_rejected(orc):
    a = np.zeros((4, 4), np.int32)
    for win in ((2, 3), (3, 0), (4, 4)):
        with pytest.raises(ValueError):
            orc.wiener(a, win, 255)
