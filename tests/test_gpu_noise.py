"""GPU tests of the on-device degradation (Alg. 1 step 3) against the oracle, which draws
the same Philox4x32-10 numbers: identical images except where the unrounded Gaussian value
sits within 1e-9 of a rounding tie (the double log / cos of the two sides may differ in the
last place there)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import degrade as odeg
from phantoms import ellipse_phantom as _ellipses


def ellipse_phantom(h, w, maxv, seed):
    inten = (40, 220) if maxv == 255 else (0, maxv)
    return _ellipses(h, w, np.random.default_rng(seed), intensity=inten)
from tests.gpu_util import gpu_available, log, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def hd():
    import paper_2005_05371_amd as hd
    hd.load()
    return hd


def _check(got, clean, sigma, density, maxv, seed, stream):
    ref, pre = odeg.degrade(clean, sigma, density, maxv, seed, stream, return_pre=True)
    frac = pre - np.floor(pre)
    tie = np.abs(frac - 0.5) < 1e-9
    bad = (got != ref) & ~tie
    assert not bad.any(), f"{int(bad.sum())} pixels differ away from ties"
    return ref


@pytest.mark.parametrize("shape,maxv,sigma,density,seed", [((300, 421), 255, 15.0, 0.2, 7),
                                                           ((517, 250), 4095, 40.0, 0.3, 2 ** 40 + 3),
                                                           ((1600, 1600), 255, 15.0, 0.2, 123),
                                                           ((3, 5), 255, 0.0, 1.0, 1),
                                                           ((2, 20000), 255, 30.0, 0.1, 4),
                                                           ((66000, 3), 4095, 30.0, 0.1, 5)])
def test_degrade_matches_oracle(hd, shape, maxv, sigma, density, seed):
    clean = ellipse_phantom(shape[0], shape[1], maxv, seed=seed % 1000)
    x = to_dev(clean, np.uint8 if maxv == 255 else np.uint16)
    log(f"degrade {shape} sigma={sigma} density={density}")
    got = to_host(hd.degrade_image(x, sigma, density, seed, stream_id=3, max_value=maxv)).astype(np.int32)
    _check(got, clean, sigma, density, maxv, seed, 3)


def test_degrade_in_place_and_pitched(hd):
    clean = ellipse_phantom(200, 300, 255, seed=4)
    big = torch.zeros((200, 320), dtype=torch.uint8, device="cuda")
    view = big[:, 7:307]  # row pitch 320, unaligned start
    view.copy_(to_dev(clean, np.uint8))
    hd.degrade_image(view, 20.0, 0.1, 99, stream_id=1, out=view)  # in place
    got = to_host(view).astype(np.int32)
    _check(got, clean, 20.0, 0.1, 255, 99, 1)
    assert torch.all(big[:, :7] == 0) and torch.all(big[:, 307:] == 0)


def test_degrade_then_denoise_end_to_end(hd):
    """Noise made on the device, filtered on the device: the AMF equals the oracle's AMF of
    the oracle's noisy image (where the two noisy images agree, everywhere in practice)."""
    clean = ellipse_phantom(256, 256, 255, seed=9)
    x = to_dev(clean, np.uint8)
    noisy = hd.degrade_image(x, 15.0, 0.2, 5)
    g = to_host(noisy).astype(np.int32)
    ref = _check(g, clean, 15.0, 0.2, 255, 5, 0)
    if np.array_equal(g, ref):
        np.testing.assert_array_equal(to_host(hd.amf_filter(noisy, 9)).astype(np.int32), oracle.amf(ref, 9))


def test_degrade_bad_args(hd):
    x = torch.zeros((16, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(hd.HDError):
        hd.degrade_image(x, 1.0, 1.5, 0)
    with pytest.raises(hd.HDError):
        hd.degrade_image(x, -1.0, 0.5, 0)
