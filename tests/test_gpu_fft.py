"""GPU tests of the paper's frequency-domain Wiener step (Alg. 1 step d, wnrFn with the
clean original) against the float64 numpy oracle, and of Alg. 1 as printed (partitioned
AMF, this Wiener step, contrast stretch)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import wiener_fft as owf
from phantoms import ellipse_phantom as _ellipses
from oracle import degrade as odeg
from tests.gpu_util import gpu_available, log, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]
TOL = 1e-4


@pytest.fixture(scope="module")
def hd():
    import paper_2005_05371_amd as hd
    hd.load()
    return hd


def _images(h, w, maxv, seed, sigma=20.0, dens=0.0):
    inten = (40, 220) if maxv == 255 else (0, maxv)
    clean = _ellipses(h, w, np.random.default_rng(seed), intensity=inten)
    noisy = odeg.degrade(clean, sigma, dens, maxv, seed)
    return clean, noisy


@pytest.mark.parametrize("shape,maxv", [((64, 80), 255), ((300, 240), 255), ((45, 27), 4095), ((1, 5), 255),
                                        ((1600, 1600), 255), ((1024, 60), 4095), ((4096, 8), 255)])
def test_wiener_fft_matches_oracle(hd, shape, maxv):
    clean, noisy = _images(shape[0], shape[1], maxv, seed=shape[0] + shape[1])
    dt = np.uint8 if maxv == 255 else np.uint16
    log(f"wiener_fft {shape}")
    got = to_host(hd.wiener_fft(to_dev(noisy, dt), to_dev(clean, dt), maxv)).astype(np.float64)
    ref = owf.wiener_fft(noisy, clean, maxv)
    err = np.max(np.abs(got - ref))
    assert err <= TOL, err


def test_wiener_fft_rejects_unsupported_sizes(hd):
    x = torch.zeros((7, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(hd.HDError, match="prime factors"):
        hd.wiener_fft(x, x)
    y = torch.zeros((8, 5000), dtype=torch.uint8, device="cuda")
    with pytest.raises(hd.HDError):
        hd.wiener_fft(y, y)


def test_algorithm_1_as_printed(hd):
    """Partitioned AMF (4 strips), the frequency-domain Wiener step with the original, the
    contrast stretch: against the oracle's composition of the same three steps."""
    clean, noisy = _images(400, 360, 255, seed=8, sigma=15.0, dens=0.2)
    log("algorithm 1 as printed")
    got = to_host(hd.hybrid_paper(to_dev(noisy, np.uint8), to_dev(clean, np.uint8), 9, parts=4)).astype(np.float64)
    y = owf.wiener_fft(oracle.amf_partitioned(noisy, 9, 4), clean, 255)
    ref = oracle.contrast_stretch(y)
    assert np.max(np.abs(got - ref)) <= 2 * TOL / (y.max() - y.min()) + 1e-6
