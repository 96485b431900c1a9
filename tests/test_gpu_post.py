"""GPU tests of the post-processing contrast stretch (Alg. 1, step e): the library's
stretched output against the oracle's stretch, resident and staged paths bit-identical,
per-slice ranges in batches, constant slices unchanged."""
import numpy as np
import pytest
import torch

import oracle
from phantoms import noisy_phantom
from tests.gpu_util import gpu_available, log, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def hd():
    import paper_2005_05371_amd as hd
    hd.load()
    yield hd
    hd.set_option(hd.HD_OPT_RESIDENT, -1)


def _bits(t):
    return to_host(t).view(np.uint32)


@pytest.mark.parametrize("shape,maxv,smax,win", [((300, 421), 255, 7, 3), ((517, 250), 4095, 11, 5),
                                                 ((1600, 1600), 255, 9, 5), ((64, 64), 4095, 5, 7),
                                                 ((1000, 1300), 4095, 9, 5), ((300, 300), 65535, 7, 5)])
def test_stretch_matches_oracle(hd, shape, maxv, smax, win):
    g = noisy_phantom(shape[0], shape[1], maxv, 20, 0.2, seed=shape[0] + win)
    x = to_dev(g, np.uint8 if maxv == 255 else np.uint16)
    res = {}
    for resident in (1, 0):
        hd.set_option(hd.HD_OPT_RESIDENT, resident)
        log(f"stretch {shape} resident={resident}")
        plain = hd.hybrid_denoise(x, smax, win, maxv)
        st = hd.hybrid_denoise(x, smax, win, maxv, stretch=True)
        res[resident] = (_bits(plain), _bits(st))
        y, s = to_host(plain).astype(np.float64), to_host(st).astype(np.float64)
        # the stretch of the library's own Wiener output, in float64
        np.testing.assert_allclose(s, oracle.contrast_stretch(y), rtol=0, atol=2e-6)
        assert s.min() == 0.0 and s.max() == 1.0
    np.testing.assert_array_equal(res[0][1], res[1][1])
    # end to end against the oracle at every size: Wiener error (<= 1e-4) scaled by 1 / range, twice
    ref, _, _ = oracle.hybrid(g, smax, win, maxv)
    span = ref.max() - ref.min()
    got = to_host(st).astype(np.float64)
    assert np.max(np.abs(got - oracle.contrast_stretch(ref))) <= 2e-4 / span + 1e-6


def test_stretch_batched_per_slice(hd):
    imgs = [noisy_phantom(h, w, 255, 15, 0.1, seed=70 + i)
            for i, (h, w) in enumerate([(120, 77), (33, 300), (256, 256), (9, 5), (200, 131)])]
    imgs.append(np.full((50, 60), 77, np.int32))  # constant slice: unchanged
    ins = [to_dev(g, np.uint8) for g in imgs]
    for resident in (1, 0):
        hd.set_option(hd.HD_OPT_RESIDENT, resident)
        log(f"stretch batched resident={resident}")
        plain = [to_host(o).astype(np.float64) for o in hd.hybrid_denoise_batched(ins, 9, 5, 255)]
        outs = [torch.empty(x.shape, dtype=torch.float32, device="cuda") for x in ins]
        for rep in range(2):
            for o in outs:
                o.fill_(-1.0)
            hd.hybrid_denoise_batched(ins, 9, 5, 255, outs=outs, stretch=True)
            for i, (o, y) in enumerate(zip(outs, plain)):
                np.testing.assert_allclose(to_host(o), oracle.contrast_stretch(y), rtol=0, atol=2e-6,
                                           err_msg=f"slice {i} rep {rep}")
        np.testing.assert_array_equal(to_host(outs[-1]), plain[-1].astype(np.float32))


@pytest.mark.parametrize("shape,maxv,smax,parts", [((300, 421), 255, 7, 2), ((517, 250), 4095, 11, 4),
                                                   ((1600, 1600), 255, 9, 8), ((37, 100), 255, 9, 8),
                                                   ((64, 64), 4095, 5, 3)])
def test_partitioned_amf_matches_oracle(hd, shape, maxv, smax, parts):
    """The paper's partitioned AMF (independent strips) bit-exact against the oracle's."""
    g = noisy_phantom(shape[0], shape[1], maxv, 20, 0.3, seed=parts * 100 + smax)
    x = to_dev(g, np.uint8 if maxv == 255 else np.uint16)
    log(f"partitioned amf {shape} parts={parts}")
    a = hd.amf_filter(x, smax, parts=parts)
    np.testing.assert_array_equal(to_host(a).astype(np.int32), oracle.amf_partitioned(g, smax, parts))
    if parts > 1:  # near the cuts the strips differ from the whole-image filter
        assert np.any(to_host(hd.amf_filter(x, smax)) != to_host(a))


@pytest.mark.parametrize("stretch", [False, True])
def test_partitioned_hybrid_matches_oracle(hd, stretch):
    g = noisy_phantom(400, 333, 255, 15, 0.2, seed=5)
    x = to_dev(g, np.uint8)
    log(f"partitioned hybrid stretch={stretch}")
    y = to_host(hd.hybrid_partitioned(x, 9, 5, 255, parts=4, stretch=stretch)).astype(np.float64)
    ref = oracle.wiener(oracle.amf_partitioned(g, 9, 4), 5, 255)
    if stretch:
        span = ref.max() - ref.min()
        ref = oracle.contrast_stretch(ref)
        assert np.max(np.abs(y - ref)) <= 2e-4 / span + 1e-6
    else:
        assert np.max(np.abs(y - ref)) <= 1e-4


def test_contrast_stretch_entry_point(hd):
    rng = np.random.default_rng(4)
    y = rng.uniform(0.2, 0.7, size=(333, 517)).astype(np.float32)
    t = torch.from_numpy(y).cuda()
    hd.contrast_stretch(t)
    np.testing.assert_allclose(to_host(t), oracle.contrast_stretch(y.astype(np.float64)), rtol=0, atol=2e-6)
    c = torch.full((70, 90), 0.25, dtype=torch.float32, device="cuda")
    hd.contrast_stretch(c)
    assert torch.all(c == 0.25)
