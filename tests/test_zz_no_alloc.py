"""The no-allocation entry point (hybrid_denoise_noalloc): same results as hybrid_denoise,
bit for bit, through the C ABI, on consecutive calls that share the library's static
device scratch (the second call smaller than the first); no library allocation (the
allocation fault injector stays armed across it); oversized images rejected up front."""
import numpy as np
import pytest
import torch

from phantoms import noisy_phantom
from tests.gpu_util import gpu_available, log, to_dev, to_host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def hd():
    import paper_2005_05371_amd as hd
    hd.load()
    yield hd
    hd.set_option(hd.HD_OPT_FAIL_ALLOC, 0)


def _bits(t):
    return to_host(t).view(np.uint32)


def _pair(hd, x, smax, win, maxv, stretch=False):
    ref = hd.hybrid_denoise(x, smax, win, maxv, stretch=stretch)
    out = torch.full(x.shape, -3.0, dtype=torch.float32, device="cuda")
    # armed injector: any library scratch allocation in the call below would fail it
    hd.set_option(hd.HD_OPT_FAIL_ALLOC, 1)
    hd.hybrid_denoise_noalloc(x, smax, win, maxv, out=out, stretch=stretch)
    torch.cuda.synchronize()
    hd.set_option(hd.HD_OPT_FAIL_ALLOC, 0)
    return ref, out


@pytest.mark.parametrize("case", [
    # (first shape, second shape, dtype max value, Smax, window): single launch (fits the
    # device at once) and staged launches (does not), each followed by a smaller image
    ((1600, 1600), (700, 500), 255, 9, 5),
    ((3000, 2900), (1000, 1300), 4095, 11, 5),
    ((4096, 4096), (333, 517), 4095, 15, 7),
])
def test_noalloc_matches_hybrid_denoise(hd, case):
    s1, s2, maxv, smax, win = case
    dt = np.uint8 if maxv == 255 else np.uint16
    for i, shape in enumerate((s1, s2)):
        g = noisy_phantom(shape[0], shape[1], maxv, 20 * maxv / 255, 0.3, seed=shape[0] + 7 * i)
        x = to_dev(g, dt)
        log(f"no-alloc {shape} maxv {maxv} smax {smax} win {win} call {i}")
        ref, out = _pair(hd, x, smax, win, maxv, stretch=(i == 1))
        np.testing.assert_array_equal(_bits(out), _bits(ref), err_msg=f"call {i} {shape}")
    hd.check_errors()


def test_noalloc_rejects_oversized(hd):
    x = torch.zeros((6000, 6000), dtype=torch.uint16, device="cuda")
    out = torch.full(x.shape, -3.0, dtype=torch.float32, device="cuda")
    log("no-alloc oversized")
    with pytest.raises(hd.HDError) as ei:
        hd.hybrid_denoise_noalloc(x, 9, 5, 4095, out=out)
    assert ei.value.name == "HD_ERR_DIMS"
    assert "HD_NOALLOC_SCRATCH_BYTES" in str(ei.value)
    assert bool((out == -3.0).all())
