"""GPU tests of the failure paths that kernels report after their launch: the bounded
waits of the single-launch exchange (forced from the host to give up at once, so every
kernel still ends normally) and the scratch-allocation fault injector."""
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
    hd.check_errors()  # start from a clear error word
    yield hd
    hd.set_option(hd.HD_OPT_WAIT_LIMIT_US, -1)
    hd.set_option(hd.HD_OPT_FAIL_ALLOC, 0)
    hd.set_option(hd.HD_OPT_RESIDENT, -1)
    hd.set_option(hd.HD_OPT_SELECT, -1)
    hd.check_errors()


def _bits(t):
    return to_host(t).view(np.uint32)


@pytest.mark.parametrize("shape,maxv,stretch", [((1600, 1600), 255, False), ((1000, 1300), 4095, False),
                                                ((900, 1100), 255, True)])
def test_resident_wait_timeout_is_reported(hd, shape, maxv, stretch):
    """With the wait bound at zero every workgroup but the last arrival gives up: the launch
    still ends, its pixels are NaN, and hd_check_errors reports HD_ERR_TIMEOUT once. With the
    default bound the next launch is exact again."""
    g = noisy_phantom(shape[0], shape[1], maxv, 20, 0.2, seed=shape[0] + maxv)
    x = to_dev(g, np.uint8 if maxv == 255 else np.uint16)
    dt = torch.uint8 if maxv == 255 else torch.uint16
    # the adaptive strategy (whatever an earlier autotuning chose for this key): its register
    # count lets the whole image take the single launch
    hd.set_option(hd.HD_OPT_SELECT, 0)
    assert hd.tiles_of(*shape) <= hd.resident_capacity(dt, 9, 5, 0), "case must take the single launch"
    hd.set_option(hd.HD_OPT_RESIDENT, 0)
    staged = _bits(hd.hybrid_denoise(x, 9, 5, maxv, stretch=stretch))
    hd.set_option(hd.HD_OPT_RESIDENT, 1)
    hd.check_errors()
    log(f"forced wait timeout {shape} maxv {maxv} stretch {stretch}")
    hd.set_option(hd.HD_OPT_WAIT_LIMIT_US, 0)
    out = hd.hybrid_denoise(x, 9, 5, maxv, stretch=stretch)
    with pytest.raises(hd.HDError) as ei:
        hd.check_errors()
    assert ei.value.name == "HD_ERR_TIMEOUT"
    got = to_host(out)
    assert np.isnan(got).sum() > 0
    hd.check_errors()  # cleared by the previous check
    hd.set_option(hd.HD_OPT_WAIT_LIMIT_US, -1)
    log(f"default wait bound {shape}")
    out = hd.hybrid_denoise(x, 9, 5, maxv, stretch=stretch)
    hd.check_errors()
    np.testing.assert_array_equal(_bits(out), staged)
    hd.set_option(hd.HD_OPT_RESIDENT, -1)
    hd.set_option(hd.HD_OPT_SELECT, -1)


def test_alloc_fault_injector(hd):
    """An injected scratch-allocation failure returns HD_ERR_NOMEM with nothing enqueued (the
    output keeps its contents); the injector then disarms and the same calls succeed."""
    g = noisy_phantom(300, 400, 255, 15, 0.2, seed=11)
    x = to_dev(g, np.uint8)
    ref = _bits(hd.hybrid_denoise(x, 9, 5, 255))
    out = torch.full(x.shape, -2.0, dtype=torch.float32, device="cuda")
    log("fault injector: single call")
    hd.set_option(hd.HD_OPT_FAIL_ALLOC, 1)
    with pytest.raises(hd.HDError) as ei:
        hd.hybrid_denoise(x, 9, 5, 255, out=out)
    assert ei.value.name == "HD_ERR_NOMEM"
    assert np.all(to_host(out) == -2.0)
    hd.hybrid_denoise(x, 9, 5, 255, out=out)
    np.testing.assert_array_equal(_bits(out), ref)
    # the second allocation of a new batched plan (its slice table) fails
    log("fault injector: batched plan")
    ins = [x, to_dev(noisy_phantom(200, 150, 255, 15, 0.2, seed=12), np.uint8)]
    outs = [torch.full(t.shape, -2.0, dtype=torch.float32, device="cuda") for t in ins]
    hd.set_option(hd.HD_OPT_FAIL_ALLOC, 2)
    with pytest.raises(hd.HDError) as ei:
        hd.hybrid_denoise_batched(ins, 9, 5, 255, outs=outs)
    assert ei.value.name == "HD_ERR_NOMEM"
    assert all(np.all(to_host(o) == -2.0) for o in outs)
    hd.hybrid_denoise_batched(ins, 9, 5, 255, outs=outs)
    np.testing.assert_array_equal(_bits(outs[0]), ref)
    with pytest.raises(hd.HDError):
        hd.set_option(hd.HD_OPT_FAIL_ALLOC, -1)
