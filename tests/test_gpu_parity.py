"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar: AMF bit-exact; Wiener / hybrid within 1e-4 absolute in normalised intensity of the
float64 oracle. Inputs are seeded phantoms and random images with the workloads' shapes,
noise levels, Smax and windows, plus edge cases (1-pixel sides, ragged tiles, windows
larger than the image, flat images, extreme values, pitched rows, keep mode).
"""
import numpy as np
import pytest

import oracle
from phantoms import CONFIGS, noisy_phantom, random_image
from tests.gpu_util import gpu_available, log, to_dev, to_host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-4


@pytest.fixture(scope="module")
def hd():
    import paper_2005_05371_amd as hd
    hd.load()
    return hd


def np_dtype(maxv):
    return np.uint8 if maxv <= 255 else np.uint16


SHAPES = [(1, 1), (1, 37), (29, 1), (2, 2), (3, 5), (7, 7), (31, 65), (64, 64), (65, 33),
          (97, 131), (128, 200), (257, 67)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("smax", [3, 5, 7, 15])
@pytest.mark.parametrize("maxv", [255, 4095])
def test_amf_random_shapes(hd, shape, smax, maxv):
    h, w = shape
    for vals, seed in ((None, 1), ([0, 1, 2, maxv], 2)):
        g = random_image(shape, maxv, seed + h * 1000 + w, values=vals)
        for keep in (False, True):
            log(f"amf random {shape} smax={smax} maxv={maxv} vals={vals} keep={keep}")
            ref = oracle.amf(g, smax, keep=keep)
            got = to_host(hd.amf_filter(to_dev(g, np_dtype(maxv)), smax, keep=keep))
            np.testing.assert_array_equal(got.astype(np.int32), ref)


@pytest.mark.parametrize("h,w,smax,maxv,sigma,dens", [
    (512, 512, 7, 255, 10, 0.10),
    (300, 257, 9, 255, 15, 0.20),
    (256, 256, 11, 4095, 40, 0.30),
    (200, 333, 15, 4095, 60, 0.50),
    (129, 190, 31, 255, 25, 0.85),   # extreme density: deep levels, unresolved pixels
    (100, 101, 21, 65535, 900, 0.6),
])
def test_amf_phantoms(hd, h, w, smax, maxv, sigma, dens):
    g = noisy_phantom(h, w, maxv, sigma, dens, seed=h + w + smax)
    for keep in (False, True):
        log(f"amf phantom {h}x{w} smax={smax} maxv={maxv} d={dens} keep={keep}")
        ref = oracle.amf(g, smax, keep=keep)
        got = to_host(hd.amf_filter(to_dev(g, np_dtype(maxv)), smax, keep=keep))
        np.testing.assert_array_equal(got.astype(np.int32), ref)


@pytest.mark.parametrize("value", [0, 1, 77, 255])
@pytest.mark.parametrize("smax", [3, 9, 31])
def test_amf_constant_unchanged(hd, value, smax):
    g = np.full((70, 130), value, np.int32)
    log(f"amf constant {value} smax={smax}")
    got = to_host(hd.amf_filter(to_dev(g, np.uint8), smax))
    np.testing.assert_array_equal(got, g.astype(np.uint8))


def test_amf_pitched(hd):
    g = noisy_phantom(90, 100, 4095, 40, 0.3, seed=5)
    log("amf pitched")
    inp = to_dev(g, np.uint16, pitch=160)
    import torch
    out_big = torch.zeros((90, 144), dtype=torch.uint16, device="cuda")
    out = out_big[:, :100]
    hd.amf_filter(inp, 11, out=out)
    np.testing.assert_array_equal(to_host(out).astype(np.int32), oracle.amf(g, 11))
    assert (to_host(out_big)[:, 100:] == 0).all()  # nothing written past the width


@pytest.mark.parametrize("shape", [(1, 1), (1, 40), (33, 1), (5, 5), (64, 64), (77, 130), (200, 257)])
@pytest.mark.parametrize("win", [1, 3, 5, 7, 15])
@pytest.mark.parametrize("maxv", [255, 4095, 65535])
def test_wiener_random(hd, shape, win, maxv):
    a = random_image(shape, maxv, 7 + shape[0] * 3 + shape[1] + win)
    dt = np_dtype(maxv)
    for noise in (-1.0, 0.0, 123.0, 1e12):
        log(f"wiener random {shape} win={win} maxv={maxv} noise={noise}")
        ref, nu2 = oracle.wiener(a, (win, win), maxv, noise, return_nu2=True)
        import torch
        nu = torch.zeros(1, dtype=torch.float64, device="cuda")
        got = to_host(hd.wiener_filter(to_dev(a, dt), win, maxv, noise, nu2_out=nu))
        assert np.max(np.abs(got - ref)) <= TOL
        assert abs(float(nu.item()) - nu2) <= 1e-9 * max(1.0, nu2)


def test_wiener_rectangular_window(hd):
    a = random_image((60, 90), 255, 99)
    for win in ((3, 7), (7, 3), (1, 5), (15, 1)):
        log(f"wiener window {win}")
        ref = oracle.wiener(a, win, 255)
        got = to_host(hd.wiener_filter(to_dev(a, np.uint8), win, 255))
        assert np.max(np.abs(got - ref)) <= TOL


def _extreme_u16(kind, shape, seed):
    rng = np.random.default_rng(seed)
    h, w = shape
    if kind == "max":
        return np.full(shape, 65535, np.int32)
    if kind == "checker":
        return (((np.arange(h)[:, None] + np.arange(w)[None, :]) & 1) * 65535).astype(np.int32)
    if kind == "binary":
        return (rng.integers(0, 2, shape) * 65535).astype(np.int32)
    return rng.integers(65000, 65536, shape).astype(np.int32)  # "high"


@pytest.mark.parametrize("kind", ["max", "checker", "binary", "high"])
@pytest.mark.parametrize("win", [(15, 15), (15, 1), (1, 15), (7, 7)])
def test_wiener_extreme_u16_sums(hd, kind, win):
    """16-bit windows at the top of the sums' ranges: S1 up to 225 * 65535 (just under
    2^24) and S2 up to 225 * 65535^2 (just under 2^40), the bounds the 24-bit partial
    products of the window numerator rely on; also samples with v^2 >= 2^31."""
    a = _extreme_u16(kind, (70, 150), 11 + win[0] * 16 + win[1])
    log(f"wiener extreme u16 {kind} win={win}")
    import torch
    for noise in (-1.0, 0.0):
        ref, nu2 = oracle.wiener(a, win, 65535, noise, return_nu2=True)
        nu = torch.zeros(1, dtype=torch.float64, device="cuda")
        got = to_host(hd.wiener_filter(to_dev(a, np.uint16), win, 65535, noise, nu2_out=nu))
        assert np.max(np.abs(got - ref)) <= TOL
        assert abs(float(nu.item()) - nu2) <= 1e-9 * max(1.0, nu2)
    # the resident single-launch hybrid (AMF on the window ring, then the same sums)
    ref = oracle.hybrid(a, 3, win, 65535)[0]
    got = to_host(hd.hybrid_denoise(to_dev(a, np.uint16), 3, win, 65535))
    assert np.max(np.abs(got - ref)) <= TOL


def _narrow_max(n):
    """Largest 16-bit value v with n * v^2 < 2^32 (above it a window's S2 needs 64 bits)."""
    v = 0
    while (v + 1) <= 65535 and n * (v + 1) ** 2 <= 0xFFFFFFFF:
        v += 1
    return v


@pytest.mark.parametrize("win", [7, 15, 3])
def test_wiener_narrow_wide_boundary(hd, win):
    """16-bit tiles take 32-bit sums of squares only while their largest sample keeps
    N * max^2 below 2^32, else 64-bit ones. Images straddling the bound (tiles just below it,
    tiles just above it, and a slice mixing both, whose noise power sums both kinds of tile)
    match the oracle; so does the stand-alone Wiener filter with a given noise power."""
    import torch
    n = win * win
    v = _narrow_max(n)
    rng = np.random.default_rng(win)
    below = rng.integers(v - 300, v + 1, (96, 200))
    above = rng.integers(v - 300, v + 1, (96, 200))
    above[::17, ::13] = v + 1  # one sample past the bound in many tiles
    mixed = below.copy()
    mixed[:, 128:] = above[:, 128:]
    for name, a in (("below", below), ("above", above), ("mixed", mixed)):
        for noise in (-1.0, 5000.0):
            log(f"wiener narrow/wide {name} win={win} noise={noise}")
            ref, nu2 = oracle.wiener(a, (win, win), 65535, noise, return_nu2=True)
            nu = torch.zeros(1, dtype=torch.float64, device="cuda")
            got = to_host(hd.wiener_filter(to_dev(a, np.uint16), win, 65535, noise, nu2_out=nu))
            assert np.max(np.abs(got - ref)) <= TOL
            assert abs(float(nu.item()) - nu2) <= 1e-9 * max(1.0, nu2)


@pytest.mark.parametrize("value", [0, 200, 4095])
def test_hybrid_constant_unchanged(hd, value):
    g = np.full((50, 70), value, np.int32)
    log(f"hybrid constant {value}")
    got = to_host(hd.hybrid_denoise(to_dev(g, np.uint16), 11, 5, 4095))
    np.testing.assert_array_equal(got, np.float32(value / 4095.0) * np.ones_like(got))


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_hybrid_full_size_single(hd, name):
    """The single-image workloads at their full size, as the benchmark runs them."""
    import torch
    wl = CONFIGS[name]
    s = wl.make_slice(0)
    log(f"hybrid full {name} {wl.shapes[0]}")
    ref, a_ref, nu2 = oracle.hybrid(s.noisy, wl.smax, wl.win, wl.max_value)
    inp = to_dev(s.noisy, wl.np_dtype)
    a = torch.empty_like(inp)
    nu = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = hd.hybrid_denoise(inp, wl.smax, wl.win, wl.max_value, amf_out=a, nu2_out=nu)
    np.testing.assert_array_equal(to_host(a).astype(np.int32), a_ref)
    assert abs(float(nu.item()) - nu2) <= 1e-9 * nu2
    assert np.max(np.abs(to_host(out) - ref)) <= TOL


def test_hybrid_stress_slice(hd):
    """One full 4096^2 12-bit slice of the stress workload (Smax 15, Wiener 7x7, d 0.5)."""
    import torch
    wl = CONFIGS["c5"]
    s = wl.make_slice(0)
    log("hybrid stress slice 4096^2")
    ref, a_ref, nu2 = oracle.hybrid(s.noisy, wl.smax, wl.win, wl.max_value)
    inp = to_dev(s.noisy, np.uint16)
    a = torch.empty_like(inp)
    out = hd.hybrid_denoise(inp, wl.smax, wl.win, wl.max_value, amf_out=a)
    np.testing.assert_array_equal(to_host(a).astype(np.int32), a_ref)
    assert np.max(np.abs(to_host(out) - ref)) <= TOL


def test_hybrid_batched_workload_slices(hd):
    """A few slices of each size of the uneven 12-bit batch, one call per slice."""
    wl = CONFIGS["c3"]
    for i in (0, 95, 96, 150, 208, 255):
        s = wl.make_slice(i)
        log(f"hybrid c3 slice {i} {s.noisy.shape}")
        ref, a_ref, nu2 = oracle.hybrid(s.noisy, wl.smax, wl.win, wl.max_value)
        got = to_host(hd.hybrid_denoise(to_dev(s.noisy, np.uint16), wl.smax, wl.win, wl.max_value))
        assert np.max(np.abs(got - ref)) <= TOL


def test_hybrid_keep_mode_and_given_noise(hd):
    g = noisy_phantom(150, 170, 255, 20, 0.7, seed=3)
    for keep in (False, True):
        for noise in (-1.0, 50.0):
            log(f"hybrid keep={keep} noise={noise}")
            ref, a_ref, _ = oracle.hybrid(g, 7, 5, 255, noise_var=noise, keep=keep)
            got = to_host(hd.hybrid_denoise(to_dev(g, np.uint8), 7, 5, 255, noise_var=noise, keep=keep))
            assert np.max(np.abs(got - ref)) <= TOL


def test_deterministic_repeat(hd):
    g = noisy_phantom(700, 900, 4095, 60, 0.5, seed=8)
    inp = to_dev(g, np.uint16)
    log("determinism")
    a = to_host(hd.hybrid_denoise(inp, 15, 7, 4095))
    b = to_host(hd.hybrid_denoise(inp, 15, 7, 4095))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("maxv,dt", [(255, np.uint8), (4095, np.uint16), (65535, np.uint16)])
def test_flat_blocks_exact(hd, maxv, dt):
    """Every grey level on a flat 16 x 16 block: inside each block the window is flat, so
    the Wiener output must be exactly float32(v / max_value)."""
    levels = np.arange(0, maxv + 1, max(1, (maxv + 1) // 4096), dtype=np.int64)
    nb = int(np.ceil(np.sqrt(len(levels))))
    vals = np.zeros(nb * nb, np.int64)
    vals[:len(levels)] = levels
    img = np.kron(vals.reshape(nb, nb), np.ones((16, 16), np.int64)).astype(np.int32)
    log(f"flat blocks maxv={maxv} {img.shape}")
    out = to_host(hd.hybrid_denoise(to_dev(img, dt), 5, 5, maxv))
    centres = out[8::16, 8::16].ravel()[:len(levels)]
    expect = (levels / maxv).astype(np.float32)
    np.testing.assert_array_equal(centres, expect)
