"""Pins for the CPU oracle's adaptive median filter (no GPU).

Each test checks the oracle against something other than itself:
  * a brute-force per-pixel implementation built on numpy's own symmetric padding;
  * the whole-image formulation of the paper's level loop (Alg. 1, parallelAdapMedian:
    per-level min / max / median images and boolean masks), with the order statistics
    taken from scipy.ndimage (mode 'reflect' is the same half-sample mirror);
  * closed forms and invariants the method fixes (constant image, stage-B pixel kept,
    Smax = 3 on an image of distinct values).
"""
import itertools

import numpy as np
import pytest
import scipy.ndimage as ndi

from phantoms import noisy_phantom, random_image


def brute_amf(g, smax, keep=False):
    """Per-pixel AMF with numpy's 'symmetric' pad and Python's sorted()."""
    g = np.asarray(g, dtype=np.int64)
    h, w = g.shape
    R = smax // 2
    p = np.pad(g, R, mode="symmetric")
    out = g.copy()
    lvl = np.zeros_like(g)
    for y in range(h):
        for x in range(w):
            c = int(g[y, x])
            zmed = None
            for k in range(3, smax + 1, 2):
                r = k // 2
                vals = sorted(int(v) for v in p[y + R - r:y + R + r + 1, x + R - r:x + R + r + 1].ravel())
                lo, med, hi = vals[0], vals[len(vals) // 2], vals[-1]
                zmed = med
                if lo < med < hi:
                    out[y, x] = c if lo < c < hi else med
                    lvl[y, x] = k
                    break
            else:
                out[y, x] = c if keep else zmed
    return out, lvl


def masks_amf(g, smax, keep=False):
    """Whole-image AMF: per level, min / max / median images and masks over all pixels.

    Pixels that pass the level test for the first time are written (centre value when
    it is not an extreme of the window, else the window median) and frozen.
    """
    g = np.asarray(g, dtype=np.int64)
    out = g.copy()
    done = np.zeros(g.shape, dtype=bool)
    last_med = g.copy()
    for k in range(3, smax + 1, 2):
        lo = ndi.minimum_filter(g, size=k, mode="reflect")
        hi = ndi.maximum_filter(g, size=k, mode="reflect")
        med = ndi.median_filter(g, size=k, mode="reflect")
        last_med = med
        newly = (lo < med) & (med < hi) & ~done
        centre_ok = (lo < g) & (g < hi)
        out[newly & centre_ok] = g[newly & centre_ok]
        out[newly & ~centre_ok] = med[newly & ~centre_ok]
        done |= newly
        if done.all():
            break
    if not keep:
        out[~done] = last_med[~done]  # the loop ran to Smax when any pixel is left
    return out, done


def masks_amf_stack(stack, smax, keep=False):
    """Same whole-image form on a stack (N, H, W); the window never crosses images."""
    g = np.asarray(stack, dtype=np.int64)
    out = g.copy()
    done = np.zeros(g.shape, dtype=bool)
    last_med = g.copy()
    for k in range(3, smax + 1, 2):
        sz = (1, k, k)
        lo = ndi.minimum_filter(g, size=sz, mode="reflect")
        hi = ndi.maximum_filter(g, size=sz, mode="reflect")
        med = ndi.median_filter(g, size=sz, mode="reflect")
        last_med = med
        newly = (lo < med) & (med < hi) & ~done
        centre_ok = (lo < g) & (g < hi)
        out[newly & centre_ok] = g[newly & centre_ok]
        out[newly & ~centre_ok] = med[newly & ~centre_ok]
        done |= newly
    if not keep:
        out[~done] = last_med[~done]
    return out


def test_mirror_matches_numpy_symmetric(orc):
    for n in range(1, 7):
        row = np.arange(n)
        for pad in (1, 3, 8, 15):
            p = np.pad(row, pad, mode="symmetric")
            got = [orc.mirror(i, n) for i in range(-pad, n + pad)]
            assert got == list(p), (n, pad)


@pytest.mark.parametrize("smax", [3, 5, 7, 9])
def test_bruteforce_tiny_with_ties(orc, smax):
    """All shapes 1..9 x 1..9 (windows wider than the image included), values forcing ties."""
    seed = 0
    for h in range(1, 10):
        for w in range(1, 10):
            for vals in ([0, 1, 2, 255], None):
                seed += 1
                g = random_image((h, w), 255, seed, values=vals)
                for keep in (False, True):
                    ref, ref_lvl = brute_amf(g, smax, keep)
                    got, lvl = orc.amf(g, smax, keep=keep, return_level=True)
                    np.testing.assert_array_equal(got, ref, err_msg=f"{h}x{w} smax={smax} keep={keep}")
                    np.testing.assert_array_equal(lvl, ref_lvl)


@pytest.mark.parametrize("smax", [3, 5])
def test_exhaustive_3x3_ternary(orc, smax):
    """Every 3x3 image over {0, 1, 2}: 19683 images, checked against the mask form."""
    imgs = np.array(list(itertools.product([0, 1, 2], repeat=9)), dtype=np.int32).reshape(-1, 3, 3)
    for keep in (False, True):
        ref = masks_amf_stack(imgs, smax, keep)
        # the oracle filters each image on its own; tile them with a separator-free
        # batch by calling it per image
        got = np.stack([orc.amf(im, smax, keep=keep, threads=1) for im in imgs])
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("h,w,smax,maxv,sigma,dens,seed", [
    (512, 512, 7, 255, 10, 0.10, 1),        # the 512^2 u8 workload's parameters
    (160, 200, 9, 255, 15, 0.20, 2),        # the 1600^2 workload's parameters, smaller image
    (96, 128, 11, 4095, 40, 0.30, 3),       # 12-bit, Smax 11
    (64, 80, 15, 4095, 60, 0.50, 4),        # 12-bit stress parameters
    (37, 53, 15, 255, 25, 0.70, 5),         # very dense impulses: unresolved pixels
])
def test_against_whole_image_mask_form(orc, h, w, smax, maxv, sigma, dens, seed):
    g = noisy_phantom(h, w, maxv, sigma, dens, seed)
    for keep in (False, True):
        ref, done = masks_amf(g, smax, keep)
        got, lvl = orc.amf(g, smax, keep=keep, return_level=True)
        np.testing.assert_array_equal(got, ref)
        np.testing.assert_array_equal(lvl > 0, done)


@pytest.mark.parametrize("smax", [3, 5, 7, 11, 15])
@pytest.mark.parametrize("value", [0, 1, 128, 255, 4095, 65535])
def test_constant_image_unchanged(orc, smax, value):
    for shape in [(1, 1), (1, 7), (5, 1), (9, 13), (32, 33)]:
        g = np.full(shape, value, dtype=np.int32)
        for keep in (False, True):
            out, lvl = orc.amf(g, smax, keep=keep, return_level=True)
            np.testing.assert_array_equal(out, g)
            assert (lvl == 0).all()  # a flat window never passes stage A


def test_stage_b_pixel_kept(orc):
    """A centre value strictly inside (zmin, zmax) of a 3x3 window of distinct values
    passes both stages at k = 3 and is kept."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        g = rng.permutation(400).reshape(20, 20).astype(np.int32)
        out, lvl = orc.amf(g, 7, return_level=True)
        lo = ndi.minimum_filter(g, 3, mode="reflect")
        hi = ndi.maximum_filter(g, 3, mode="reflect")
        inner = (lo < g) & (g < hi)
        assert (lvl == 3).all()
        np.testing.assert_array_equal(out[inner], g[inner])


@pytest.mark.parametrize("h,w", [(2, 2), (2, 9), (7, 3), (16, 16), (31, 17)])
def test_smax3_distinct_values_closed_form(orc, h, w):
    """Smax = 3, all values distinct, H, W >= 2: each value occurs at most 4 times in a
    mirrored 3x3 window, so stage A always passes at k = 3 and the output is g when g is
    not an extreme of its window, else the 3x3 median."""
    rng = np.random.default_rng(h * 100 + w)
    g = rng.permutation(h * w).astype(np.int32).reshape(h, w) * 3 + 1
    lo = ndi.minimum_filter(g, 3, mode="reflect")
    hi = ndi.maximum_filter(g, 3, mode="reflect")
    med = ndi.median_filter(g, 3, mode="reflect")
    expect = np.where((lo < g) & (g < hi), g, med)
    out, lvl = orc.amf(g, 3, return_level=True)
    assert (lvl == 3).all()
    np.testing.assert_array_equal(out, expect)


def test_impulse_in_flat_region(orc):
    """An isolated impulse in a flat region: stage A fails at 3 (median = flat value =
    min), so the window grows; with an all-flat neighbourhood it never passes, and the
    default reading outputs the Smax median (the flat value) while keep-mode leaves it."""
    g = np.full((15, 15), 100, dtype=np.int32)
    g[7, 7] = 255
    out = orc.amf(g, 7)
    assert out[7, 7] == 100
    out_keep = orc.amf(g, 7, keep=True)
    assert out_keep[7, 7] == 255
    # a textured neighbourhood resolves the impulse to the window median at k = 3
    g2 = np.arange(225, dtype=np.int32).reshape(15, 15)
    g2[7, 7] = 10_000
    out2, lvl2 = orc.amf(g2, 7, return_level=True)
    win = g2[6:9, 6:9].ravel()
    assert lvl2[7, 7] == 3 and out2[7, 7] == int(np.sort(win)[4])


def test_bad_smax_rejected(orc):
    g = np.zeros((4, 4), np.int32)
    for bad in (1, 0, -3, 4, 10):
        with pytest.raises(ValueError, match="SMAX"):
            orc.amf(g, bad)


def test_level_histogram_sums_to_one(orc):
    g = noisy_phantom(128, 128, 4095, 60, 0.5, 11)
    _, lvl = orc.amf(g, 15, return_level=True)
    hist = orc.level_histogram(lvl, 15)
    assert abs(sum(hist.values()) - 1.0) < 1e-12
    e = orc.window_elements_per_pixel(lvl, 15)
    assert 9.0 <= e <= sum(k * k for k in range(3, 16, 2))


def test_level_counts_hand_map(orc):
    """A hand-written level map at Smax 7 (0 = never resolved): the pixel resolved at 3
    is tested at 3 only (9 elements); at 5, at 3 and 5 (9 + 25); at 7 and never
    resolved, at all three levels (9 + 25 + 49 = 83). Counting only the resolving
    level, or skipping the unresolved pixel's last level, gives another mean."""
    lvl = np.array([[3, 5], [0, 7]], dtype=np.int32)
    assert orc.window_elements_per_pixel(lvl, 7) == (9 + 34 + 83 + 83) / 4
    assert orc.level_histogram(lvl, 7) == {3: 0.25, 5: 0.25, 7: 0.25, 0: 0.25}
    # a larger Smax adds levels only for the pixel that never resolved
    assert orc.window_elements_per_pixel(lvl, 9) == (9 + 34 + 83 + 83 + 81) / 4


def test_level_counts_smax3_closed_form(orc):
    """Smax = 3: every pixel is tested at level 3 only, resolved or not: exactly 9."""
    g = np.random.default_rng(5).permutation(24 * 31).reshape(24, 31).astype(np.int32)
    _, lvl = orc.amf(g, 3, return_level=True)
    assert orc.window_elements_per_pixel(lvl, 3) == 9.0
    g2 = np.full((6, 7), 9, np.int32)  # never resolves: still one level tested
    _, lvl2 = orc.amf(g2, 3, return_level=True)
    assert np.all(lvl2 == 0) and orc.window_elements_per_pixel(lvl2, 3) == 9.0


def _brute_elements(g, smax):
    """Window elements the level loop visits, counted while it runs: k^2 added at every
    level a pixel is tested at, per pixel, with numpy's symmetric pad."""
    g = np.asarray(g, dtype=np.int64)
    h, w = g.shape
    R = smax // 2
    p = np.pad(g, R, mode="symmetric")
    total = 0
    hist = {k: 0 for k in range(3, smax + 1, 2)}
    hist[0] = 0
    for y in range(h):
        for x in range(w):
            for k in range(3, smax + 1, 2):
                r = k // 2
                vals = sorted(int(v) for v in p[y + R - r:y + R + r + 1, x + R - r:x + R + r + 1].ravel())
                total += len(vals)
                if vals[0] < vals[len(vals) // 2] < vals[-1]:
                    hist[k] += 1
                    break
            else:
                hist[0] += 1
    return total / (h * w), {k: v / (h * w) for k, v in hist.items()}


@pytest.mark.parametrize("smax,sigma,d,seed", [(15, 60, 0.5, 3), (9, 15, 0.3, 4), (11, 40, 0.7, 5)])
def test_level_counts_brute_force(orc, smax, sigma, d, seed):
    """The oracle's level map turned into work counts equals a count taken inside an
    independent per-pixel loop, on dense impulse noise where deep levels occur."""
    g = noisy_phantom(20, 23, 4095, sigma, d, seed)
    _, lvl = orc.amf(g, smax, return_level=True)
    e_ref, h_ref = _brute_elements(g, smax)
    assert abs(orc.window_elements_per_pixel(lvl, smax) - e_ref) < 1e-12
    h = orc.level_histogram(lvl, smax)
    assert h.keys() == h_ref.keys()
    for k in h:
        assert abs(h[k] - h_ref[k]) < 1e-12
    assert h_ref[5] > 0 and e_ref > 9.0  # deep levels were exercised
