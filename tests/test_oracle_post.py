"""Pins of the oracle's post-processing and partition steps (Alg. 1 steps b and e):
invariants that a dropped term, a wrong sign or a shifted cut would break."""
import numpy as np
import pytest

import oracle
from phantoms import noisy_phantom


def test_contrast_stretch_spans_unit_interval():
    rng = np.random.default_rng(1)
    y = rng.uniform(0.13, 0.71, size=(37, 53))
    s = oracle.contrast_stretch(y)
    assert s.min() == 0.0 and s.max() == 1.0
    # the extreme pixels are the ones that land on 0 and 1
    assert s.flat[np.argmin(y)] == 0.0 and s.flat[np.argmax(y)] == 1.0


def test_contrast_stretch_affine_invariant_and_monotone():
    rng = np.random.default_rng(2)
    y = rng.uniform(0, 1, size=(41, 29))
    s = oracle.contrast_stretch(y)
    for a, b in [(3.5, -1.25), (0.01, 7.0), (1.0, 0.5)]:
        np.testing.assert_allclose(oracle.contrast_stretch(a * y + b), s, rtol=0, atol=1e-12)
    order = np.argsort(y, axis=None, kind="stable")
    assert np.all(np.diff(s.flat[order]) >= 0)
    # strictly affine in y: equal steps in y give equal steps in the output
    lin = np.linspace(0.2, 0.8, 13).reshape(1, 13)
    np.testing.assert_allclose(np.diff(oracle.contrast_stretch(lin)), 1 / 12, atol=1e-12)


def test_contrast_stretch_constant_unchanged():
    y = np.full((5, 7), 0.375)
    np.testing.assert_array_equal(oracle.contrast_stretch(y), y)


@pytest.mark.parametrize("h,parts", [(10, 2), (11, 4), (1600, 8), (3, 8), (7, 7)])
def test_strip_bounds_tile_the_rows(h, parts):
    b = oracle.strip_bounds(h, parts)
    assert len(b) == parts and b[0][0] == 0 and b[-1][1] == h
    assert all(b[i][1] == b[i + 1][0] for i in range(parts - 1))
    sizes = [r1 - r0 for r0, r1 in b]
    assert max(sizes) - min(sizes) <= 1 and min(sizes) >= 0


@pytest.mark.parametrize("parts", [1, 2, 4, 8])
def test_partitioned_amf_matches_whole_image_away_from_cuts(parts):
    """One partition is the whole-image filter; with more, every pixel whose largest window
    stays inside its strip is unchanged, and pixels next to a cut are filtered as at an
    image border (they differ from the whole-image result somewhere)."""
    smax = 7
    g = noisy_phantom(96, 80, 255, 20, 0.3, seed=11)
    whole = oracle.amf(g, smax)
    part = oracle.amf_partitioned(g, smax, parts)
    if parts == 1:
        np.testing.assert_array_equal(part, whole)
        return
    r = smax // 2
    cuts = [r0 for r0, _ in oracle.strip_bounds(g.shape[0], parts)[1:]]
    far = np.ones(g.shape[0], bool)
    for c in cuts:
        far[max(0, c - r):c + r] = False
    np.testing.assert_array_equal(part[far], whole[far])
    assert np.any(part[~far] != whole[~far])
    # each strip is the filter of that strip as an image of its own
    for r0, r1 in oracle.strip_bounds(g.shape[0], parts):
        np.testing.assert_array_equal(part[r0:r1], oracle.amf(g[r0:r1], smax))


def test_partitioned_amf_constant_image():
    g = np.full((33, 17), 140, np.int32)
    np.testing.assert_array_equal(oracle.amf_partitioned(g, 9, 4), g)
