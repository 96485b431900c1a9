"""GPU tests of the batched path (one work list over many uneven slices, captured graph,
replays) and of the interchangeable strategies (selection networks vs bisection, fused vs
separate noise sums): every variant must give bit-identical results, and match the oracle."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from phantoms import CONFIGS, noisy_phantom
from tests.gpu_util import gpu_available, log, to_dev, to_host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-4


@pytest.fixture(scope="module")
def hd():
    import paper_2005_05371_amd as hd
    hd.load()
    yield hd
    for k in (hd.HD_OPT_SELECT, hd.HD_OPT_FUSE_MOMENTS, hd.HD_OPT_RESIDENT, hd.HD_OPT_TILE_ROWS):
        hd.set_option(k, -1)
    hd.set_option(hd.HD_OPT_GRAPHS, 1)
    hd.release_plans()


def _bits(t):
    return to_host(t).view(np.uint32)


@pytest.mark.parametrize("smax,win,maxv,dens", [(7, 3, 255, 0.3), (11, 5, 4095, 0.5), (15, 7, 4095, 0.6),
                                               (9, 5, 255, 0.85)])
def test_strategies_bit_identical(hd, smax, win, maxv, dens):
    g = noisy_phantom(300, 421, maxv, 30, dens, seed=smax * 7 + win)
    dt = np.uint8 if maxv == 255 else np.uint16
    inp = to_dev(g, dt)
    ref = None
    ref_a = None
    # tile heights other than 32 apply to the staged, unfused AMF stage only
    cases = [(sel, fuse, res, 32) for sel, fuse, res in itertools.product((0, 1, 2, 3), (1, 0), (1, 0))]
    cases += [(sel, 0, 0, rows) for sel in (0, 1, 2, 3) for rows in (16, 64)]
    for sel, fuse, res, rows in cases:
        log(f"strategy select={sel} fuse={fuse} resident={res} rows={rows} smax={smax} win={win}")
        hd.set_option(hd.HD_OPT_SELECT, sel)
        hd.set_option(hd.HD_OPT_FUSE_MOMENTS, fuse)
        hd.set_option(hd.HD_OPT_RESIDENT, res)
        hd.set_option(hd.HD_OPT_TILE_ROWS, rows)
        a = torch.empty_like(inp)
        out = hd.hybrid_denoise(inp, smax, win, maxv, amf_out=a)
        am = hd.amf_filter(inp, smax)
        if ref is None:
            ref, ref_a = _bits(out), to_host(a)
            o_ref, a_orc, _ = oracle.hybrid(g, smax, win, maxv)
            np.testing.assert_array_equal(ref_a.astype(np.int32), a_orc)
            assert np.max(np.abs(to_host(out) - o_ref)) <= TOL
        else:
            np.testing.assert_array_equal(_bits(out), ref)
            np.testing.assert_array_equal(to_host(a), ref_a)
        np.testing.assert_array_equal(to_host(am), ref_a)
    hd.set_option(hd.HD_OPT_SELECT, -1)
    hd.set_option(hd.HD_OPT_FUSE_MOMENTS, -1)
    hd.set_option(hd.HD_OPT_RESIDENT, -1)
    hd.set_option(hd.HD_OPT_TILE_ROWS, -1)


@pytest.mark.parametrize("rows", [16, 64])
def test_tile_rows_batched_uneven(hd, rows):
    """Batched uneven slices (1-row, tile-height-ragged, single-tile and multi-tile shapes)
    with 16- and 64-row AMF tiles give the 32-row result to the bit, and the AMF equals the
    oracle's."""
    imgs = [noisy_phantom(h, w, 4095, 40, 0.4, seed=90 + i)
            for i, (h, w) in enumerate([(1, 70), (17, 33), (33, 64), (65, 129), (200, 131), (96, 64), (31, 300)])]
    ins = [to_dev(g, np.uint16) for g in imgs]
    hd.set_option(hd.HD_OPT_RESIDENT, 0)
    hd.set_option(hd.HD_OPT_FUSE_MOMENTS, 0)
    try:
        hd.set_option(hd.HD_OPT_TILE_ROWS, 32)
        log(f"tile rows 32 (reference) for {rows}")
        ref = [to_host(o).view(np.uint32) for o in hd.hybrid_denoise_batched(ins, 11, 5, 4095)]
        hd.set_option(hd.HD_OPT_TILE_ROWS, rows)
        log(f"tile rows {rows}")
        got = [to_host(o).view(np.uint32) for o in hd.hybrid_denoise_batched(ins, 11, 5, 4095)]
        for i, (a, b) in enumerate(zip(got, ref)):
            np.testing.assert_array_equal(a, b, err_msg=f"slice {i}")
        for i, (g, x) in enumerate(zip(imgs, ins)):
            am = to_host(hd.amf_filter(x, 11)).astype(np.int32)  # amf_filter keeps 32-row tiles
            ab = torch.empty_like(x)
            hd.hybrid_denoise(x, 11, 5, 4095, amf_out=ab)
            np.testing.assert_array_equal(to_host(ab).astype(np.int32), oracle.amf(g, 11), err_msg=f"slice {i}")
            np.testing.assert_array_equal(am, oracle.amf(g, 11))
    finally:
        for k in (hd.HD_OPT_RESIDENT, hd.HD_OPT_FUSE_MOMENTS, hd.HD_OPT_TILE_ROWS):
            hd.set_option(k, -1)
        hd.release_plans()


def _uneven_batch(n, maxv, seed):
    rng = np.random.default_rng(seed)
    imgs = []
    for i in range(n):
        h, w = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        if i % 5 == 0:
            h, w = int(rng.integers(1, 4)), int(rng.integers(1, 70))  # degenerate shapes
        imgs.append(noisy_phantom(h, w, maxv, 25, float(rng.uniform(0.05, 0.6)), seed=seed * 1000 + i))
    return imgs


@pytest.mark.parametrize("graphs", [1, 0])
def test_batched_equals_single_and_oracle(hd, graphs):
    hd.set_option(hd.HD_OPT_GRAPHS, graphs)
    imgs = _uneven_batch(23, 4095, seed=5 + graphs)
    ins = [to_dev(g, np.uint16) for g in imgs]
    log(f"batched uneven graphs={graphs}")
    outs = hd.hybrid_denoise_batched(ins, 11, 5, 4095)
    for i, (g, x) in enumerate(zip(imgs, ins)):
        single = hd.hybrid_denoise(x, 11, 5, 4095)
        np.testing.assert_array_equal(_bits(outs[i]), _bits(single), err_msg=f"slice {i} {g.shape}")
        ref, _, _ = oracle.hybrid(g, 11, 5, 4095)
        assert np.max(np.abs(to_host(outs[i]) - ref)) <= TOL, f"slice {i}"
    hd.set_option(hd.HD_OPT_GRAPHS, 1)


def test_graph_replays_match_eager(hd):
    """Replays of the captured graph, with other device work in between, all equal the
    eager result."""
    imgs = _uneven_batch(9, 255, seed=77)
    ins = [to_dev(g, np.uint8) for g in imgs]
    outs = [torch.empty(x.shape, dtype=torch.float32, device="cuda") for x in ins]
    hd.set_option(hd.HD_OPT_GRAPHS, 0)
    log("graph replay: eager reference")
    eager = [_bits(o) for o in hd.hybrid_denoise_batched(ins, 9, 5, 255)]
    hd.set_option(hd.HD_OPT_GRAPHS, 1)
    for rep in range(4):
        log(f"graph replay {rep}")
        for o in outs:
            o.fill_(-1.0)
        hd.hybrid_denoise_batched(ins, 9, 5, 255, outs=outs)
        junk = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
        torch.cuda.synchronize()
        del junk
        for i, o in enumerate(outs):
            np.testing.assert_array_equal(_bits(o), eager[i], err_msg=f"replay {rep} slice {i}")


@pytest.mark.parametrize("shape,maxv", [((1600, 1600), 255), ((1000, 1300), 4095), ((600, 700), 65535),
                                        ((2900, 2900), 255)])
def test_resident_matches_staged(hd, shape, maxv):
    """One resident launch (grid-wide noise exchange) equals the staged launches to the
    bit, on images that fit the device at once (1600^2: 1250 tiles) and on one that does
    not (2900^2: the library falls back to the staged launches); repeated launches reuse
    the synchronisation words. The fitting cases take both exchange forms: count and sum
    packed in one word per group (8-bit data), and partials read back (16-bit data, whose
    sum could overflow the packed word)."""
    g = noisy_phantom(shape[0], shape[1], maxv, 20, 0.2, seed=shape[0] + maxv)
    x = to_dev(g, np.uint8 if maxv == 255 else np.uint16)
    hd.set_option(hd.HD_OPT_RESIDENT, 0)
    log(f"resident vs staged {shape}: staged")
    staged = _bits(hd.hybrid_denoise(x, 9, 5, maxv))
    staged_b = _bits(hd.hybrid_denoise_batched([x], 9, 5, maxv)[0])
    np.testing.assert_array_equal(staged_b, staged)
    hd.set_option(hd.HD_OPT_RESIDENT, 1)
    outs = [torch.empty(x.shape, dtype=torch.float32, device="cuda")]
    for rep in range(3):
        log(f"resident vs staged {shape}: resident rep {rep}")
        np.testing.assert_array_equal(_bits(hd.hybrid_denoise(x, 9, 5, maxv)), staged)
        outs[0].fill_(-1.0)
        hd.hybrid_denoise_batched([x], 9, 5, maxv, outs=outs)
        np.testing.assert_array_equal(_bits(outs[0]), staged)
    hd.set_option(hd.HD_OPT_RESIDENT, -1)
    ref, _, _ = oracle.hybrid(g, 9, 5, maxv) if shape[0] <= 1600 else (None, None, None)
    if ref is not None:
        assert np.max(np.abs(to_host(outs[0]) - ref)) <= TOL


def test_resident_alternating_sizes(hd):
    """Resident launches of different grid sizes share the library's barrier words: every
    workgroup's release word only ever changes by exclusive-or, so words that a smaller
    launch leaves alone stay consistent for the next larger one. Each launch equals the
    staged result to the bit."""
    shapes = [(1600, 1600), (700, 500), (1600, 1600), (96, 2000), (1200, 1300), (700, 500)]
    imgs = [noisy_phantom(h, w, 255, 15, 0.2, seed=300 + i) for i, (h, w) in enumerate(shapes)]
    xs = [to_dev(g, np.uint8) for g in imgs]
    hd.set_option(hd.HD_OPT_RESIDENT, 0)
    staged = [_bits(hd.hybrid_denoise(x, 9, 5, 255)) for x in xs]
    hd.set_option(hd.HD_OPT_RESIDENT, 1)
    for rep in range(2):
        for i, x in enumerate(xs):
            log(f"resident alternating sizes rep {rep} {tuple(x.shape)}")
            np.testing.assert_array_equal(_bits(hd.hybrid_denoise(x, 9, 5, 255)), staged[i],
                                          err_msg=f"rep {rep} image {i}")
    hd.set_option(hd.HD_OPT_RESIDENT, -1)


@pytest.mark.parametrize("shape,dt,maxv,top", [((700, 900), np.uint8, 100, 255),
                                                ((100, 120), np.uint16, 4095, 65535)])
def test_resident_values_above_max(hd, shape, dt, maxv, top):
    """Pixel values above the declared max value are legal (they only scale the output):
    the resident exchange's packed sum is bounded by the dtype's range, so such images give
    the staged result to the bit (8-bit: 330 tiles; 16-bit: 8 tiles, still packed)."""
    rng = np.random.default_rng(7)
    g = rng.integers(0, top + 1, size=shape)
    x = to_dev(g, dt)
    hd.set_option(hd.HD_OPT_RESIDENT, 0)
    staged = _bits(hd.hybrid_denoise(x, 7, 5, maxv))
    hd.set_option(hd.HD_OPT_RESIDENT, 1)
    for rep in range(2):
        log(f"values above max {shape} rep {rep}")
        np.testing.assert_array_equal(_bits(hd.hybrid_denoise(x, 7, 5, maxv)), staged)
    hd.set_option(hd.HD_OPT_RESIDENT, -1)


@pytest.mark.parametrize("n", [6, 31])
def test_resident_batched_uneven(hd, n):
    """Resident launch over a few uneven slices (one noise power per slice; 31 slices take
    the staged launches) equals the staged path; graph replays with other work between
    them keep agreeing."""
    imgs = _uneven_batch(n, 255, seed=91)
    ins = [to_dev(g, np.uint8) for g in imgs]
    hd.set_option(hd.HD_OPT_RESIDENT, 0)
    log("resident uneven: staged")
    staged = [_bits(o) for o in hd.hybrid_denoise_batched(ins, 9, 3, 255)]
    hd.set_option(hd.HD_OPT_RESIDENT, 1)
    outs = [torch.empty(x.shape, dtype=torch.float32, device="cuda") for x in ins]
    for rep in range(4):
        log(f"resident uneven rep {rep}")
        for o in outs:
            o.fill_(-1.0)
        hd.hybrid_denoise_batched(ins, 9, 3, 255, outs=outs)
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        del junk
        for i, o in enumerate(outs):
            np.testing.assert_array_equal(_bits(o), staged[i], err_msg=f"rep {rep} slice {i}")
    hd.set_option(hd.HD_OPT_RESIDENT, -1)


@pytest.mark.parametrize("form", ["packed_u8", "readback_u16", "readback_6_slices", "stretch_u8"])
def test_resident_fresh_data_each_launch(hd, form):
    """Consecutive resident launches on the same buffers (same plan, same barrier words)
    with different contents: each launch's noise power and output follow its own data, so
    no launch reads partials, noise powers or ranges left over from the previous one. Every
    exchange form: count and sum packed (one 8-bit slice), partials read back (one 16-bit
    slice, whose sum could overflow the packed word; six 8-bit slices), and the contrast
    stretch's second (range) round."""
    params = [(5, 0.05), (30, 0.3), (15, 0.15), (5, 0.05)]
    maxv = 4095 if form == "readback_u16" else 255
    dt = np.uint16 if maxv == 4095 else np.uint8
    stretch = form == "stretch_u8"
    if form == "readback_6_slices":
        shapes = [(300, 500), (257, 190), (64, 64), (400, 333), (31, 700), (128, 256)]
    elif form == "readback_u16":
        shapes = [(1000, 1300)]
    else:
        shapes = [(1100, 1500)]
    sets = [[noisy_phantom(h, w, maxv, sig * maxv / 255, dens, seed=40 + 10 * k + i)
             for i, (h, w) in enumerate(shapes)] for k, (sig, dens) in enumerate(params)]
    xs = [to_dev(g, dt) for g in sets[0]]
    outs = [torch.empty(x.shape, dtype=torch.float32, device="cuda") for x in xs]
    tiles = sum(hd.tiles_of(h, w) for h, w in shapes)
    hd.set_option(hd.HD_OPT_SELECT, 0)  # whatever an earlier autotuning chose for this key
    assert tiles <= hd.resident_capacity(torch.from_numpy(np.zeros(1, dt)).dtype, 9, 5, 0), "single launch"
    hd.set_option(hd.HD_OPT_RESIDENT, 0)
    staged = []
    for imgs in sets:
        for x, g in zip(xs, imgs):
            x.copy_(to_dev(g, dt))
        staged.append([_bits(o) for o in hd.hybrid_denoise_batched(xs, 9, 5, maxv, outs=outs, stretch=stretch)])
    hd.set_option(hd.HD_OPT_RESIDENT, 1)
    for rep in range(2):
        for k, imgs in enumerate(sets):
            log(f"resident fresh data {form} rep {rep} set {k}")
            for x, g in zip(xs, imgs):
                x.copy_(to_dev(g, dt))
            for o in outs:
                o.fill_(-1.0)
            hd.hybrid_denoise_batched(xs, 9, 5, maxv, outs=outs, stretch=stretch)
            for i, o in enumerate(outs):
                np.testing.assert_array_equal(_bits(o), staged[k][i], err_msg=f"rep {rep} set {k} slice {i}")
            if len(xs) == 1:
                nu2 = torch.empty(1, dtype=torch.float64, device="cuda")
                single = hd.hybrid_denoise(xs[0], 9, 5, maxv, nu2_out=nu2, stretch=stretch)
                np.testing.assert_array_equal(_bits(single), staged[k][0])
    hd.check_errors()
    hd.set_option(hd.HD_OPT_RESIDENT, -1)
    hd.set_option(hd.HD_OPT_SELECT, -1)


def test_batched_workload_c3(hd):
    """The 256-slice uneven 12-bit workload (96 x 256^2, 112 x 512^2, 48 x 1024^2)."""
    wl = CONFIGS["c3"]
    slices = wl.slices()
    ins = [to_dev(s.noisy, np.uint16) for s in slices]
    log("batched c3 full")
    outs = hd.hybrid_denoise_batched(ins, wl.smax, wl.win, wl.max_value)
    outs2 = hd.hybrid_denoise_batched(ins, wl.smax, wl.win, wl.max_value)  # graph replay
    worst = 0.0
    for i, s in enumerate(slices):
        ref, _, _ = oracle.hybrid(s.noisy, wl.smax, wl.win, wl.max_value)
        got = to_host(outs2[i])
        worst = max(worst, float(np.max(np.abs(got - ref))))
        np.testing.assert_array_equal(got.view(np.uint32), to_host(outs[i]).view(np.uint32))
    assert worst <= TOL, worst


def test_batched_workload_c4_plain(hd):
    """The surrogate workload's plain path at full size: 64 x 1024^2 u8 slices (sigma 5-25,
    salt and pepper 0.05-0.30, Smax 9, Wiener 5 x 5), staged plan replayed as a graph."""
    wl = CONFIGS["c4"]
    slices = wl.slices()
    ins = [to_dev(s.noisy, np.uint8) for s in slices]
    log("batched c4 plain full")
    outs = hd.hybrid_denoise_batched(ins, wl.smax, wl.win, wl.max_value)
    worst = 0.0
    for i, s in enumerate(slices):
        ref, _, _ = oracle.hybrid(s.noisy, wl.smax, wl.win, wl.max_value)
        worst = max(worst, float(np.max(np.abs(to_host(outs[i]) - ref))))
    assert worst <= TOL, worst


def test_batched_bad_slice_named(hd):
    ins = [to_dev(np.zeros((8, 8), np.int32), np.uint8), to_dev(np.zeros((8, 8), np.int32), np.uint8)]
    with pytest.raises(hd.HDError, match="slice"):
        hd.hybrid_denoise_batched(ins, 4, 3, 255)


def test_autotune_picks_a_strategy(hd, tmp_path, monkeypatch):
    g = noisy_phantom(512, 512, 255, 15, 0.2, seed=3)
    inp = to_dev(g, np.uint8)
    log("autotune")
    sel, fuse, rows = hd.autotune_hybrid(inp, 9, 5, 255, iters=3)
    assert sel in (0, 1, 2, 3) and fuse in (0, 1)
    out = hd.hybrid_denoise(inp, 9, 5, 255)  # uses the tuned strategy
    ref, _, _ = oracle.hybrid(g, 9, 5, 255)
    assert np.max(np.abs(to_host(out) - ref)) <= TOL


def test_gpu_argument_errors_real_buffers(hd):
    x = to_dev(np.zeros((16, 16), np.int32), np.uint8)
    with pytest.raises(hd.HDError, match="SMAX"):
        hd.amf_filter(x, 4)
    with pytest.raises(hd.HDError) as ei:
        hd.amf_filter(x, 5, out=x)
    assert ei.value.name == "HD_ERR_ALIAS"
    with pytest.raises(hd.HDError) as ei:
        hd.wiener_filter(x, 4, 255)
    assert ei.value.name == "HD_ERR_WINDOW"


def test_batched_workload_c5_full(hd):
    """The stress workload at full size, as the benchmark runs it: all 16 slices of 4096^2
    12-bit data (sigma 60, salt and pepper 0.5, Smax 15, Wiener 7 x 7) in ONE batched call
    with the autotuned strategy, replayed. Four slices are checked against the oracle: the
    AMF bit-exact (single-slice call with the AMF image returned, whose Wiener output must
    equal the batched output to the bit) and the output within 1e-4."""
    wl = CONFIGS["c5"]
    slices = wl.slices()
    ins = [to_dev(s.noisy, np.uint16) for s in slices]
    log("c5 full: autotune")
    hd.autotune_hybrid(ins[0], wl.smax, wl.win, wl.max_value, iters=2)
    log("c5 full: batched")
    outs = hd.hybrid_denoise_batched(ins, wl.smax, wl.win, wl.max_value)
    outs = hd.hybrid_denoise_batched(ins, wl.smax, wl.win, wl.max_value, outs=outs)  # replay
    hd.check_errors()
    for i in (0, 5, 10, 15):
        log(f"c5 full: slice {i} vs oracle")
        ref, a_ref, _ = oracle.hybrid(slices[i].noisy, wl.smax, wl.win, wl.max_value)
        a = torch.empty_like(ins[i])
        single = hd.hybrid_denoise(ins[i], wl.smax, wl.win, wl.max_value, amf_out=a)
        np.testing.assert_array_equal(to_host(a).astype(np.int32), a_ref, err_msg=f"AMF slice {i}")
        got = to_host(outs[i])
        np.testing.assert_array_equal(got.view(np.uint32), _bits(single), err_msg=f"slice {i}")
        err = float(np.max(np.abs(got - ref)))
        assert err <= TOL, (i, err)
    hd.release_plans()
