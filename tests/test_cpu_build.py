"""The library's own HIP sources, built for the host against the CPU stand-in
runtime (tests/cpu_hip/: work-items as threads, AddressSanitizer on every
access), run through the C-ABI on small frames.  These tests need no GPU:
they check that every kernel terminates and stays inside its buffers, at
capacities the GPU tests use too, and compare the frames with the oracle."""
import os
import sys

import numpy as np
import pytest

from paper_2606_00352_amd import scenes

HERE = os.path.dirname(os.path.abspath(__file__))


def _cpu():
    sys.path.insert(0, os.path.join(HERE, "cpu_hip"))
    import cpu_build
    if not cpu_build.available():
        pytest.skip("no host clang++")
    return cpu_build


@pytest.mark.parametrize("sort_mode", [0, 1], ids=["segmented", "onesweep"])
def test_lists_of_many_bands_match_the_oracle(orc, sort_mode):
    """Gaussians whose macro-tile lists span one to six bands: lists of one
    or two bands go through the span word, longer ones through the predicate
    again in the emission; the sorted pairs and batches equal the oracle's bit
    for bit in both sort modes."""
    cpu = _cpu()
    sc, cam = _dense_scene(2500, 320, 256, 300.0, 51, 150, 120, 0.0)
    rng = np.random.default_rng(51)
    sc.scales[:] = rng.uniform(0.005, 0.2, (sc.n, 3)).astype(np.float32)
    fr = cpu.run_frames(sc, [cam], max_pairs=1 << 17, max_batches=4096, sort_mode=sort_mode)[0]
    o = orc.frame(sc, cam)
    bands = {}
    nx = (cam.width + 63) // 64
    for m, g in zip(o.sorted_mt.tolist(), o.sorted_gid.tolist()):
        lo, hi = bands.get(g, (1 << 30, -1))
        bands[g] = (min(lo, m // nx), max(hi, m // nx))
    spans = np.bincount([hi - lo + 1 for lo, hi in bands.values()])
    assert spans[3:5].sum() >= 50 and spans[5:].sum() >= 5, spans
    assert fr.rc == 0 and fr.overflow == 0
    want = (o.sorted_mt.astype(np.uint64) << np.uint64(32)) | o.sorted_key.astype(np.uint64)
    assert np.array_equal(fr.keys, want)
    assert np.array_equal(fr.ids, o.sorted_gid.astype(np.uint32))
    assert np.array_equal(fr.batches.astype(np.int64), o.batch_tab.astype(np.int64))


def test_small_frame_matches_the_oracle(orc):
    """Pairs, sort order and batches bit-exact, image within the tolerance."""
    cpu = _cpu()
    scene = scenes.uniform_scene(3000, seed=7)
    cam = scenes.camera_at_origin(160, 96, 140.0, (0.1, 0.2, 0.3))
    fr = cpu.run_frames(scene, [cam], max_pairs=1 << 16, max_batches=4096)[0]
    o = orc.frame(scene, cam)
    assert fr.rc == 0 and fr.overflow == 0
    want = (o.sorted_mt.astype(np.uint64) << np.uint64(32)) | o.sorted_key.astype(np.uint64)
    assert np.array_equal(fr.keys, want)
    assert np.array_equal(fr.ids, o.sorted_gid.astype(np.uint32))
    assert np.array_equal(fr.batches.astype(np.int64), o.batch_tab.astype(np.int64))
    d = np.abs(fr.image.astype(np.float64) - o.image)
    assert d[o.amb == 0].max() <= 2e-4 and d.mean() <= 1e-5


def test_capacity_overflow_stops_the_frame(orc):
    """The overflow protocol at the GPU test's capacities (16 pairs, 4
    batches): every stage after the pair scan returns at once, the image and
    T are NaN, the counts report what the frame needed; a context of exactly
    those sizes renders the oracle's image."""
    cpu = _cpu()
    sc, cams = scenes.config0()
    cam = cams[0]
    fr = cpu.run_frames(sc, [cam], max_pairs=16, max_batches=4)[0]
    assert fr.rc == 0 and fr.overflow == 1          # pairs only: the batch stage never ran
    assert fr.n_pairs > 16 and fr.n_batches == 0
    assert np.isnan(fr.image).all() and np.isnan(fr.T).all()
    fb = cpu.run_frames(sc, [cam], max_pairs=fr.n_pairs, max_batches=3)[0]
    assert fb.overflow == 2 and fb.n_pairs == fr.n_pairs and fb.n_batches > 3
    assert np.isnan(fb.image).all()
    ok = cpu.run_frames(sc, [cam], max_pairs=fr.n_pairs, max_batches=fb.n_batches)[0]
    assert ok.overflow == 0
    o = orc.frame(sc, cam)
    d = np.abs(ok.image.astype(np.float64) - o.image)
    assert d[o.amb == 0].max() <= 2e-4 and d.mean() <= 1e-5


def _psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return 10.0 * np.log10(1.0 / mse) if mse > 0 else np.inf


def test_packed_sh_matches_the_oracle_codec(orc):
    """higs_sh_compress writes the oracle codec's scales and words bit for bit,
    and the projection's colour from them is the oracle's colour from the
    decoded coefficients (the image within the float32 tolerance)."""
    from oracle import shcodec
    cpu = _cpu()
    sc, cams = scenes.config0()
    cam = cams[0]
    fr = cpu.run_frames(sc, [cam], max_pairs=1 << 17, max_batches=1 << 12, sh_format=1)[0]
    s, w = shcodec.compress(sc.sh, sc.opacities)
    assert np.array_equal(fr.packed[:256].view(np.float32)[:48], s)
    assert np.array_equal(fr.packed[256:].view(np.uint32).reshape(-1, 8), w)
    dec = scenes.Scene(sc.means, sc.scales, sc.quats, sc.opacities,
                       shcodec.decompress(s, w).reshape(sc.sh.shape))
    o = orc.frame(dec, cam)
    d = np.abs(fr.image.astype(np.float64) - o.image)
    assert d[o.amb == 0].max() <= 2e-4 and d.mean() <= 1e-5


def test_half_precision_raster(orc):
    """The reduced-precision mode: the same pairs, order and batches as the
    float32 mode, and an image within the paper's fidelity range of the oracle
    (its fp16 renderer is 67 dB from the float32 one)."""
    cpu = _cpu()
    sc, cams = scenes.config0()
    cam = cams[0]
    fr = cpu.run_frames(sc, [cam], max_pairs=1 << 17, max_batches=1 << 12, precision=1)[0]
    # the partials merged by the merge kernel instead of folded in the raster
    frm = cpu.run_frames(sc, [cam], max_pairs=1 << 17, max_batches=1 << 12, precision=1, fuse=0)[0]
    assert np.array_equal(fr.image, frm.image) and np.array_equal(fr.T, frm.T)
    o = orc.frame(sc, cam)
    want = (o.sorted_mt.astype(np.uint64) << np.uint64(32)) | o.sorted_key.astype(np.uint64)
    assert np.array_equal(fr.keys, want) and np.array_equal(fr.ids, o.sorted_gid.astype(np.uint32))
    assert np.array_equal(fr.batches.astype(np.int64), o.batch_tab.astype(np.int64))
    assert _psnr(fr.image, o.image) >= 55.0
    assert np.all(np.isfinite(fr.image)) and np.all((fr.T >= 0) & (fr.T <= 1))


@pytest.mark.parametrize("precision", [0, 1])
def test_views_in_one_frame_match_their_single_frames(precision):
    """higs_render_views: three views (different cameras, two scene sizes)
    rendered as one frame give, view by view, the images and transmittances
    of three single-view frames, bit for bit; the frame's pairs are the sum
    of the single frames' pairs."""
    cpu = _cpu()
    sc = scenes.clustered_scene(6000, seed=6, n_clusters=4)
    cams = scenes.orbit_cameras(5, 3, 160, 96, 140.0)[:3]
    uses = [6000, 4000, 6000]
    single = cpu.run_frames(sc, cams, max_pairs=1 << 17, max_batches=1 << 12, uses=uses,
                            precision=precision)
    multi = cpu.run_frames(sc, cams, max_pairs=1 << 17, max_batches=1 << 12, uses=uses, entry=2,
                           precision=precision)
    assert all(f.rc == 0 and f.overflow == 0 for f in single + multi)
    assert multi[0].n_pairs == sum(f.n_pairs for f in single)
    for a, b in zip(single, multi):
        assert np.array_equal(a.image, b.image) and np.array_equal(a.T, b.T)


def test_graph_replay_matches_kernel_by_kernel_frames():
    """params.use_graphs: frames recorded into graphs and replayed (a shape
    seen before replays its graph with a new camera and scene size inside the
    same padded range) give the images of the kernel-by-kernel frames, bit for
    bit; so does a several-view frame replayed after a first frame of the same
    shape with other cameras and outputs."""
    cpu = _cpu()
    sc = scenes.clustered_scene(6000, seed=6, n_clusters=4)
    cams = scenes.orbit_cameras(5, 3, 160, 96, 140.0)[:4]
    uses = [6000, 5800, 6000, 3000]   # frames 0-2 share one padded range, 3 another
    eager = cpu.run_frames(sc, cams, max_pairs=1 << 17, max_batches=1 << 12, uses=uses)
    graph = cpu.run_frames(sc, cams, max_pairs=1 << 17, max_batches=1 << 12, uses=uses, entry=3)
    assert [f.graphs for f in graph] == [1, 1, 1, 2]
    for a, b in zip(eager, graph):
        assert a.rc == 0 and b.rc == 0 and b.overflow == 0 and b.n_pairs == a.n_pairs
        assert np.array_equal(a.image, b.image) and np.array_equal(a.T, b.T)
    views = cpu.run_frames(sc, cams[:3], max_pairs=1 << 17, max_batches=1 << 12, uses=uses[:3], entry=4)
    assert views[0].graphs == 1
    for a, b in zip(eager[:3], views):
        assert b.rc == 0 and np.array_equal(a.image, b.image) and np.array_equal(a.T, b.T)


def test_server_frames_hold_several_requests():
    """The render server with several requests per frame and graph replay:
    every request's image is the kernel-by-kernel frame's, bit for bit, in two
    rounds (the second replays the graph on the same context)."""
    cpu = _cpu()
    sc = scenes.clustered_scene(6000, seed=6, n_clusters=4)
    cams = scenes.orbit_cameras(5, 3, 160, 96, 140.0)[:3]
    uses = [6000, 4000, 6000]
    eager = cpu.run_frames(sc, cams, max_pairs=1 << 16, max_batches=1 << 12, uses=uses)
    served = cpu.run_frames(sc, cams, max_pairs=1 << 16, max_batches=1 << 12, uses=uses, entry=5)
    for a, b in zip(eager, served):
        assert b.rc == 0 and np.array_equal(a.image, b.image)


def _dense_scene(n, w, h, f, seed, spread_x, spread_y, scale):
    sc = scenes.uniform_scene(n, seed=seed)
    rng = np.random.default_rng(seed)
    z = rng.uniform(2, 6, n).astype(np.float32)
    sc.means[:, 0] = rng.uniform(-spread_x, spread_x, n) * z / f
    sc.means[:, 1] = rng.uniform(-spread_y, spread_y, n) * z / f
    sc.means[:, 2] = z
    sc.scales[:] = scale
    return sc, scenes.camera_at_origin(w, h, f)


@pytest.mark.parametrize("case", ["config0", "equal_depths", "dense_macro_tile", "long_segment"])
def test_segmented_sort_matches_the_oracle(orc, case):
    """The segmented form (count matrix, scan, fill, tiered segment sorts,
    merges of long segments): the sorted (macro-tile, depth, id) list, the
    segment offsets and the batches equal the oracle's, bit for bit, for
    segments in every tier and a long one of several chunks."""
    cpu = _cpu()
    if case == "config0":
        sc, cams = scenes.config0()
        cam = cams[0]
    elif case == "equal_depths":
        rng = np.random.default_rng(2)
        sc = scenes.uniform_scene(2000, seed=12)
        sc.means[:, 2] = 3.0
        sc.means[:, :2] = rng.uniform(-0.5, 0.5, (2000, 2))
        cam = scenes.camera_at_origin(160, 160, 160.0)
    elif case == "dense_macro_tile":   # ~9,000 pairs in one macro-tile: tier 2
        sc, cam = _dense_scene(9000, 256, 128, 256.0, 21, 20, 10, 0.004)
    else:                              # ~40,000 in one: three chunks, two merge levels
        sc, cam = _dense_scene(40_000, 64, 32, 64.0, 21, 30, 14, 0.003)
    fr = cpu.run_frames(sc, [cam], max_pairs=1 << 17, max_batches=4096, sort_mode=0)[0]
    o = orc.frame(sc, cam)
    assert fr.rc == 0 and fr.overflow == 0
    want = (o.sorted_mt.astype(np.uint64) << np.uint64(32)) | o.sorted_key.astype(np.uint64)
    assert np.array_equal(fr.keys, want)
    assert np.array_equal(fr.ids, o.sorted_gid.astype(np.uint32))
    assert np.array_equal(fr.batches.astype(np.int64), o.batch_tab.astype(np.int64))
    if case == "long_segment":
        assert fr.n_pairs > 32768


def test_raster_chains_skip_saturated_tiles(orc):
    """A raster work item of several batches of one macro-tile leaves out the
    render tiles whose product of transmittances over its earlier batches is
    below t_eps everywhere: the image and T are those of one batch per work
    item, bit for bit, and of the oracle, with fewer evaluations.  Items of
    whole macro-tiles that fold their partials themselves (no merge kernel)
    give the same image and T as well."""
    from paper_2606_00352_amd import higs
    cpu = _cpu()
    sc, cam = _dense_scene(9000, 256, 128, 256.0, 21, 20, 10, 0.004)
    sc.opacities[:] = 0.9
    old = os.environ.get("HIGS_CPU_DEBUG")
    os.environ["HIGS_CPU_DEBUG"] = str(higs.DEBUG_COUNT_EVALS)
    try:
        kw = dict(max_pairs=1 << 16, max_batches=256, batch_cap=256)
        one = cpu.run_frames(sc, [cam], chain=1, fuse=0, **kw)[0]
        # runs of three (items of lengths 3, 2 and 1 in one list) and whole macro-tiles
        three = cpu.run_frames(sc, [cam], chain=3, fuse=0, **kw)[0]
        many = cpu.run_frames(sc, [cam], chain=64, fuse=0, **kw)[0]
        fused = cpu.run_frames(sc, [cam], fuse=1, **kw)[0]
    finally:
        if old is None:
            del os.environ["HIGS_CPU_DEBUG"]
        else:
            os.environ["HIGS_CPU_DEBUG"] = old
    assert one.rc == 0 and three.rc == 0 and many.rc == 0 and fused.rc == 0 and one.n_batches > 8
    for r in (three, many, fused):
        assert np.array_equal(one.image, r.image) and np.array_equal(one.T, r.T)
    assert fused.n_evaluations == many.n_evaluations
    assert 0 < many.n_evaluations <= three.n_evaluations <= one.n_evaluations
    assert many.n_evaluations < one.n_evaluations
    prm = orc.Params()
    prm.batch_cap = 256
    o = orc.frame(sc, cam, prm)
    d = np.abs(many.image.astype(np.float64) - o.image)
    assert d[o.amb == 0].max() <= 2e-4 and d.mean() <= 1e-5
