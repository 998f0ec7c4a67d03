"""GPU parity of every stage of the frame path against the oracle, through
the C-ABI: projection fields bit-exact, emitted pairs, sorted pairs,
macro-tile offsets and batch table bit-exact, per-batch partials and the
final image within the float32 tolerance (2e-4 max abs, 1e-5 mean abs per
channel).  Sizes span several macro-tiles, batches and sort tiles with
ragged tails; edge cases cover the method's degenerate inputs."""
import math

import numpy as np
import pytest

from paper_2606_00352_amd import scenes
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu


SORT_MODES = pytest.mark.parametrize("sort_mode", [0, 1], ids=["segmented", "onesweep"])


def _merged_T_before(orc, fr, cam, prm, b, t):
    """The merge's transmittance at tile t of batch b's macro-tile after its
    earlier batches (Eq. 1, stopping per pixel below t_eps), from the oracle's
    batch partials."""
    m = int(fr.batch_tab[b, 0])
    T = np.ones(64)
    for bb in range(b):
        if int(fr.batch_tab[bb, 0]) != m:
            continue
        o = orc.batch_partials(fr.geo, fr.sorted_gid, fr.batch_tab[bb], cam, prm)
        go = T >= prm.t_eps
        T = np.where(go, T * o[t][:, 3], T)
    return T


def _full_check(orc, scene, cam, cap=1024, report=None, check_partials=True, sort_mode=0,
                debug=0):
    report = {} if report is None else report
    ctx, img, T = gc.gpu_frame(scene, cam, batch_cap=cap, sort_mode=sort_mode, debug=debug)
    prm = gc.oracle_params(orc, batch_cap=cap)
    fr = orc.frame(scene, cam, prm)
    gc.check_projection(orc, ctx, fr, report)
    gc.check_pairs_sort_batches(orc, ctx, fr, cap)
    cmax = float(fr.geo[fr.valid == 1, orc.G_R:orc.G_BL + 1].max()) if fr.valid.any() else 1.0
    gc.check_image(img, T, fr.image, fr.T, fr.amb, report, cmax)
    if check_partials and fr.batch_tab.shape[0]:
        # the partials of a frame with the merge kernel (fuse_merge = 0), whose
        # image and T equal the fused frame's bit for bit
        pctx, pimg, pT = gc.gpu_frame(scene, cam, batch_cap=cap, sort_mode=sort_mode, debug=debug,
                                      fuse_merge=0)
        assert np.array_equal(pimg, img) and np.array_equal(pT, T)
        parts = pctx.partials()
        act = pctx.active()
        rng = np.random.default_rng(0)
        pick = rng.choice(fr.batch_tab.shape[0], size=min(12, fr.batch_tab.shape[0]), replace=False)
        nmx = (cam.width + 63) // 64
        p_ = np.arange(64)
        for b in pick:
            o, o_amb = orc.batch_partials(fr.geo, fr.sorted_gid, fr.batch_tab[b], cam, prm, with_amb=True)
            m = int(fr.batch_tab[b, 0])
            for t in range(32):
                x = (m % nmx) * 64 + (t % 8) * 8 + p_ % 8
                y = (m // nmx) * 32 + (t // 8) * 8 + p_ // 8
                inside = (x < cam.width) & (y < cam.height)   # lanes past the image edge are never read
                if (act[b] >> t) & 1:
                    d = np.abs(parts[b, t].astype(np.float64) - o[t])
                    clean = inside & (o_amb[t] == 0)
                    # the image tolerance on pixels whose decisions are not
                    # flagged; a flagged alpha moves a partial by at most ~2/255
                    assert d[clean].max(initial=0.0) <= gc.IMG_MAX_ABS, (b, t, d[clean].max(initial=0.0))
                    assert d[inside & ~clean].max(initial=0.0) <= 2.0 / 255.0 * max(1.0, cmax), (b, t)
                elif np.any(np.abs(o[t][:, 3] - 1.0) > 1e-6):
                    # a tile with gaussians left out by the raster: only where
                    # the merge has stopped reading it, i.e. the product of
                    # the macro-tile's earlier batches' T is below t_eps at
                    # all 64 pixels (a raster work item takes several batches
                    # of one macro-tile and drops such tiles)
                    assert _merged_T_before(orc, fr, cam, prm, b, t).max() < prm.t_eps * 1.001, (b, t)
    return ctx, report


@SORT_MODES
def test_config0_all_stages(orc, sort_mode):
    sc, cams = scenes.config0()
    ctx, rep = _full_check(orc, sc, cams[0], sort_mode=sort_mode)
    c = ctx.counts()
    assert c.n_pairs > 10_000 and c.n_batches > 30
    print("config0", rep)


@pytest.mark.parametrize("cap", [4, 64, 333])
@SORT_MODES
def test_small_batch_caps(orc, cap, sort_mode):
    sc, cams = scenes.config0()
    _full_check(orc, sc, cams[0], cap=cap, check_partials=(cap != 4), sort_mode=sort_mode)


@pytest.mark.parametrize("W,H", [(200, 150), (130, 70), (250, 171)])
@SORT_MODES
def test_ragged_images(orc, sort_mode, W, H):
    """Widths/heights that are not multiples of the macro-tile (64x32) or of
    the render tile (8x8)."""
    sc = scenes.uniform_scene(6000, seed=W + H)
    cam = scenes.camera_at_origin(W, H, 0.9 * W, (0.2, 0.4, 0.1))
    _full_check(orc, sc, cam, sort_mode=sort_mode)


@SORT_MODES
def test_orbit_camera_clustered(orc, sort_mode):
    """Rotated camera, clustered scene (config-1 generator at a small size)."""
    sc = scenes.clustered_scene(60_000, seed=5, n_clusters=20)
    cam = scenes.orbit_cameras(3, 7, 320, 180, 200.0)[1]
    _full_check(orc, sc, cam, sort_mode=sort_mode)


def test_empty_and_single(orc):
    cam = scenes.camera_at_origin(96, 80, 80.0, (0.3, 0.6, 0.9))
    empty = scenes.Scene(*(np.zeros((0,) + s, np.float32) for s in [(3,), (3,), (4,), (), (16, 3)]))
    ctx, img, T = gc.gpu_frame(empty, cam)
    bg = np.float32([0.3, 0.6, 0.9])
    assert np.all(img == bg) and np.all(T == 1.0)
    c = ctx.counts()
    assert c.n_pairs == 0 and c.n_batches == 0
    one = scenes.uniform_scene(1, seed=3)
    one.means[0] = [0.05, -0.02, 3.0]
    one.scales[0] = 0.05
    one.opacities[0] = 0.8
    _full_check(orc, one, cam)


def test_culled_inputs(orc):
    """Behind the near plane, zero quaternion, NaN mean, opacity < 1/255:
    culled, no pairs; the remaining gaussians render as usual."""
    sc = scenes.uniform_scene(500, seed=4)
    sc.means[0] = [0.0, 0.0, 0.1]
    sc.means[1] = [0.0, 0.0, -2.0]
    sc.quats[2] = 0.0
    sc.means[3] = [np.nan, 0.0, 3.0]
    sc.opacities[4] = np.float32(0.5 / 255.0)
    sc.scales[5] = np.inf
    cam = scenes.camera_at_origin(128, 128, 128.0)
    ctx, _ = _full_check(orc, sc, cam)
    cnt = ctx.proj_fields()["count"]
    assert np.all(cnt[:6] == 0)


def _border_and_huge_splat_scene():
    rng = np.random.default_rng(8)
    sc = scenes.uniform_scene(3000, seed=8)
    W, H = 256, 192
    cam = scenes.camera_at_origin(W, H, 200.0)
    # centres just outside / on the border
    k = 200
    z = rng.uniform(2, 5, k).astype(np.float32)
    u = rng.choice([-3.0, -0.2, 0.0, W + 0.3, W + 4.0], k)
    v = rng.uniform(-10, H + 10, k)
    sc.means[:k, 0] = (u - W / 2) * z / 200.0
    sc.means[:k, 1] = (v - H / 2) * z / 200.0
    sc.means[:k, 2] = z
    sc.scales[:k] = 0.02
    sc.means[k] = [0.0, 0.0, 8.0]
    sc.scales[k] = [6.0, 4.0, 5.0]
    sc.opacities[k] = 0.95
    return sc, cam, k


def test_edge_straddling_and_huge_splat(orc):
    """Splats straddling the image border, and one splat covering every
    macro-tile (hundreds of pairs from one gaussian)."""
    sc, cam, k = _border_and_huge_splat_scene()
    ctx, _ = _full_check(orc, sc, cam)
    cnt = ctx.proj_fields()["count"]
    assert cnt[k] == ctx.n_mt


@SORT_MODES
def test_binning_fields_stored_only_where_needed(orc, sort_mode):
    """Without HIGS_DEBUG_PROJ_FIELDS the projection stores the binning fields
    only for gaussians whose macro-tile list the emission derives again (the
    splat over every macro-tile): sorted pairs, batches and image are the
    same as with every field stored."""
    from paper_2606_00352_amd import higs
    sc, cam, k = _border_and_huge_splat_scene()
    out = []
    for flags in (higs.DEBUG_PROJ_FIELDS, 0):
        ctx = higs.Context(sc.n, cam.width, cam.height, max_pairs=64 * sc.n, sort_mode=sort_mode)
        ctx.set_debug(flags)
        ctx, img, T = gc.gpu_frame(sc, cam, keep_pairs=False, ctx=ctx)
        out.append((ctx.sorted_pairs(), ctx.batches(), img, T))
        assert ctx.counts().n_pairs > ctx.n_mt
    for a, b in zip(out[0], out[1]):
        a = a if isinstance(a, tuple) else (a,)
        b = b if isinstance(b, tuple) else (b,)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@SORT_MODES
def test_equal_depths_tie_break(orc, sort_mode):
    """2,000 gaussians at one depth: ties resolved by gaussian id."""
    rng = np.random.default_rng(2)
    n = 2000
    sc = scenes.uniform_scene(n, seed=12)
    sc.means[:, 2] = 3.0
    sc.means[:, :2] = rng.uniform(-0.5, 0.5, (n, 2))
    cam = scenes.camera_at_origin(160, 160, 160.0)
    ctx, _ = _full_check(orc, sc, cam, sort_mode=sort_mode)
    keys, vals = ctx.sorted_pairs()
    mts = (keys >> np.uint64(32)).astype(np.int64)
    for m in np.unique(mts):
        assert np.all(np.diff(vals[mts == m].astype(np.int64)) > 0)


@SORT_MODES
def test_dense_macro_tile_many_batches(orc, sort_mode):
    """> 8,000 gaussians in one macro-tile (several 1,024-batches and more than
    one sort tile inside one segment)."""
    n = 9000
    sc = scenes.uniform_scene(n, seed=21)
    rng = np.random.default_rng(21)
    z = rng.uniform(2, 6, n).astype(np.float32)
    sc.means[:, 0] = rng.uniform(-20, 20, n) * z / 256.0
    sc.means[:, 1] = rng.uniform(-10, 10, n) * z / 256.0
    sc.means[:, 2] = z
    sc.scales[:] = 0.004
    cam = scenes.camera_at_origin(256, 128, 256.0)
    ctx, _ = _full_check(orc, sc, cam, sort_mode=sort_mode)
    c = ctx.counts()
    assert c.n_batches >= 9


def test_repeat_renders_bit_identical(orc):
    """Every stage is deterministic: repeated frames are identical."""
    import torch
    from paper_2606_00352_amd import higs
    sc = scenes.clustered_scene(50_000, seed=6, n_clusters=10)
    cam = scenes.orbit_cameras(2, 3, 320, 240, 240.0)[0]
    ctx, img0, T0 = gc.gpu_frame(sc, cam)
    k0, v0 = ctx.sorted_pairs()
    t = higs.scene_tensors(sc)
    for _ in range(9):
        img, T = higs.render(ctx, t, cam)
        torch.cuda.synchronize()
        assert np.array_equal(img.cpu().numpy(), img0) and np.array_equal(T.cpu().numpy(), T0)
        k, v = ctx.sorted_pairs()
        assert np.array_equal(k, k0) and np.array_equal(v, v0)


def test_untiled_definition_within_eps(orc):
    """The GPU image against the plain per-pixel definition: within
    t_eps * max(c_max, |bg|) plus float32 rounding, away from ambiguous pixels."""
    sc, cams = scenes.config0()
    cam = scenes.camera_at_origin(256, 256, 256.0, (0.1, 0.1, 0.1))
    ctx, img, T = gc.gpu_frame(sc, cam)
    valid, geo = orc.project(sc, cam)
    o_img, o_T, amb = orc.render_untiled(valid, geo, cam)
    cmax = max(float(geo[valid == 1, orc.G_R:orc.G_BL + 1].max()), 0.1)
    d = np.abs(img - o_img)[amb == 0]
    assert d.max() <= 1e-4 * cmax + 2e-5


@SORT_MODES
def test_one_segment_of_seventy_thousand(orc, sort_mode):
    """70,000 gaussians in one 64x32 macro-tile: a segment of five 16,384-pair
    chunks, merged over three levels (an odd run at each) in the segmented
    sort."""
    n = 70_000
    sc = scenes.uniform_scene(n, seed=21)
    rng = np.random.default_rng(21)
    z = rng.uniform(2, 6, n).astype(np.float32)
    sc.means[:, 0] = rng.uniform(-30, 30, n) * z / 64.0
    sc.means[:, 1] = rng.uniform(-14, 14, n) * z / 64.0
    sc.means[:, 2] = z
    sc.scales[:] = 0.003
    cam = scenes.camera_at_origin(64, 32, 64.0)
    ctx, _ = _full_check(orc, sc, cam, sort_mode=sort_mode, check_partials=False)
    assert ctx.counts().n_pairs > 4 * 16384


def test_sort_modes_give_identical_frames(orc):
    """Both sort implementations: the same ids, batches and image, bit for bit."""
    sc = scenes.clustered_scene(120_000, seed=17, n_clusters=12)
    cam = scenes.orbit_cameras(4, 9, 400, 300, 300.0)[2]
    out = []
    for mode in (0, 1):
        ctx, img, T = gc.gpu_frame(sc, cam, sort_mode=mode)
        out.append((ctx.sorted_pairs(), ctx.batches(), img, T))
    (k0, v0), b0, i0, t0 = out[0]
    (k1, v1), b1, i1, t1 = out[1]
    assert np.array_equal(k0, k1) and np.array_equal(v0, v1) and np.array_equal(b0, b1)
    assert np.array_equal(i0, i1) and np.array_equal(t0, t1)


def _tie_scene():
    rng = np.random.default_rng(2)
    n = 2000
    sc = scenes.uniform_scene(n, seed=12)
    sc.means[:, 2] = 3.0
    sc.means[:, :2] = rng.uniform(-0.5, 0.5, (n, 2))
    return sc, scenes.camera_at_origin(160, 160, 160.0)


def _dense_scene():
    n = 9000
    sc = scenes.uniform_scene(n, seed=21)
    rng = np.random.default_rng(21)
    z = rng.uniform(2, 6, n).astype(np.float32)
    sc.means[:, 0] = rng.uniform(-20, 20, n) * z / 256.0
    sc.means[:, 1] = rng.uniform(-10, 10, n) * z / 256.0
    sc.means[:, 2] = z
    sc.scales[:] = 0.004
    return sc, scenes.camera_at_origin(256, 128, 256.0)


def _config0_scene():
    sc, cams = scenes.config0()
    return sc, cams[0]


@pytest.mark.parametrize("make", [_config0_scene, _dense_scene, _tie_scene],
                         ids=["config0", "dense", "ties"])
def test_two_array_pairs(orc, make):
    """The onesweep with key and id in separate arrays (the layout of frames
    whose key and id do not fit one word), forced by a debug flag: every stage
    against the oracle, and the same pairs, batches and image as the one-word
    layout of the same frame."""
    from paper_2606_00352_amd import higs
    sc, cam = make()
    out = []
    for debug, pair_bytes in ((higs.DEBUG_TWO_WORD_PAIRS, 12), (0, 8)):
        ctx, _ = _full_check(orc, sc, cam, sort_mode=1, debug=debug)
        assert ctx.counts().sort_pair_bytes == pair_bytes
        img, T = higs.render(ctx, higs.scene_tensors(sc), cam)
        out.append((ctx.sorted_pairs(), ctx.batches(), img.cpu().numpy(), T.cpu().numpy()))
    (k0, v0), b0, i0, t0 = out[0]
    (k1, v1), b1, i1, t1 = out[1]
    assert np.array_equal(k0, k1) and np.array_equal(v0, v1) and np.array_equal(b0, b1)
    assert np.array_equal(i0, i1) and np.array_equal(t0, t1)


def test_work_item_forms_give_one_frame(orc):
    """The raster's work items of 1, 2, 7 and 64 batches of a macro-tile with
    stored partials and the merge kernel, and whole macro-tiles folding their
    partials (the default), render the same image and T bit for bit; an item
    that knows all earlier batches of its macro-tile evaluates no more
    pixel-gaussian pairs than one that knows fewer, and the frame matches the
    oracle (a dense, saturating scene: tiles fall below t_eps within a few
    batches)."""
    import torch
    from paper_2606_00352_amd import higs
    gc.need_gpu()
    # 30,000 gaussians of opacity 0.9 in front of a 384 x 192 image: by the
    # oracle's count half of the per-batch evaluations lie in tiles the merge
    # no longer reads
    n = 30_000
    sc = scenes.uniform_scene(n, seed=43)
    rng = np.random.default_rng(43)
    z = rng.uniform(2, 6, n).astype(np.float32)
    sc.means[:, 0] = rng.uniform(-150, 150, n) * z / 384.0
    sc.means[:, 1] = rng.uniform(-75, 75, n) * z / 384.0
    sc.means[:, 2] = z
    sc.scales[:] = 0.02
    sc.opacities[:] = 0.9
    cam = scenes.camera_at_origin(384, 192, 384.0)
    t = higs.scene_tensors(sc)
    runs = []
    for params in ({"fuse_merge": 0, "raster_chain": 1}, {"fuse_merge": 0, "raster_chain": 2},
                   {"fuse_merge": 0, "raster_chain": 7}, {"fuse_merge": 0, "raster_chain": 64}, {}):
        ctx = higs.Context(sc.n, cam.width, cam.height, max_pairs=16 * sc.n, batch_cap=256, **params)
        ctx.set_debug(higs.DEBUG_COUNT_EVALS)
        img, T = higs.render(ctx, t, cam)
        torch.cuda.synchronize()
        c = ctx.counts()
        assert c.overflow == 0 and c.n_batches > 40
        runs.append((img.cpu().numpy(), T.cpu().numpy(), int(c.n_evaluations)))
        ctx.close()
    for img, T, _ in runs[1:]:
        assert np.array_equal(img, runs[0][0]) and np.array_equal(T, runs[0][1])
    ev = [r[2] for r in runs]
    assert ev[0] >= max(ev[1], ev[2]) and min(ev[1], ev[2]) >= ev[3] == ev[4] > 0, ev
    assert ev[3] < 0.75 * ev[0], ev
    prm = gc.oracle_params(orc, batch_cap=256)
    fr = orc.frame(sc, cam, prm)
    cmax = float(fr.geo[fr.valid == 1, orc.G_R:orc.G_BL + 1].max())
    gc.check_image(runs[-1][0], runs[-1][1], fr.image, fr.T, fr.amb, {}, cmax)
