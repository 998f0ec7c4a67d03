"""Shared helpers of the GPU parity tests: run the HIP path through the C-ABI
binding and compare each stage with the oracle."""
import numpy as np
import pytest

IMG_MAX_ABS = 2e-4   # per channel, pixels not flagged ambiguous
IMG_MEAN_ABS = 1e-5  # per channel, all pixels
# Pixels the oracle may flag ambiguous (an alpha decided within the pinned
# float32 band of 1/255, or a transmittance next to t_eps), as a fraction of
# the compared pixels: ~0.1% on the parity scene, ~0.6% on a 1080p view of the
# benchmark scene, where float32 centres near x = 1000 px widen the band.
AMB_MAX_FRACTION = 0.01
COLOUR_ABS = 2e-6    # float32 SH colour against the double oracle


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_frame(scene, cam, keep_pairs=True, ctx=None, debug=0, **params):
    """Renders one frame on the GPU; returns (ctx, image, T) with numpy outputs."""
    import torch
    from paper_2606_00352_amd import higs
    need_gpu()
    if ctx is None:
        n = max(scene.n, 1)
        ctx = higs.Context(n, cam.width, cam.height, max_pairs=max(64 * n, 1 << 16), **params)
    if keep_pairs:
        # every binning field stored too, for the projection's bit-exact check
        ctx.set_debug(higs.DEBUG_KEEP_PAIRS | higs.DEBUG_PROJ_FIELDS | debug)
    t = higs.scene_tensors(scene)
    img, T = higs.render(ctx, t, cam)
    torch.cuda.synchronize()
    c = ctx.counts()
    assert c.overflow == 0, "capacity overflow"
    return ctx, img.cpu().numpy(), T.cpu().numpy()


def oracle_params(orc, **params):
    p = orc.Params()
    for k, v in params.items():
        setattr(p, k, v)
    return p


def check_projection(orc, ctx, fr, report):
    """Float32 geometry fields bit-exact; colour within COLOUR_ABS."""
    pf = ctx.proj_fields()
    valid = fr.valid.astype(bool)
    culled_gpu = pf["key"] == 0
    np.testing.assert_array_equal(culled_gpu, ~valid, err_msg="culling decisions differ")
    f6 = orc.stored_fields(fr.geo)
    names = ["mx", "my", "a", "b", "c", "tau"]
    for k, nm in enumerate(names):
        g = pf[nm][valid].view(np.uint32)
        o = f6[valid, k].view(np.uint32)
        bad = np.nonzero(g != o)[0]
        if nm == "tau" and bad.size:
            # a 1-ulp difference of the two libraries' log can only move the
            # float32 rounding when the double value sits at a rounding tie
            tau64 = fr.geo[valid, orc.G_TAU][bad]
            lo = np.nextafter(f6[valid, k][bad], np.float32(-np.inf)).astype(np.float64)
            hi = np.nextafter(f6[valid, k][bad], np.float32(np.inf)).astype(np.float64)
            mid_gap = np.minimum(np.abs(tau64 - (lo + f6[valid, k][bad]) / 2), np.abs(tau64 - (hi + f6[valid, k][bad]) / 2))
            assert np.all(mid_gap <= 1e-12 * np.abs(tau64)), "tau mismatch away from a rounding tie"
            report["tau_ulp_cases"] = int(bad.size)
        else:
            assert bad.size == 0, f"field {nm}: {bad.size} mismatches, first gid {np.nonzero(valid)[0][bad[:5]]}"
    np.testing.assert_array_equal(pf["key"][valid], fr.geo[valid, orc.G_TZ].astype(np.float32).view(np.uint32))
    np.testing.assert_array_equal(pf["count"].astype(np.int64), fr.counts.astype(np.int64))
    rec = ctx.records()
    vis = fr.counts > 0
    for col, gcol in ((2, orc.G_L0), (3, orc.G_L1), (4, orc.G_L2)):
        np.testing.assert_array_equal(rec[vis, col].view(np.uint32), fr.geo[vis, gcol].astype(np.float32).view(np.uint32))
    np.testing.assert_array_equal(rec[vis, 5], fr.geo[vis, orc.G_OP].astype(np.float32))
    if vis.any():
        d = np.abs(rec[vis, 6:9].astype(np.float64) - fr.geo[vis, orc.G_R:orc.G_BL + 1])
        report["colour_max_abs"] = float(d.max())
        assert d.max() <= COLOUR_ABS


def check_pairs_sort_batches(orc, ctx, fr, cap, check_emission=True):
    n_mt = ctx.n_mt
    if check_emission:
        keys, vals = ctx.pairs()
        want = (fr.pairs_mt.astype(np.uint64) << np.uint64(32)) | fr.pairs_key.astype(np.uint64)
        if ctx.params.sort_mode == 0:
            # segmented binning writes each macro-tile's pairs in any order: the
            # pair set is what is unique, and the segments must be contiguous
            order_g = np.lexsort((vals, keys))
            order_o = np.lexsort((fr.pairs_gid, want))
            np.testing.assert_array_equal(keys[order_g], want[order_o], err_msg="emitted keys differ")
            np.testing.assert_array_equal(vals[order_g], fr.pairs_gid[order_o].astype(np.uint32),
                                          err_msg="emitted ids differ")
            mts = keys >> np.uint64(32)
            assert np.all(np.diff(mts.astype(np.int64)) >= 0), "segments not contiguous"
        else:
            np.testing.assert_array_equal(keys, want, err_msg="emitted keys differ")
            np.testing.assert_array_equal(vals, fr.pairs_gid.astype(np.uint32), err_msg="emitted ids differ")
    keys, vals = ctx.sorted_pairs()
    want = (fr.sorted_mt.astype(np.uint64) << np.uint64(32)) | fr.sorted_key.astype(np.uint64)
    np.testing.assert_array_equal(keys, want, err_msg="sorted keys differ")
    np.testing.assert_array_equal(vals, fr.sorted_gid.astype(np.uint32), err_msg="sorted ids differ")
    np.testing.assert_array_equal(ctx.mt_offsets().astype(np.int64), fr.mt_off[:n_mt + 1])
    np.testing.assert_array_equal(ctx.batches().astype(np.int64), fr.batch_tab.astype(np.int64))


def check_image(img, T, o_img, o_T, amb, report, cmax=None):
    """Max abs over unambiguous pixels, mean abs over all, per channel."""
    d = np.abs(img.astype(np.float64) - o_img)
    clean = amb == 0
    report["ambiguous_pixels"] = int((~clean).sum())
    report["ambiguous_fraction"] = float((~clean).mean()) if clean.size else 0.0
    assert report["ambiguous_fraction"] <= AMB_MAX_FRACTION, report
    report["max_abs"] = float(d[clean].max()) if clean.any() else 0.0
    report["mean_abs"] = float(d.mean()) if d.size else 0.0
    if clean.any():
        worst = np.unravel_index(np.argmax(np.where(clean[..., None], d, 0)), d.shape)
        report["worst_pixel"] = tuple(int(v) for v in worst)
    assert report["max_abs"] <= IMG_MAX_ABS, report
    for ch in range(3):
        assert d[..., ch].mean() <= IMG_MEAN_ABS, report
    dT = np.abs(T.astype(np.float64) - o_T)
    assert dT[clean].max(initial=0.0) <= IMG_MAX_ABS
    if (~clean).any():
        # an alpha decided at 1/255 moves a pixel by at most ~2/255 of its colour scale
        bound = 2.0 / 255.0 * max(1.0, cmax or 1.0)
        assert d[~clean].max() <= bound, (d[~clean].max(), bound)
