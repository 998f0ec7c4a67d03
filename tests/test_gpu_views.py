"""Several views in one frame (higs_render_views): every stage runs once for
all of them, and each view's image and transmittance equal those of a
single-view frame of the same scene and camera, bit for bit.  Single-view
frames are pinned to the oracle by the parity tests; here the multi-view frame
is pinned to them, and one view of each frame to the oracle on sampled rows."""
import numpy as np
import pytest

from paper_2606_00352_amd import scenes
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu


def _single(tens, cam, n, **params):
    import torch
    from paper_2606_00352_amd import higs
    ctx = higs.Context(n, cam.width, cam.height, **params)
    img, T = higs.render(ctx, tens, cam)
    torch.cuda.synchronize()
    c = ctx.counts()
    ctx.close()
    return img, T, c


def _multi(views_in, n_max, max_pairs, **params):
    """views_in: [(tensors, cam)]; returns (images, Ts, counts, ctx)."""
    import torch
    from paper_2606_00352_amd import higs
    cam0 = views_in[0][1]
    ctx = higs.Context(n_max, cam0.width, cam0.height, max_pairs=max_pairs,
                       max_views=len(views_in), **params)
    outs = []
    for tens, cam in views_in:
        img = torch.full((cam.height, cam.width, 3), -1.0, device="cuda:0")
        T = torch.full((cam.height, cam.width), -1.0, device="cuda:0")
        outs.append((tens, cam, img, T))
    ctx.render_views(outs)
    torch.cuda.synchronize()
    return [o[2] for o in outs], [o[3] for o in outs], ctx.counts(), ctx


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_views_match_single_frames(precision):
    import torch
    from paper_2606_00352_amd import higs
    gc.need_gpu()
    prec = higs.RASTER_FP32 if precision == "fp32" else higs.RASTER_FP16
    a = scenes.clustered_scene(300_000, seed=21, n_clusters=30)
    b = scenes.clustered_scene(120_000, seed=22, n_clusters=12)
    ta, tb = higs.scene_tensors(a), higs.scene_tensors(b)
    cams = scenes.orbit_cameras(7, 5, 1280, 720, 730.0)
    views = [(ta, cams[0]), (tb, cams[1]), (ta, cams[2]), (ta, cams[3]), (tb, cams[6])]
    singles = [_single(t, c, int(t[0].shape[0]), raster_precision=prec) for t, c in views]
    pairs = sum(int(s[2].n_pairs) for s in singles)
    imgs, Ts, cnt, ctx = _multi(views, a.n, pairs + 4096, raster_precision=prec)
    assert cnt.overflow == 0 and cnt.n_pairs == pairs
    assert cnt.n_visible == sum(int(s[2].n_visible) for s in singles)
    for k, (img_s, T_s, _) in enumerate(singles):
        assert torch.equal(imgs[k], img_s), f"view {k} image"
        assert torch.equal(Ts[k], T_s), f"view {k} T"
    # the same context renders another set of views (fewer, other cameras)
    views2 = [(tb, cams[4]), (ta, cams[5])]
    singles2 = [_single(t, c, int(t[0].shape[0]), raster_precision=prec) for t, c in views2]
    outs = [(t, c, torch.empty((c.height, c.width, 3), device="cuda:0"),
             torch.empty((c.height, c.width), device="cuda:0")) for t, c in views2]
    ctx.render_views(outs)
    torch.cuda.synchronize()
    for k, (img_s, T_s, _) in enumerate(singles2):
        assert torch.equal(outs[k][2], img_s) and torch.equal(outs[k][3], T_s), f"second frame view {k}"
    ctx.close()


def test_one_view_of_a_frame_against_the_oracle(orc):
    """A view inside a three-view frame against the oracle's frame of that view
    alone, on every 16th pixel row (the parity tolerance)."""
    import torch
    from paper_2606_00352_amd import higs
    gc.need_gpu()
    sc = scenes.clustered_scene(150_000, seed=23, n_clusters=15)
    t = higs.scene_tensors(sc)
    cams = scenes.orbit_cameras(3, 9, 960, 544, 560.0)
    imgs, Ts, cnt, ctx = _multi([(t, c) for c in cams], sc.n, 3 * 8 * sc.n)
    assert cnt.overflow == 0
    ctx.close()
    cam = cams[1]
    fr = orc.frame(sc, cam, render=False)
    ys = np.arange(0, cam.height, 16)
    xs = np.arange(cam.width)
    pix = np.stack(np.meshgrid(xs, ys), -1).reshape(-1, 2)
    img_o, T_o, amb = orc.render_tiled(fr.geo, fr.sorted_gid, fr.mt_off, fr.batch_tab, cam, pixels=pix)
    g = imgs[1].cpu().numpy()[pix[:, 1], pix[:, 0]].astype(np.float64)
    d = np.abs(g - img_o)
    ok = amb == 0
    assert (~ok).mean() <= gc.AMB_MAX_FRACTION
    assert d[ok].max() <= gc.IMG_MAX_ABS and d.mean() <= gc.IMG_MEAN_ABS
    gT = Ts[1].cpu().numpy()[pix[:, 1], pix[:, 0]].astype(np.float64)
    assert np.abs(gT - T_o)[ok].max() <= gc.IMG_MAX_ABS


def test_views_overflow_and_arguments():
    """A frame whose pairs exceed the capacity stops: every view's image is
    NaN and the counts report the frame's need; a context of that size renders
    it.  Views of another size, more views than max_views, and a view count of
    zero are rejected before anything is enqueued."""
    import torch
    from paper_2606_00352_amd import higs
    gc.need_gpu()
    sc = scenes.clustered_scene(50_000, seed=24, n_clusters=5)
    t = higs.scene_tensors(sc)
    cams = scenes.orbit_cameras(2, 3, 640, 360, 380.0)
    imgs, Ts, cnt, ctx = _multi([(t, cams[0]), (t, cams[1])], sc.n, 1 << 14)
    assert cnt.overflow != 0 and cnt.n_pairs > (1 << 14)
    assert all(torch.isnan(i).all() for i in imgs)
    need = int(cnt.n_pairs)
    ctx.close()
    imgs, Ts, cnt, ctx = _multi([(t, cams[0]), (t, cams[1])], sc.n, need)
    assert cnt.overflow == 0 and all(torch.isfinite(i).all() for i in imgs)
    small = scenes.orbit_cameras(1, 3, 320, 180, 190.0)[0]
    bad = [(t, cams[0], imgs[0], Ts[0]), (t, small, imgs[1], Ts[1])]
    with pytest.raises(higs.HigsError):
        ctx.render_views(bad)
    three = [(t, cams[0], imgs[0], Ts[0])] * 3
    with pytest.raises(higs.HigsError):
        ctx.render_views(three)
    with pytest.raises(higs.HigsError):
        ctx.render_views([])
    ctx.close()
