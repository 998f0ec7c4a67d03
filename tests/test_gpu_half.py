"""The reduced-precision mode on the GPU (sec. 3.5, sec. 4.2, sec. 4.5): the
packed SH codec against the oracle's (bit for bit), the projection on packed SH
against the oracle on the decoded coefficients (the float32 tolerance), and the
half-precision raster by PSNR, with pairs, order and batches identical to the
float32 mode.  The paper reports 67.0 dB for its fp16 renderer against a
float32 one, 55.6 dB with SH compression."""
import numpy as np
import pytest

from paper_2606_00352_amd import scenes
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu


def _psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return 10.0 * np.log10(1.0 / mse) if mse > 0 else np.inf


def _render(scene_tensors, cam, n, **params):
    import torch
    from paper_2606_00352_amd import higs
    ctx = higs.Context(n, cam.width, cam.height, **params)
    img, T = higs.render(ctx, scene_tensors, cam)
    torch.cuda.synchronize()
    return ctx, img.cpu().numpy(), T.cpu().numpy()


@pytest.mark.parametrize("which", ["config0", "clustered200k"])
def test_packed_sh_codec_and_projection(orc, which):
    import torch
    from oracle import shcodec
    from paper_2606_00352_amd import higs
    gc.need_gpu()
    if which == "config0":
        sc, cams = scenes.config0()
        cam = cams[0]
    else:
        sc = scenes.clustered_scene(200_000, seed=8, n_clusters=20)
        cam = scenes.orbit_cameras(4, 9, 640, 360, 380.0)[1]
    print(f"packed SH case: {which}", flush=True)
    t = higs.scene_tensors(sc)
    packed = higs.sh_compress(t[4], t[3])
    torch.cuda.synchronize()
    raw = packed.cpu().numpy().view(np.uint8)
    s, w = shcodec.compress(sc.sh, sc.opacities)
    np.testing.assert_array_equal(raw[:256].view(np.float32)[:48], s)
    np.testing.assert_array_equal(raw[256:].view(np.uint32).reshape(-1, 8), w)
    tp = (*t[:4], packed)
    ctx, img, T = _render(tp, cam, sc.n, sh_format=higs.SH_PACKED32)
    assert ctx.counts().overflow == 0
    dec = scenes.Scene(sc.means, sc.scales, sc.quats, sc.opacities, shcodec.decompress(s, w).reshape(sc.sh.shape))
    fr = orc.frame(dec, cam)
    report = {}
    gc.check_image(img, T, fr.image, fr.T, fr.amb, report, 2.0)
    full = orc.frame(sc, cam)
    report["psnr_vs_float_sh"] = round(_psnr(img, full.image), 2)
    print(report, flush=True)


@pytest.mark.parametrize("which", ["config0", "1080p_view0"])
def test_half_precision_raster(orc, which):
    from paper_2606_00352_amd import higs
    gc.need_gpu()
    if which == "config0":
        sc, cams = scenes.config0()
        cam = cams[0]
    else:
        sc, cams = scenes.config1()
        cam = cams[0]
    print(f"half raster case: {which}", flush=True)
    t = higs.scene_tensors(sc)
    c32, img32, T32 = _render(t, cam, sc.n)
    c16, img16, T16 = _render(t, cam, sc.n, raster_precision=higs.RASTER_FP16)
    # the half-precision partials merged by the merge kernel: the same image and T
    _, img16m, T16m = _render(t, cam, sc.n, raster_precision=higs.RASTER_FP16, fuse_merge=0)
    assert np.array_equal(img16m, img16) and np.array_equal(T16m, T16)
    k32, v32 = c32.sorted_pairs()
    k16, v16 = c16.sorted_pairs()
    assert np.array_equal(k32, k16) and np.array_equal(v32, v16)
    assert np.array_equal(c32.batches(), c16.batches())
    assert np.all(np.isfinite(img16)) and np.all((T16 >= 0) & (T16 <= 1))
    p_gpu = _psnr(img16, img32)
    rep = {"psnr_vs_float32_gpu": round(p_gpu, 2)}
    if which == "config0":
        fr = orc.frame(sc, cam)
        rep["psnr_vs_oracle"] = round(_psnr(img16, fr.image), 2)
        assert rep["psnr_vs_oracle"] >= 55.0
    print(rep, flush=True)
    assert p_gpu >= 50.0


def test_half_precision_refuses_the_adjoint():
    import torch
    from paper_2606_00352_amd import higs
    gc.need_gpu()
    sc, cams = scenes.config0()
    t = higs.scene_tensors(sc)
    ctx, img, T = _render(t, cams[0], sc.n, raster_precision=higs.RASTER_FP16)
    outs = [torch.empty_like(x) for x in t]
    with pytest.raises(higs.HigsError) as e:
        ctx.raster_backward(torch.zeros((256, 256, 3), device="cuda"), None, *outs)
    assert e.value.code == higs.E_UNSUPPORTED
