"""The allocation-free entry point (higs_render_noalloc), called through the
C-ABI, against higs_render on a context: two calls in a row, the second with
fewer gaussians and a smaller image, each bit-identical to the context's frame
(both run the same kernels) and within the image tolerance of the oracle."""
import ctypes

import numpy as np
import pytest

from paper_2606_00352_amd import higs, scenes


@pytest.mark.gpu
def test_noalloc_matches_the_context_entry_point(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = higs.lib()
    sc, cams = scenes.config0()
    t = higs.scene_tensors(sc)
    small = scenes.camera_at_origin(160, 96, 140.0, (0.1, 0.2, 0.3))
    cases = [("config0 10000 gaussians 256x256", sc.n, cams[0]),
             ("3000 gaussians 160x96", 3000, small)]
    ctx = higs.Context(sc.n, 256, 256, max_pairs=1 << 17)
    stream = torch.cuda.current_stream().cuda_stream
    for name, n, cam in cases:
        print(f"noalloc case: {name}", flush=True)
        part = [x[:n].contiguous() for x in t]
        c = higs.camera_c(cam)
        img = torch.full((cam.height, cam.width, 3), -1.0, device="cuda")
        T = torch.full((cam.height, cam.width), -1.0, device="cuda")
        rc = lib.higs_render_noalloc(n, *(ctypes.c_void_p(x.data_ptr()) for x in part), ctypes.byref(c),
                                     ctypes.c_void_p(img.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                     ctypes.c_void_p(stream))
        assert rc == higs.OK
        torch.cuda.synchronize()
        ref_img = torch.full_like(img, -2.0)
        ref_T = torch.full_like(T, -2.0)
        ctx.render(*part, cam, ref_img, ref_T)
        torch.cuda.synchronize()
        assert ctx.counts().overflow == 0
        assert torch.equal(img, ref_img) and torch.equal(T, ref_T)
        fr = orc.frame(scenes.Scene(*(a[:n] for a in sc.arrays())), cam)
        d = np.abs(img.cpu().numpy().astype(np.float64) - fr.image)
        assert d[fr.amb == 0].max() <= 2e-4 and d.mean() <= 1e-5


def test_noalloc_rejects_sizes_beyond_its_limits():
    """Host-side checks: no work is queued for a size beyond the maxima."""
    lib = higs.lib()
    cam = higs.camera_c(scenes.camera_at_origin(64, 64, 64.0))
    null = ctypes.c_void_p(0)
    assert lib.higs_render_noalloc(131073, null, null, null, null, null, ctypes.byref(cam), ctypes.c_void_p(16),
                                   null, null) == higs.E_CAPACITY
    big = higs.camera_c(scenes.camera_at_origin(2048, 64, 64.0))
    assert lib.higs_render_noalloc(0, null, null, null, null, null, ctypes.byref(big), ctypes.c_void_p(16),
                                   null, null) == higs.E_CAPACITY
    assert lib.higs_render_noalloc(-1, null, null, null, null, null, ctypes.byref(cam), ctypes.c_void_p(16),
                                   null, null) == higs.E_INVALID
