"""Pins of the oracle's count of the pixel-gaussian evaluations the batched
form needs (oc_count_evals: the per-tile visibility of Alg. 1 taken exactly,
the unanimous early-out of Alg. 2, and the merge of Eq. 1 that stops reading
a tile's later batches once its transmittance is below t_eps)."""
import math

import numpy as np
import pytest

from paper_2606_00352_amd import scenes


def _iso(means, s, opac, w=64, h=64, f=64.0):
    n = len(means)
    sh = np.zeros((n, 16, 3), np.float32)
    sh[:, 0, :] = 0.5
    sc = scenes.Scene(np.asarray(means, np.float32), np.full((n, 3), s, np.float32),
                      np.tile(np.float32([1, 0, 0, 0]), (n, 1)), np.asarray(opac, np.float32), sh)
    return sc, scenes.camera_at_origin(w, h, f)


def test_single_gaussian_inside_one_tile(orc):
    """A compact splat centred in render tile (4, 4) of a 64x64 image: its
    level ellipse (radius sqrt(tau a) < 3 px) holds pixel centres of that tile
    only, so it is evaluated at 64 pixels once; with a second, farther copy
    and the first opaque, the merge still reads the second's tile (a single
    gaussian cannot drive T below 1e-4)."""
    sc, cam = _iso([[0.0, 0.0, 2.0]], 0.02, [0.9])  # centre (32, 32): tile (4, 4)
    fr = orc.frame(sc, cam, render=False)
    a = fr.geo[0, orc.G_A]
    assert math.sqrt(fr.geo[0, orc.G_TAU] * a) < 3.0
    # centre 32.0 is a tile corner: shift it to the middle of tile (4, 4)
    sc.means[0, :2] = np.float32(4.0 * 2.0 / 64.0)
    fr = orc.frame(sc, cam, render=False)
    assert orc.count_evals(fr.geo, fr.sorted_gid, fr.batch_tab, cam) == (64, 64)


def test_epsilon_zero_counts_every_tile_with_a_covered_centre(orc):
    """With t_eps = 0 nothing saturates: the count is 64 x the number of
    (gaussian, render tile) pairs with a pixel centre inside the gaussian's
    level ellipse, found here by brute force over every pixel of the image
    from the projected fields (no bounding box, no early-out)."""
    sc, cams = scenes.config0()
    cam = cams[0]
    prm = orc.Params(t_eps=0.0, batch_cap=64)
    fr = orc.frame(sc, cam, prm, render=False)
    g = fr.geo[fr.valid == 1]
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    px, py = xs.ravel() + 0.5, ys.ravel() + 0.5
    tile = (ys.ravel() // 8) * (cam.width // 8) + xs.ravel() // 8
    pairs = 0
    for r in g:
        dx, dy = px - r[orc.G_MX], py - r[orc.G_MY]
        q = (r[orc.G_L0] * dx + r[orc.G_L1] * dy) ** 2 + (r[orc.G_L2] * dy) ** 2
        pairs += np.unique(tile[q <= r[orc.G_TAU]]).size
    got = orc.count_evals(fr.geo, fr.sorted_gid, fr.batch_tab, cam, prm)
    assert got == (64 * pairs, 64 * pairs)


def test_saturation_and_merge_reduce_the_count(orc):
    """A stack of 40 wide opaque splats (sigma ~40 px) saturates the central
    tiles after a few gaussians: the early-out and the merge's stop can only
    remove evaluations, and with 4-gaussian batches the merge stops reading
    those tiles after the first batches."""
    n = 40
    means = [[0.0, 0.0, 2.0 + 0.01 * k] for k in range(n)]
    sc, cam = _iso(means, 1.25, [0.99] * n)
    sc.scales[:] = np.float32(1.25) * np.asarray([[2.0 + 0.01 * k] for k in range(n)], np.float32) / 2.0
    for cap in (4, 1024):
        prm0 = orc.Params(t_eps=0.0, batch_cap=cap)
        prm = orc.Params(batch_cap=cap)
        fr = orc.frame(sc, cam, prm, render=False)
        a0, r0 = orc.count_evals(fr.geo, fr.sorted_gid, fr.batch_tab, cam, prm0)
        a1, r1 = orc.count_evals(fr.geo, fr.sorted_gid, fr.batch_tab, cam, prm)
        assert a0 == r0 and a1 < a0 and r1 <= a1
        if cap == 4:
            assert r1 < a1
        else:
            assert r1 == a1  # one batch per macro-tile: the merge reads every first batch
