"""Pins of the oracle's gaussian-to-macro-tile test and pair emission (sec.
3.2 and sec. 4.3 of the paper) against brute force: dense sub-pixel sampling
of the opacity-level ellipse, and an independent closed-rectangle minimum of
the Mahalanobis form."""
import json
import math
import os

import numpy as np
import pytest

from paper_2606_00352_amd import scenes

HERE = os.path.dirname(os.path.abspath(__file__))


def _random_fields(rng, n, W, H):
    """(mx, my, a, b, c, tau) float32 with a positive-definite (a, b; b, c)."""
    out = []
    while len(out) < n:
        mx = rng.uniform(-40, W + 40)
        my = rng.uniform(-40, H + 40)
        s1, s2 = np.exp(rng.normal(math.log(6.0), 0.9, 2))
        th = rng.uniform(0, math.pi)
        c_, s_ = math.cos(th), math.sin(th)
        a = c_ * c_ * s1 * s1 + s_ * s_ * s2 * s2 + 0.3
        c = s_ * s_ * s1 * s1 + c_ * c_ * s2 * s2 + 0.3
        b = c_ * s_ * (s1 * s1 - s2 * s2)
        tau = rng.uniform(0.0, 2 * math.log(255))
        f = np.array([mx, my, a, b, c, tau], np.float32)
        if float(f[2]) * float(f[4]) - float(f[3]) ** 2 > 0:
            out.append(f)
    return out


def _qform(f, dx, dy):
    a, b, c = float(f[2]), float(f[3]), float(f[4])
    det = a * c - b * b
    return (c * dx * dx - 2 * b * dx * dy + a * dy * dy) / det


def _min_q_on_rect(f, x0, x1, y0, y1):
    """Minimum of q over the closed rectangle, by the boundary argument: the
    unconstrained minimum is the centre; otherwise it lies on an edge, where q
    is a 1D quadratic minimised by clamping its vertex."""
    mx, my = float(f[0]), float(f[1])
    a, b, c = float(f[2]), float(f[3]), float(f[4])
    if x0 <= mx <= x1 and y0 <= my <= y1:
        return 0.0
    best = math.inf
    for y in (y0, y1):           # horizontal edges: q(x) = (c dx^2 - 2b dx dy + a dy^2)/det
        dy = y - my
        dx = min(max(b * dy / c, x0 - mx), x1 - mx)
        best = min(best, _qform(f, dx, dy))
    for x in (x0, x1):           # vertical edges
        dx = x - mx
        dy = min(max(b * dx / a, y0 - my), y1 - my)
        best = min(best, _qform(f, dx, dy))
    return best


@pytest.mark.parametrize("W,H", [(256, 256), (200, 150), (130, 70)])
def test_predicate_equals_rectangle_minimum(orc, W, H):
    rng = np.random.default_rng(W * 1000 + H)
    nmx, nmy = orc.n_macro_tiles(W, H)
    checked = 0
    for f in _random_fields(rng, 400, W, H):
        got = set(orc.mt_list(f, W, H).tolist())
        tau = float(f[5])
        for j in range(nmy):
            for i in range(nmx):
                x0, x1 = 64.0 * i, min(64.0 * (i + 1), W)
                y0, y1 = 32.0 * j, min(32.0 * (j + 1), H)
                qmin = _min_q_on_rect(f, x0, x1, y0, y1)
                if abs(qmin - tau) <= 1e-9 * (1 + tau):
                    continue  # on the boundary: either answer is exact to rounding
                assert ((j * nmx + i) in got) == (qmin <= tau), (f, i, j, qmin, tau)
                checked += 1
    assert checked > 1000


def test_predicate_conservative_on_subpixel_grid(orc):
    W, H = 200, 150
    rng = np.random.default_rng(11)
    nmx, _ = orc.n_macro_tiles(W, H)
    xs = np.arange(0.125, W, 0.25)
    ys = np.arange(0.125, H, 0.25)
    X, Y = np.meshgrid(xs, ys)
    mtid = (Y // 32).astype(np.int64) * nmx + (X // 64).astype(np.int64)
    for f in _random_fields(rng, 120, W, H):
        q = _qform(f, X - float(f[0]), Y - float(f[1]))
        need = set(np.unique(mtid[q <= float(f[5])]).tolist())
        got = set(orc.mt_list(f, W, H).tolist())
        assert need <= got


def test_emission_order_and_counts(orc):
    sc, cams = scenes.config0()
    cam = cams[0]
    valid, geo = orc.project(sc, cam)
    counts, mt, key, gid = orc.bin_pairs(valid, geo, cam.width, cam.height)
    assert counts.sum() == mt.shape[0]
    assert np.all(np.diff(gid) >= 0)
    same = gid[1:] == gid[:-1]
    assert np.all(mt[1:][same] > mt[:-1][same])
    # every pair's key is the float32 depth of its gaussian; culled ones emit nothing
    np.testing.assert_array_equal(key, geo[gid, orc.G_TZ].astype(np.float32).view(np.uint32))
    assert np.all(counts[valid == 0] == 0)
    # per-gaussian list equals the stand-alone predicate
    f6 = orc.stored_fields(geo)
    for i in np.nonzero(counts)[0][:300]:
        np.testing.assert_array_equal(mt[gid == i], orc.mt_list(f6[i], cam.width, cam.height))


def test_macro_tile_grid_matches_paper_scale(orc):
    """The paper quotes ~1,000 macro-tiles at 1080p and ~4,000 at 4K for its
    64x32-pixel macro-tiles, and 30,000-130,000 8x8 render tiles."""
    with open(os.path.join(HERE, "golden", "macro_tile_scale.json")) as fh:
        gold = json.load(fh)
    for row in gold["cases"]:
        nmx, nmy = orc.n_macro_tiles(row["width"], row["height"])
        assert nmx * nmy == row["macro_tiles"]
        assert abs(nmx * nmy - row["paper_approx_macro_tiles"]) <= 0.03 * row["paper_approx_macro_tiles"]
        rt = ((row["width"] + 7) // 8) * ((row["height"] + 7) // 8)
        assert rt == row["render_tiles"]
