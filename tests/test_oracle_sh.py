"""Pins of the oracle's degree-3 SH colour (sec. 4.2 of the paper): the basis
against scipy's complex spherical harmonics, orthonormality by exact
quadrature, and the colour rule on simple configurations."""
import math

import numpy as np
import pytest
import scipy.special as sp

from paper_2606_00352_amd import scenes

# the library interface carries these parameters as float32
F32_DIL = float(np.float32(0.3))
F32_AMAX = float(np.float32(0.99))


def _real_sh_scipy(l, m, d):
    """Real SH with the Condon-Shortley phase kept (3DGS checkpoint
    convention): m<0 -> sqrt2 Im Y_l^|m|, m>0 -> sqrt2 Re Y_l^m."""
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x) % (2 * math.pi)
    if m == 0:
        return sp.sph_harm_y(l, 0, theta, phi).real
    val = sp.sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2.0) * (val.imag if m < 0 else val.real)


def test_basis_matches_scipy(orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        got = orc.sh_basis(d, 3)
        for l in range(4):
            for m in range(-l, l + 1):
                assert got[l * l + l + m] == pytest.approx(_real_sh_scipy(l, m, d), abs=1e-13)


def test_basis_orthonormal_by_quadrature(orc):
    # Gauss-Legendre in cos(theta) x uniform phi integrates degree <= 6 exactly
    xs, ws = np.polynomial.legendre.leggauss(16)
    nphi = 32
    G = np.zeros((16, 16))
    for ct, w in zip(xs, ws):
        st = math.sqrt(1 - ct * ct)
        for k in range(nphi):
            ph = 2 * math.pi * k / nphi
            y = orc.sh_basis([st * math.cos(ph), st * math.sin(ph), ct], 3)
            G += np.outer(y, y) * w * (2 * math.pi / nphi)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_lower_degree_zeroes_higher_bands(orc):
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    full = orc.sh_basis(d, 3)
    for deg in range(4):
        part = orc.sh_basis(d, deg)
        k = (deg + 1) ** 2
        np.testing.assert_array_equal(part[:k], full[:k])
        assert np.all(part[k:] == 0)


def _one(mean, sh, deg=3):
    return scenes.Scene(np.array([mean], np.float32), np.full((1, 3), 0.05, np.float32),
                        np.array([[1, 0, 0, 0]], np.float32), np.array([0.8], np.float32),
                        np.asarray(sh, np.float32).reshape(1, 16, 3))


def test_colour_degree0_and_view_direction(orc):
    cam = scenes.camera_at_origin(256, 256, 256.0)
    sh = np.zeros((16, 3))
    sh[0] = [0.2, -2.0, 2.0]
    sh[2] = [0.5, 0.0, -0.1]     # l=1, m=0: along the view axis
    _, geo = orc.project(_one([0, 0, 4.0], sh), cam, orc.Params(sh_degree=0))
    y00 = sp.sph_harm_y(0, 0, 0.0, 0.0).real
    exp0 = [max(0.0, 0.5 + y00 * float(np.float32(c))) for c in sh[0]]
    np.testing.assert_allclose(geo[0, orc.G_R:orc.G_BL + 1], exp0, rtol=1e-15)
    _, geo = orc.project(_one([0, 0, 4.0], sh), cam, orc.Params(sh_degree=1))
    y10 = sp.sph_harm_y(1, 0, 0.0, 0.0).real  # direction (0, 0, 1)
    exp1 = [max(0.0, 0.5 + y00 * float(np.float32(a)) + y10 * float(np.float32(b))) for a, b in zip(sh[0], sh[2])]
    np.testing.assert_allclose(geo[0, orc.G_R:orc.G_BL + 1], exp1, rtol=1e-15)
    assert geo[0, orc.G_G] == 0.0   # clamped at zero, no upper clamp
    assert geo[0, orc.G_BL] > 1.0


def test_colour_uses_direction_from_camera_centre(orc):
    # rotated, translated camera: direction = normalize(mean - eye)
    eye = np.array([3.0, -2.0, -9.0])
    cam = scenes.look_at_origin(eye, 256, 256, 256.0)
    rt = cam.world_to_cam.astype(np.float64)
    eye = -rt[:, :3].T @ rt[:, 3]        # the centre of the float32 camera
    sh = np.zeros((16, 3))
    sh[1] = [1.0, 0.0, 0.0]              # l=1, m=-1
    sh[3] = [0.0, 1.0, 0.0]              # l=1, m=+1
    sh[2] = [0.0, 0.0, 1.0]              # l=1, m=0
    mean = np.float32([0.4, 0.3, -0.2])
    _, geo = orc.project(_one(mean, sh), cam, orc.Params(sh_degree=1))
    d = mean.astype(np.float64) - eye
    d /= np.linalg.norm(d)
    for ch, (l, m) in enumerate([(1, -1), (1, 1), (1, 0)]):
        want = max(0.0, 0.5 + _real_sh_scipy(l, m, d))
        assert geo[0, orc.G_R + ch] == pytest.approx(want, abs=1e-7)
