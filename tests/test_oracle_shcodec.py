"""Pins of the oracle's 32-byte SH codec (oracle/shcodec.py, sec. 4.2's
YCoCg + square-root gamma + per-basis percentile scaling, 6/4 bits)."""
import numpy as np
import pytest

from oracle import shcodec as sc

F = np.float32


def test_ycocg_is_the_rational_transform_and_inverts_exactly():
    # the rational matrix of YCoCg and its inverse (numpy's solve)
    M = np.array([[0.25, 0.5, 0.25], [0.5, 0.0, -0.5], [-0.25, 0.5, -0.25]])
    rng = np.random.default_rng(1)
    # dyadic values: every step of the transform is exact in float32
    rgb = (rng.integers(-512, 512, (4000, 3)) / 64.0).astype(F)
    c = sc.to_ycocg(rgb)
    np.testing.assert_array_equal(c.astype(np.float64), rgb.astype(np.float64) @ M.T)
    back = sc.from_ycocg(c)
    np.testing.assert_array_equal(back, rgb)
    np.testing.assert_allclose(np.linalg.solve(M, c.astype(np.float64).T).T, rgb, atol=0)


@pytest.mark.parametrize("bits", [4, 6, 10, 12])
def test_quantiser_grid_and_error_bound(bits):
    m = (1 << (bits - 1)) - 1
    codes = np.arange(2 * m + 1, dtype=np.uint32)
    vals = sc.dequantise(codes, bits, 1.0)
    # the grid is symmetric, monotone, hits -1, 0, 1, and re-encodes to itself
    assert vals[0] == -1.0 and vals[m] == 0.0 and vals[-1] == 1.0
    assert np.all(np.diff(vals) > 0)
    np.testing.assert_array_equal(sc.quantise(vals, 1.0, bits), codes)
    # error bound of the sqrt-domain quantiser: |y - y_q| <= 1/(2M), so
    # |x - x_q| = |y^2 - y_q^2| <= (2|y| + 1/(2M)) / (2M)
    x = np.linspace(-1, 1, 20001).astype(F)
    xq = sc.dequantise(sc.quantise(x, 1.0, bits), bits, 1.0)
    y = np.sqrt(np.abs(x.astype(np.float64)))
    bound = (2 * y + 1 / (2 * m)) / (2 * m) + 1e-6
    assert np.all(np.abs(xq - x) <= bound)
    # outside [-scale, scale] the value clamps to the end codes
    assert sc.quantise(np.array([5.0, -5.0], F), 1.0, bits).tolist() == [2 * m, 0]


def test_scale_is_the_percentile_bin_edge():
    rng = np.random.default_rng(2)
    n = 20000
    sh = rng.normal(0, 0.1, (n, 16, 3)).astype(F)
    sh[:, 0] = rng.uniform(0, 1, (n, 3))
    op = rng.uniform(0, 1, n).astype(F)
    op[::7] = 0.001  # below 1/255: left out of the scaling
    s = sc.scales(sh, op)
    vis = op * F(255) >= 1
    c = np.abs(sc.to_ycocg(sh[vis]).reshape(-1, 48)).astype(np.float64)
    for k in range(48):
        q = np.quantile(c[:, k], sc.PERCENTILE, method="inverted_cdf")
        assert q <= s[k] * (1 + 1e-6)
        assert s[k] - q <= c[:, k].max() / sc.BINS * (1 + 1e-6)


def test_bit_layout():
    """Words built by hand from chosen codes decode to those codes' values."""
    rng = np.random.default_rng(3)
    s = rng.uniform(0.5, 2.0, 48).astype(F)
    n = 50
    dc = [rng.integers(0, 1 << b, n) for b in sc.DC_BITS]
    ac = [[rng.integers(0, 1 << b, n) for b in sc.AC_BITS] for _ in range(15)]
    words = np.zeros((n, 8), np.uint32)
    for i in range(n):
        words[i, 0] = int(dc[0][i]) | (int(dc[1][i]) << 12) | (int(dc[2][i]) << 22)
        acc = 0
        for k in range(15):
            f = int(ac[k][0][i]) | (int(ac[k][1][i]) << 6) | (int(ac[k][2][i]) << 10)
            acc |= f << (14 * k)
        for w in range(7):
            words[i, 1 + w] = (acc >> (32 * w)) & 0xFFFFFFFF
    got = sc.decompress(s, words)
    want = np.zeros((n, 16, 3), F)
    for q, b in enumerate(sc.DC_BITS):
        want[:, 0, q] = sc.dequantise(dc[q].astype(np.uint32), b, s[q])
    for k in range(15):
        for q, b in enumerate(sc.AC_BITS):
            want[:, k + 1, q] = sc.dequantise(ac[k][q].astype(np.uint32), b, s[3 * (k + 1) + q])
    np.testing.assert_array_equal(got, sc.from_ycocg(want))


def test_round_trip_within_the_quantiser_bound():
    rng = np.random.default_rng(4)
    n = 3000
    sh = rng.normal(0, 0.1, (n, 16, 3)).astype(F)
    sh[:, 0] = rng.uniform(0, 1, (n, 3))
    op = np.ones(n, F)
    s, w = sc.compress(sh, op)
    assert w.shape == (n, 8) and w.dtype == np.uint32
    d = sc.decompress(s, w)
    c, cd = sc.to_ycocg(sh).astype(np.float64), sc.to_ycocg(d).astype(np.float64)
    for k in range(16):
        bits = sc.DC_BITS if k == 0 else sc.AC_BITS
        for q in range(3):
            m = (1 << (bits[q] - 1)) - 1
            scale = float(s[3 * k + q])
            inside = np.abs(c[:, k, q]) <= scale
            err = np.abs(cd[:, k, q] - c[:, k, q])[inside]
            assert err.max(initial=0) <= scale * (2 / (2 * m) + 1 / (4 * m * m)) + 1e-5
