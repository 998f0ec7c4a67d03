"""The paper's 32-byte SH representation (sec. 4.2, the optional packed SH
front end), written plainly in numpy for the tests.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py); shares nothing with the
GPU library.

What sec. 4.2 states: the RGB SH coefficients go through the YCoCg colour
transform (the lifting form YCoCg-R, whose exact rational form is
Y = (R + 2G + B) / 4, Co = (R - B) / 2, Cg = (-R + 2G - B) / 4), a square-root
gamma, per-basis percentile scaling computed from the visible gaussians, and
quantisation to 6 bits of luma and 4 of chroma, 32 bytes per gaussian.

Readings taken where it says no more:
  * "visible" gaussians: those with opacity >= 1/255 (the only ones any view
    can show); the percentile is the 99.9th of |component| per (basis,
    component), taken as the upper edge of the 1024-bin histogram bin under the
    component's maximum in which the count first reaches it;
  * the DC basis, which 6/4 bits would render visibly wrong, uses the 46 bits
    the 15 higher bases leave free: 12/10/10;
  * a b-bit component stores rint(sgn(x) sqrt|x| M) + M, M = 2^(b-1) - 1, with
    x = clamp(c / scale, -1, 1); decoding gives y |y| scale, y = (code - M) / M;
  * layout: word 0 = DC (Y | Co << 12 | Cg << 22), words 1..7 a bit stream
    holding basis k = 1..15 at bit 14 (k - 1) as Y | Co << 6 | Cg << 10.
Encoding decides integers from float arithmetic, so it is written in float32
with the operation order of its definition (no fused operations), as the
kernels evaluate it.
"""
from __future__ import annotations

import numpy as np

BASES = 16
DC_BITS = (12, 10, 10)
AC_BITS = (6, 4, 4)
AC_WIDTH = sum(AC_BITS)
PERCENTILE = 0.999
BINS = 1024
F = np.float32


def to_ycocg(rgb):
    """[..., 3] float32 -> [..., 3] (Y, Co, Cg), float32, term by term."""
    r, g, b = (rgb[..., k].astype(F) for k in range(3))
    y = (F(0.25) * r + F(0.5) * g) + F(0.25) * b
    co = F(0.5) * r - F(0.5) * b
    cg = (F(-0.25) * r + F(0.5) * g) - F(0.25) * b
    return np.stack([y, co, cg], -1)


def from_ycocg(c):
    y, co, cg = (c[..., k].astype(F) for k in range(3))
    return np.stack([(y + co) - cg, y + cg, (y - co) - cg], -1)


def scales(sh, opacities):
    """[48] float32: per (basis, component) the percentile scale."""
    vis = (opacities.astype(F) * F(255.0)) >= F(1.0)
    c = np.abs(to_ycocg(sh[vis].reshape(-1, BASES, 3)).reshape(-1, 3 * BASES))
    n_valid = c.shape[0]
    out = np.ones(3 * BASES, dtype=F)
    need = int(np.ceil(PERCENTILE * n_valid))
    for k in range(3 * BASES):
        mx = c[:, k].max() if n_valid else F(0.0)
        if not mx > 0:
            continue
        bins = np.minimum(np.floor((c[:, k] / mx) * F(BINS)).astype(np.int64), BINS - 1)
        cum = np.cumsum(np.bincount(bins, minlength=BINS))
        found = int(np.nonzero(cum >= need)[0][0]) if need > 0 else 0
        s = (F(mx) * F(found + 1)) / F(BINS)
        out[k] = s if s > 0 else F(1.0)
    return out


def quantise(c, scale, bits):
    m = F((1 << (bits - 1)) - 1)
    x = np.clip(c.astype(F) / F(scale), F(-1.0), F(1.0))
    y = np.copysign(np.sqrt(np.abs(x)), x).astype(F)
    return (np.rint(y * m) + m).astype(np.int64).astype(np.uint32)


def dequantise(code, bits, scale):
    m = F((1 << (bits - 1)) - 1)
    y = (code.astype(F) - m) / m
    return (y * np.abs(y)) * F(scale)


def compress(sh, opacities):
    """(scales [48] float32, words [n, 8] uint32) of sh [n, 16, 3]."""
    sh = np.asarray(sh, dtype=F).reshape(-1, BASES, 3)
    s = scales(sh, np.asarray(opacities, dtype=F))
    c = to_ycocg(sh)
    n = sh.shape[0]
    words = np.zeros((n, 8), dtype=np.uint64)
    w0 = quantise(c[:, 0, 0], s[0], DC_BITS[0]).astype(np.uint64)
    w0 |= quantise(c[:, 0, 1], s[1], DC_BITS[1]).astype(np.uint64) << np.uint64(DC_BITS[0])
    w0 |= quantise(c[:, 0, 2], s[2], DC_BITS[2]).astype(np.uint64) << np.uint64(DC_BITS[0] + DC_BITS[1])
    words[:, 0] = w0
    for k in range(1, BASES):
        v = quantise(c[:, k, 0], s[3 * k], AC_BITS[0]).astype(np.uint64)
        v |= quantise(c[:, k, 1], s[3 * k + 1], AC_BITS[1]).astype(np.uint64) << np.uint64(AC_BITS[0])
        v |= quantise(c[:, k, 2], s[3 * k + 2], AC_BITS[2]).astype(np.uint64) << np.uint64(AC_BITS[0] + AC_BITS[1])
        # basis k at bit 14 (k - 1) of the stream in words 1..7
        bit = AC_WIDTH * (k - 1)
        wi, sh = 1 + bit // 32, bit % 32
        words[:, wi] |= (v << np.uint64(sh)) & np.uint64(0xFFFFFFFF)
        if sh + AC_WIDTH > 32:
            words[:, wi + 1] |= v >> np.uint64(32 - sh)
    return s, words.astype(np.uint32)


def decompress(s, words):
    """[n, 16, 3] float32 RGB coefficients decoded from (scales, words)."""
    words = np.asarray(words, dtype=np.uint64)
    n = words.shape[0]
    c = np.zeros((n, BASES, 3), dtype=F)
    w0 = words[:, 0]
    mask = lambda b: np.uint64((1 << b) - 1)
    c[:, 0, 0] = dequantise(w0 & mask(DC_BITS[0]), DC_BITS[0], s[0])
    c[:, 0, 1] = dequantise((w0 >> np.uint64(DC_BITS[0])) & mask(DC_BITS[1]), DC_BITS[1], s[1])
    c[:, 0, 2] = dequantise((w0 >> np.uint64(DC_BITS[0] + DC_BITS[1])) & mask(DC_BITS[2]), DC_BITS[2], s[2])
    for k in range(1, BASES):
        bit = AC_WIDTH * (k - 1)
        wi, sh = 1 + bit // 32, bit % 32
        v = words[:, wi] >> np.uint64(sh)
        if sh + AC_WIDTH > 32:
            v |= words[:, wi + 1] << np.uint64(32 - sh)
        c[:, k, 0] = dequantise(v & mask(AC_BITS[0]), AC_BITS[0], s[3 * k])
        c[:, k, 1] = dequantise((v >> np.uint64(AC_BITS[0])) & mask(AC_BITS[1]), AC_BITS[1], s[3 * k + 1])
        c[:, k, 2] = dequantise((v >> np.uint64(AC_BITS[0] + AC_BITS[1])) & mask(AC_BITS[2]), AC_BITS[2],
                                s[3 * k + 2])
    return from_ycocg(c)
