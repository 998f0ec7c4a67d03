// Gaussian-to-macro-tile intersection (sec. 3.2 of the paper, "conservative
// per-row ellipse-contour scan" at macro-tile granularity), evaluated exactly
// in double precision on the float32 stored fields so that the projection's
// count pass and the emission's fill pass take identical decisions.
//
// The ellipse {q <= tau}, q = (c dx^2 - 2 b dx dy + a dy^2) / det, is visited
// one macro-tile row (32-pixel band) at a time.  Over a band's clipped y-range
// the right branch x(dy) = (b/c) dy + sqrt((det/c)(tau - dy^2/c)) is concave,
// so its maximum sits at the clamp of its stationary point dy* = b sqrt(tau/a)
// into the range; the left branch is convex with its minimum at the clamp of
// -dy*.  Every macro-tile column between floor(x_min/64) and floor(x_max/64)
// is hit.  The operation order below is fixed (no contraction).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace higs {

struct BinFields {
  float mx, my, a, b, c, tau;
};

// Visits every macro-tile the ellipse meets, ascending (band j, then column
// i); fn(j, i) per hit.
template <class Fn>
__device__ __forceinline__ uint32_t visit_macro_tiles_ji(const BinFields& f, int width,
                                                         int height, int n_mt_x, int n_mt_y,
                                                         Fn&& fn) {
#pragma clang fp contract(off)
  const double mx = f.mx, my = f.my, a = f.a, b = f.b, c = f.c, tau = f.tau;
  const double W = (double)width, H = (double)height;
  const double det = a * c - b * b;
  const double ry = sqrt(tau * c);
  const double dys = b * sqrt(tau / a);
  // band range, clamped into [-1, n_mt_y] before conversion
  double vlo = floor((my - ry) / 32.0);
  double vhi = floor((my + ry) / 32.0);
  vlo = vlo < -1.0 ? -1.0 : (vlo > (double)n_mt_y ? (double)n_mt_y : vlo);
  vhi = vhi < -1.0 ? -1.0 : (vhi > (double)n_mt_y ? (double)n_mt_y : vhi);
  int jlo = (int)vlo, jhi = (int)vhi;
  if (jlo < 0) jlo = 0;
  if (jhi > n_mt_y - 1) jhi = n_mt_y - 1;
  uint32_t cnt = 0;
  for (int j = jlo; j <= jhi; ++j) {
    const double ytop = (double)(j * 32);
    double ybot = (double)((j + 1) * 32);
    if (ybot > H) ybot = H;
    double dlo = ytop - my, dhi = ybot - my;
    if (dlo < -ry) dlo = -ry;
    if (dhi > ry) dhi = ry;
    if (dlo > dhi) continue;
    double yp = dys, ym = -dys;
    if (yp < dlo) yp = dlo;
    if (yp > dhi) yp = dhi;
    if (ym < dlo) ym = dlo;
    if (ym > dhi) ym = dhi;
    double rp = (det / c) * (tau - (yp * yp) / c);
    double rm = (det / c) * (tau - (ym * ym) / c);
    if (rp < 0.0) rp = 0.0;
    if (rm < 0.0) rm = 0.0;
    const double xmax = (mx + (b / c) * yp) + sqrt(rp);
    const double xmin = (mx + (b / c) * ym) - sqrt(rm);
    if (xmax < 0.0 || xmin > W) continue;
    double ulo = floor(xmin / 64.0), uhi = floor(xmax / 64.0);
    ulo = ulo < -1.0 ? -1.0 : (ulo > (double)n_mt_x ? (double)n_mt_x : ulo);
    uhi = uhi < -1.0 ? -1.0 : (uhi > (double)n_mt_x ? (double)n_mt_x : uhi);
    int ilo = (int)ulo, ihi = (int)uhi;
    if (ilo < 0) ilo = 0;
    if (ihi > n_mt_x - 1) ihi = n_mt_x - 1;
    for (int i = ilo; i <= ihi; ++i) {
      fn(j, i);
      ++cnt;
    }
  }
  return cnt;
}

// Visits every macro-tile id the ellipse meets, ascending; fn(mt) per hit.
template <class Fn>
__device__ __forceinline__ uint32_t visit_macro_tiles(const BinFields& f, int width, int height,
                                                      int n_mt_x, int n_mt_y, Fn&& fn) {
  return visit_macro_tiles_ji(f, width, height, n_mt_x, n_mt_y,
                              [&](int j, int i) { fn((uint32_t)(j * n_mt_x + i)); });
}

// The same list in one 32-bit word when it is short: within a band the hits
// are one run of columns, so a list of at most two consecutive bands with at
// most 16 columns each (band < 256, column < 128) is
//   bit 31 set | band << 23 | first column << 16 | (columns - 1) << 12
//   | second band present << 11 | its first column << 4 | its columns - 1.
// Other lists encode as 0 (recompute them).  The projection records the word
// during its count; the fill expands it in the same order.
struct SpanTracker {
  int ja = -1, ia0 = 0, ia1 = 0, jb = -1, ib0 = 0, ib1 = 0;
  bool ok = true;
  __device__ __forceinline__ void add(int j, int i) {
    if (j == ja) ia1 = i;
    else if (ja < 0) ja = j, ia0 = ia1 = i;
    else if (j == jb) ib1 = i;
    else if (jb < 0 && j == ja + 1) jb = j, ib0 = ib1 = i;
    else ok = false;
  }
  __device__ __forceinline__ uint32_t encode() const {
    if (!ok || ja < 0 || ja > 255 || ia0 > 127 || ia1 - ia0 > 15) return 0u;
    uint32_t w = 0x80000000u | ((uint32_t)ja << 23) | ((uint32_t)ia0 << 16) |
                 ((uint32_t)(ia1 - ia0) << 12);
    if (jb >= 0) {
      if (ib0 > 127 || ib1 - ib0 > 15) return 0u;
      w |= 0x800u | ((uint32_t)ib0 << 4) | (uint32_t)(ib1 - ib0);
    }
    return w;
  }
};

// fn(mt) for every macro-tile of a nonzero span word, in visit order.
template <class Fn>
__device__ __forceinline__ void visit_span(uint32_t w, int n_mt_x, Fn&& fn) {
  const uint32_t ja = (w >> 23) & 255u, ia0 = (w >> 16) & 127u, la = (w >> 12) & 15u;
  for (uint32_t i = 0; i <= la; ++i) fn(ja * (uint32_t)n_mt_x + ia0 + i);
  if (w & 0x800u) {
    const uint32_t ib0 = (w >> 4) & 127u, lb = w & 15u;
    for (uint32_t i = 0; i <= lb; ++i) fn((ja + 1u) * (uint32_t)n_mt_x + ib0 + i);
  }
}

}  // namespace higs
