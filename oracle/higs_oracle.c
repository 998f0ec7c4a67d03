/*
 * Plain FP64 CPU oracle for the HiGS forward frame path
 * (Pajak, Bisson, Lima: "HiGS: A Hierarchical Rendering Architecture for
 * Real-Time 3D Gaussian Splatting", arXiv 2606.00352).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library; the two are written
 * independently from the same definitions.
 *
 * Everything is double precision on float inputs widened exactly, evaluated
 * in the written operation order (built with -ffp-contract=off, no fast-math).
 * The pieces, with the part of the paper each follows:
 *   - oc_project:       per-gaussian EWA projection, Cholesky factors of the
 *                       inverse covariance (sec. 3.5, Numerical
 *                       representation), opacity level, depth key
 *                       (sec. 4.3, Fill pass), degree<=3 SH colour (sec. 4.2).
 *   - oc_mt_list / oc_bin_count / oc_bin_fill:
 *                       gaussian-to-macro-tile intersection and pair emission
 *                       (sec. 3.2, Gaussian partitioning; sec. 4.3).
 *   - oc_sort_pairs:    ordering of each macro-tile's list by depth
 *                       (sec. 3.3, Segmented depth sort), ties by gaussian id.
 *   - oc_batches:       split of each macro-tile list into batches of at most
 *                       B_r gaussians (sec. 3.1).
 *   - oc_render_untiled: the plain definition of the image: per pixel, all
 *                       gaussians in depth order, sequential front-to-back
 *                       compositing (sec. 3.4; Eq. 1 with one gaussian per
 *                       "batch").
 *   - oc_render_tiled:  per (macro-tile, batch) partial (C, T) from (0, 1),
 *                       then the post-blend merge of Eq. 1 with its
 *                       transmittance early-out (sec. 3.4, Post-rasterization
 *                       compositing).
 * Parity of the paper-level fidelity figures (PSNR against a trained model)
 * is unpinned here: it needs datasets that are not available.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "higs_oracle.h"

static int is_finite_d(double v) { return isfinite(v) != 0; }

/* ---------------------------------------------------------------- SH ---- */
/* Real spherical harmonics up to degree 3 in the sign convention of the
 * standard 3DGS checkpoints (Condon-Shortley phase kept in the real form):
 * for m < 0, sqrt(2) Im Y_l^|m|; m = 0, Y_l^0; m > 0, sqrt(2) Re Y_l^m.
 * Index k = l*l + l + m.  Normalisations are written from their closed forms. */
void oc_sh_basis(const double d[3], int degree, double out[16]) {
  const double pi = 3.14159265358979323846;
  double x = d[0], y = d[1], z = d[2];
  for (int k = 0; k < 16; ++k) out[k] = 0.0;
  out[0] = 0.5 * sqrt(1.0 / pi);
  if (degree < 1) return;
  double k1 = sqrt(3.0 / (4.0 * pi));
  out[1] = -k1 * y;
  out[2] = k1 * z;
  out[3] = -k1 * x;
  if (degree < 2) return;
  double xx = x * x, yy = y * y, zz = z * z;
  double k2a = 0.5 * sqrt(15.0 / pi);
  double k2b = 0.25 * sqrt(5.0 / pi);
  double k2c = 0.25 * sqrt(15.0 / pi);
  out[4] = k2a * (x * y);
  out[5] = -k2a * (y * z);
  out[6] = k2b * (2.0 * zz - xx - yy);
  out[7] = -k2a * (x * z);
  out[8] = k2c * (xx - yy);
  if (degree < 3) return;
  double k3a = 0.25 * sqrt(35.0 / (2.0 * pi));
  double k3b = 0.5 * sqrt(105.0 / pi);
  double k3c = 0.25 * sqrt(21.0 / (2.0 * pi));
  double k3d = 0.25 * sqrt(7.0 / pi);
  double k3e = 0.25 * sqrt(105.0 / pi);
  out[9] = -k3a * y * (3.0 * xx - yy);
  out[10] = k3b * x * y * z;
  out[11] = -k3c * y * (4.0 * zz - xx - yy);
  out[12] = k3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
  out[13] = -k3c * x * (4.0 * zz - xx - yy);
  out[14] = k3e * z * (xx - yy);
  out[15] = -k3a * x * (xx - 3.0 * yy);
}

/* ------------------------------------------------------- projection ---- */
/* One gaussian.  Returns 1 if it survives the culls, 0 otherwise; on 1 the
 * G_NCOL doubles of rec are filled.  Operation order is fixed as written. */
static int project_one(const float* mean, const float* scale, const float* quat,
                       float opac, const float* sh, const oc_camera* cam,
                       const oc_params* prm, double* rec) {
  double R[9], t[3];
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) R[r * 3 + k] = (double)cam->world_to_cam[r * 4 + k];
    t[r] = (double)cam->world_to_cam[r * 4 + 3];
  }
  double mx = mean[0], my = mean[1], mz = mean[2];
  double s0 = scale[0], s1 = scale[1], s2 = scale[2];
  double qw = quat[0], qx = quat[1], qy = quat[2], qz = quat[3];
  double o = opac;
  if (!(is_finite_d(mx) && is_finite_d(my) && is_finite_d(mz) && is_finite_d(s0) &&
        is_finite_d(s1) && is_finite_d(s2) && is_finite_d(qw) && is_finite_d(qx) &&
        is_finite_d(qy) && is_finite_d(qz) && is_finite_d(o)))
    return 0;

  /* camera-space mean */
  double tc[3];
  for (int r = 0; r < 3; ++r)
    tc[r] = ((R[r * 3 + 0] * mx + R[r * 3 + 1] * my) + R[r * 3 + 2] * mz) + t[r];
  double tx = tc[0], ty = tc[1], tz = tc[2];
  if (!(tz > prm->near_z)) return 0;

  /* unit quaternion -> rotation matrix */
  double n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  if (!(n2 > 0.0)) return 0;
  double nrm = sqrt(n2);
  double w = qw / nrm, x = qx / nrm, y = qy / nrm, z = qz / nrm;
  double G[9];
  G[0] = 1.0 - 2.0 * (y * y + z * z);
  G[1] = 2.0 * (x * y - w * z);
  G[2] = 2.0 * (x * z + w * y);
  G[3] = 2.0 * (x * y + w * z);
  G[4] = 1.0 - 2.0 * (x * x + z * z);
  G[5] = 2.0 * (y * z - w * x);
  G[6] = 2.0 * (x * z - w * y);
  G[7] = 2.0 * (y * z + w * x);
  G[8] = 1.0 - 2.0 * (x * x + y * y);

  /* world covariance: Sigma = (G S)(G S)^T */
  double M[9];
  for (int i = 0; i < 3; ++i) {
    M[i * 3 + 0] = G[i * 3 + 0] * s0;
    M[i * 3 + 1] = G[i * 3 + 1] * s1;
    M[i * 3 + 2] = G[i * 3 + 2] * s2;
  }
  double S[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      S[i * 3 + j] = (M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1]) +
                     M[i * 3 + 2] * M[j * 3 + 2];

  /* local affine (EWA) approximation of the perspective map */
  double fx = cam->fx, fy = cam->fy, cx = cam->cx, cy = cam->cy;
  double W = cam->width, H = cam->height;
  double tanx = W / (2.0 * fx), tany = H / (2.0 * fy);
  double xlo = -(cx / fx + 0.3 * tanx), xhi = (W - cx) / fx + 0.3 * tanx;
  double ylo = -(cy / fy + 0.3 * tany), yhi = (H - cy) / fy + 0.3 * tany;
  double xr = tx / tz, yr = ty / tz;
  if (xr < xlo) xr = xlo;
  if (xr > xhi) xr = xhi;
  if (yr < ylo) yr = ylo;
  if (yr > yhi) yr = yhi;
  double xc = xr * tz, yc = yr * tz;
  double j00 = fx / tz, j02 = -(fx * xc) / (tz * tz);
  double j11 = fy / tz, j12 = -(fy * yc) / (tz * tz);
  double T0[3], T1[3];
  for (int k = 0; k < 3; ++k) {
    T0[k] = j00 * R[0 * 3 + k] + j02 * R[2 * 3 + k];
    T1[k] = j11 * R[1 * 3 + k] + j12 * R[2 * 3 + k];
  }
  double U0[3], U1[3];
  for (int k = 0; k < 3; ++k) {
    U0[k] = (T0[0] * S[0 * 3 + k] + T0[1] * S[1 * 3 + k]) + T0[2] * S[2 * 3 + k];
    U1[k] = (T1[0] * S[0 * 3 + k] + T1[1] * S[1 * 3 + k]) + T1[2] * S[2 * 3 + k];
  }
  double s00 = (U0[0] * T0[0] + U0[1] * T0[1]) + U0[2] * T0[2];
  double s01 = (U0[0] * T1[0] + U0[1] * T1[1]) + U0[2] * T1[2];
  double s11 = (U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2];
  double a = s00 + prm->dilation, b = s01, c = s11 + prm->dilation;
  double det = a * c - b * b;
  if (!(det > 0.0)) return 0;

  /* opacity level: o exp(-q/2) >= 1/255  <=>  q <= tau = 2 ln(255 o); the
   * product 255 o of a float by 255 is exact in double, so is the cull test */
  if (!(255.0 * o >= 1.0)) return 0;
  double tau = 2.0 * log(255.0 * o);

  /* Cholesky factors of the inverse covariance (sec. 3.5) */
  double l0 = sqrt(c / det);
  double l1 = -b / sqrt(c * det);
  double l2 = 1.0 / sqrt(c);

  double px = (fx * tx) / tz + cx;
  double py = (fy * ty) / tz + cy;

  /* view-dependent colour from degree-<=3 SH */
  double campos[3];
  for (int k = 0; k < 3; ++k)
    campos[k] = -((R[0 * 3 + k] * t[0] + R[1 * 3 + k] * t[1]) + R[2 * 3 + k] * t[2]);
  double d[3] = {mx - campos[0], my - campos[1], mz - campos[2]};
  double dn = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
  if (dn > 0.0) { d[0] /= dn; d[1] /= dn; d[2] /= dn; }
  double Y[16];
  oc_sh_basis(d, prm->sh_degree, Y);
  int ncoef = (prm->sh_degree + 1) * (prm->sh_degree + 1);
  double rgb[3];
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.0;
    for (int k = 0; k < ncoef; ++k) acc += Y[k] * (double)sh[k * 3 + ch];
    double v = 0.5 + acc;
    rgb[ch] = v > 0.0 ? v : 0.0;
  }

  rec[G_TZ] = tz; rec[G_MX] = px; rec[G_MY] = py;
  rec[G_A] = a; rec[G_B] = b; rec[G_C] = c; rec[G_TAU] = tau;
  rec[G_L0] = l0; rec[G_L1] = l1; rec[G_L2] = l2; rec[G_OP] = o;
  rec[G_R] = rgb[0]; rec[G_G] = rgb[1]; rec[G_BL] = rgb[2];
  return 1;
}

/* Projects n gaussians.  valid[i] = 1 if gaussian i survives the culls,
 * geo[i*G_NCOL + ...] its double record.  Returns the number valid. */
int64_t oc_project(int64_t n, const float* means, const float* scales, const float* quats,
                   const float* opac, const float* sh, const oc_camera* cam,
                   const oc_params* prm, int8_t* valid, double* geo) {
  int ncoef = (prm->sh_degree + 1) * (prm->sh_degree + 1);
  int64_t nvalid = 0;
#pragma omp parallel for schedule(static) reduction(+ : nvalid)
  for (int64_t i = 0; i < n; ++i) {
    double* rec = geo + i * G_NCOL;
    int ok = project_one(means + 3 * i, scales + 3 * i, quats + 4 * i, opac[i],
                         sh + (int64_t)ncoef * 3 * i, cam, prm, rec);
    valid[i] = (int8_t)ok;
    if (!ok)
      for (int k = 0; k < G_NCOL; ++k) rec[k] = 0.0;
    nvalid += ok;
  }
  return nvalid;
}

/* Depth key: the bits of the float32 rounding of camera-space z (sec. 4.3:
 * positive floats order like their unsigned bit patterns). */
uint32_t oc_depth_key(double tz) {
  float f = (float)tz;
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

/* ------------------------------------------------ macro-tile binning ---- */
static int64_t floor_to_i64(double v, int64_t lo, int64_t hi) {
  /* floor(v) clamped into [lo - 1, hi + 1] without overflow */
  if (v < (double)(lo - 1)) return lo - 1;
  if (v > (double)(hi + 1)) return hi + 1;
  return (int64_t)floor(v);
}

/* The exact intersection of the closed ellipse {q <= tau} with each macro-
 * tile rectangle, visited band by band (one band = one macro-tile row) with
 * the ellipse's x-extent over the band's y-range.  Inputs are the float32
 * stored fields (mx, my, a, b, c, tau) widened to double.  Writes the
 * ascending macro-tile ids into out (when out != NULL, at most cap) and
 * returns how many there are. */
int32_t oc_mt_list(const float f[6], int32_t width, int32_t height, int32_t* out, int32_t cap) {
  double mx = f[0], my = f[1], a = f[2], b = f[3], c = f[4], tau = f[5];
  double W = width, H = height;
  int64_t nmx = (width + OC_MT_W - 1) / OC_MT_W;
  int64_t nmy = (height + OC_MT_H - 1) / OC_MT_H;
  double det = a * c - b * b;
  double ry = sqrt(tau * c);
  double dys = b * sqrt(tau / a);
  int64_t jlo = floor_to_i64((my - ry) / (double)OC_MT_H, 0, nmy - 1);
  int64_t jhi = floor_to_i64((my + ry) / (double)OC_MT_H, 0, nmy - 1);
  if (jlo < 0) jlo = 0;
  if (jhi > nmy - 1) jhi = nmy - 1;
  int32_t cnt = 0;
  for (int64_t j = jlo; j <= jhi; ++j) {
    double ytop = (double)(j * OC_MT_H);
    double ybot = (double)((j + 1) * OC_MT_H);
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
    double xmax = (mx + (b / c) * yp) + sqrt(rp);
    double xmin = (mx + (b / c) * ym) - sqrt(rm);
    if (xmax < 0.0 || xmin > W) continue;
    int64_t ilo = floor_to_i64(xmin / (double)OC_MT_W, 0, nmx - 1);
    int64_t ihi = floor_to_i64(xmax / (double)OC_MT_W, 0, nmx - 1);
    if (ilo < 0) ilo = 0;
    if (ihi > nmx - 1) ihi = nmx - 1;
    for (int64_t i = ilo; i <= ihi; ++i) {
      if (out && cnt < cap) out[cnt] = (int32_t)(j * nmx + i);
      ++cnt;
    }
  }
  return cnt;
}

static void stored_fields(const double* rec, float f[6]) {
  f[0] = (float)rec[G_MX];
  f[1] = (float)rec[G_MY];
  f[2] = (float)rec[G_A];
  f[3] = (float)rec[G_B];
  f[4] = (float)rec[G_C];
  f[5] = (float)rec[G_TAU];
}

/* Count pass: counts[i] = number of macro-tiles gaussian i overlaps (0 when
 * culled).  Returns the total number of pairs. */
int64_t oc_bin_count(int64_t n, const int8_t* valid, const double* geo, int32_t width,
                     int32_t height, int32_t* counts) {
  int64_t total = 0;
#pragma omp parallel for schedule(static) reduction(+ : total)
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = 0;
    if (valid[i]) {
      float f[6];
      stored_fields(geo + i * G_NCOL, f);
      c = oc_mt_list(f, width, height, NULL, 0);
    }
    counts[i] = c;
    total += c;
  }
  return total;
}

/* Fill pass: pairs in gaussian-id order, macro-tiles ascending within a
 * gaussian; offsets[i] = exclusive prefix sum of counts. */
void oc_bin_fill(int64_t n, const int8_t* valid, const double* geo, int32_t width, int32_t height,
                 const int64_t* offsets, int32_t* pair_mt, uint32_t* pair_key, int32_t* pair_gid) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    if (!valid[i]) continue;
    float f[6];
    stored_fields(geo + i * G_NCOL, f);
    int32_t c = oc_mt_list(f, width, height, NULL, 0);
    if (c == 0) continue;
    int32_t local[4096];
    int32_t* ids = c <= 4096 ? local : (int32_t*)malloc(sizeof(int32_t) * (size_t)c);
    oc_mt_list(f, width, height, ids, c);
    uint32_t key = oc_depth_key(geo[i * G_NCOL + G_TZ]);
    for (int32_t k = 0; k < c; ++k) {
      pair_mt[offsets[i] + k] = ids[k];
      pair_key[offsets[i] + k] = key;
      pair_gid[offsets[i] + k] = (int32_t)i;
    }
    if (ids != local) free(ids);
  }
}

/* ------------------------------------------------------------- sort ---- */
typedef struct { int32_t mt; uint32_t key; int32_t gid; } oc_pair;

static int cmp_pair(const void* pa, const void* pb) {
  const oc_pair* a = (const oc_pair*)pa;
  const oc_pair* b = (const oc_pair*)pb;
  if (a->mt != b->mt) return a->mt < b->mt ? -1 : 1;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->gid != b->gid) return a->gid < b->gid ? -1 : 1;
  return 0;
}

/* Sorts the pairs by (macro-tile, depth key, gaussian id), in place. */
void oc_sort_pairs(int64_t np, int32_t* mt, uint32_t* key, int32_t* gid) {
  oc_pair* p = (oc_pair*)malloc(sizeof(oc_pair) * (size_t)(np > 0 ? np : 1));
  for (int64_t i = 0; i < np; ++i) { p[i].mt = mt[i]; p[i].key = key[i]; p[i].gid = gid[i]; }
  qsort(p, (size_t)np, sizeof(oc_pair), cmp_pair);
  for (int64_t i = 0; i < np; ++i) { mt[i] = p[i].mt; key[i] = p[i].key; gid[i] = p[i].gid; }
  free(p);
}

/* --------------------------------------------------------- batches ---- */
/* mt_off[m] = first sorted pair of macro-tile m (n_mt + 1 entries).
 * Batches in (macro-tile, batch index) order: batch_tab[3*k] = mt,
 * [3*k+1] = start, [3*k+2] = length (<= cap).  Returns the batch count;
 * writes at most max_batches rows. */
int64_t oc_batches(int64_t np, const int32_t* sorted_mt, int32_t n_mt, int32_t cap,
                   int64_t* mt_off, int32_t* batch_tab, int64_t max_batches) {
  for (int32_t m = 0; m <= n_mt; ++m) mt_off[m] = 0;
  for (int64_t i = 0; i < np; ++i) mt_off[sorted_mt[i] + 1] += 1;
  for (int32_t m = 0; m < n_mt; ++m) mt_off[m + 1] += mt_off[m];
  int64_t nb = 0;
  for (int32_t m = 0; m < n_mt; ++m) {
    int64_t n = mt_off[m + 1] - mt_off[m];
    for (int64_t s = 0; s < n; s += cap) {
      if (nb < max_batches) {
        batch_tab[3 * nb + 0] = m;
        batch_tab[3 * nb + 1] = (int32_t)(mt_off[m] + s);
        batch_tab[3 * nb + 2] = (int32_t)((n - s) < cap ? (n - s) : cap);
      }
      ++nb;
    }
  }
  return nb;
}

/* --------------------------------------------------------- raster ---- */

/* How far a float32 evaluation of q can land from this double one: the
 * rasteriser works on the float32 roundings of the centre and the Cholesky
 * factors (half an ulp each, at unit roundoff 2^-24), forms u, v and q in
 * float32, and takes alpha through a prescaled exp2 (a few ulps, i.e. a few
 * units of 2^-24 in q).  Used to flag the decisions (alpha >= 1/255, the
 * alpha clamp) that float32 may take the other way. */
double oc_f32_q_bound(const double* rec, double dx, double dy, double u, double v, double q) {
  const double e = 1.0 / 16777216.0;
  double emx = fabs(rec[G_MX]) * e, emy = fabs(rec[G_MY]) * e;
  double du = fabs(rec[G_L0]) * emx + fabs(rec[G_L1]) * emy +
              (fabs(rec[G_L0] * dx) + fabs(rec[G_L1] * dy)) * 3.0 * e;
  double dv = fabs(rec[G_L2]) * emy + fabs(rec[G_L2] * dy) * 2.0 * e;
  return 2.0 * fabs(u) * du + 2.0 * fabs(v) * dv + (q + 4.0) * 4.0 * e;
}

/* Half-width of the band around tau inside which an alpha decision at pixel
 * centre (px, py) is flagged: twice the float32 bound plus 1e-5 (1 + tau).
 * *q_out receives the double q there. */
static double flag_band(const double* rec, double px, double py, double* q_out) {
  double dx = px - rec[G_MX], dy = py - rec[G_MY];
  double u = rec[G_L0] * dx + rec[G_L1] * dy;
  double v = rec[G_L2] * dy;
  double q = u * u + v * v;
  *q_out = q;
  return 2.0 * oc_f32_q_bound(rec, dx, dy, u, v, q) + 1e-5 * (1.0 + rec[G_TAU]);
}

/* The band and q of flag_band for n (gaussian, pixel centre) evaluations;
 * also the float32 bound alone (tests of the bound). */
void oc_alpha_flag_band(int64_t n, const double* geo, const int64_t* gid, const double* px,
                        const double* py, double* q, double* band, double* bound) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    const double* rec = geo + gid[k] * G_NCOL;
    band[k] = flag_band(rec, px[k], py[k], &q[k]);
    double dx = px[k] - rec[G_MX], dy = py[k] - rec[G_MY];
    double u = rec[G_L0] * dx + rec[G_L1] * dy;
    double v = rec[G_L2] * dy;
    bound[k] = oc_f32_q_bound(rec, dx, dy, u, v, q[k]);
  }
}

static double alpha_at(const double* rec, double px, double py, const oc_params* prm,
                       uint8_t* amb) {
  double q;
  double band = flag_band(rec, px, py, &q);
  double tau = rec[G_TAU];
  if (fabs(q - tau) <= band) *amb |= OC_AMB_ALPHA;
  double al = rec[G_OP] * exp(-0.5 * q);
  if (al > prm->alpha_max) al = prm->alpha_max;
  return al;
}

static void flag_t(double T, const oc_params* prm, uint8_t* amb) {
  if (prm->t_eps > 0.0 && fabs(T - prm->t_eps) <= 1e-4 * prm->t_eps) *amb |= OC_AMB_T;
}

/* Composites the gaussians ids[0..cnt) (already in depth order) at pixel
 * centre (px, py) front to back from state (C, T); stops once T < t_eps. */
static void composite(const double* geo, const int32_t* ids, int64_t cnt, double px, double py,
                      const oc_params* prm, double C[3], double* T, uint8_t* amb) {
  for (int64_t k = 0; k < cnt; ++k) {
    if (*T < prm->t_eps) break;
    const double* rec = geo + (int64_t)ids[k] * G_NCOL;
    double al = alpha_at(rec, px, py, prm, amb);
    if (al < prm->alpha_min) continue;
    double wgt = al * (*T);
    C[0] += wgt * rec[G_R];
    C[1] += wgt * rec[G_G];
    C[2] += wgt * rec[G_BL];
    *T = *T * (1.0 - al);
    flag_t(*T, prm, amb);
  }
}

typedef struct { uint32_t key; int32_t gid; } oc_kg;
static int cmp_kg(const void* pa, const void* pb) {
  const oc_kg* a = (const oc_kg*)pa;
  const oc_kg* b = (const oc_kg*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return a->gid < b->gid ? -1 : (a->gid > b->gid);
}

/* The plain per-pixel definition: every gaussian that survived the culls,
 * ordered by (depth key, id), composited sequentially at each pixel centre.
 * pixels: NULL for the whole image, else npix (x, y) pairs; outputs are per
 * listed pixel (image: 3 doubles each, T, amb). */
void oc_render_untiled(int64_t n, const int8_t* valid, const double* geo, const oc_camera* cam,
                       const oc_params* prm, const int32_t* pixels, int64_t npix, double* image,
                       double* Tout, uint8_t* amb) {
  int64_t nv = 0;
  for (int64_t i = 0; i < n; ++i) nv += valid[i] ? 1 : 0;
  oc_kg* order = (oc_kg*)malloc(sizeof(oc_kg) * (size_t)(nv > 0 ? nv : 1));
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i)
    if (valid[i]) { order[k].key = oc_depth_key(geo[i * G_NCOL + G_TZ]); order[k].gid = (int32_t)i; ++k; }
  qsort(order, (size_t)nv, sizeof(oc_kg), cmp_kg);
  int32_t* ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
  for (int64_t i = 0; i < nv; ++i) ids[i] = order[i].gid;
  free(order);
  int64_t total = pixels ? npix : (int64_t)cam->width * cam->height;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t p = 0; p < total; ++p) {
    int32_t x, y;
    if (pixels) { x = pixels[2 * p]; y = pixels[2 * p + 1]; }
    else { x = (int32_t)(p % cam->width); y = (int32_t)(p / cam->width); }
    double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
    uint8_t a = 0;
    composite(geo, ids, nv, x + 0.5, y + 0.5, prm, C, &T, &a);
    for (int ch = 0; ch < 3; ++ch) image[3 * p + ch] = C[ch] + T * (double)cam->background[ch];
    Tout[p] = T;
    amb[p] = a;
  }
  free(ids);
}

/* Partial (C, T) of one batch at one pixel centre, from (0, 1). */
static void batch_partial(const double* geo, const int32_t* sorted_gid, const int32_t* bt,
                          double px, double py, const oc_params* prm, double C[3], double* T,
                          uint8_t* amb) {
  C[0] = C[1] = C[2] = 0.0;
  *T = 1.0;
  composite(geo, sorted_gid + bt[1], bt[2], px, py, prm, C, T, amb);
}

/* Batched form: every (macro-tile, batch) unit composites its gaussians from
 * (0, 1); the partials of a pixel's macro-tile are merged in batch order with
 * Eq. 1, C = C0 + T0 C1 + T0 T1 C2 + ..., stopping once the product of T's
 * drops below t_eps; the output is C + T * background. */
void oc_render_tiled(const double* geo, const int32_t* sorted_gid, const int64_t* mt_off,
                     const int32_t* batch_tab, int64_t nbatches, const oc_camera* cam,
                     const oc_params* prm, const int32_t* pixels, int64_t npix, double* image,
                     double* Tout, uint8_t* amb) {
  int32_t nmx = (cam->width + OC_MT_W - 1) / OC_MT_W;
  int32_t nmy = (cam->height + OC_MT_H - 1) / OC_MT_H;
  int32_t nmt = nmx * nmy;
  /* first batch of every macro-tile (batches are in macro-tile order) */
  int64_t* first = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nmt + 1));
  for (int32_t m = 0; m <= nmt; ++m) first[m] = nbatches;
  for (int64_t bi = nbatches - 1; bi >= 0; --bi) first[batch_tab[3 * bi]] = bi;
  for (int32_t m = nmt - 1; m >= 0; --m)
    if (first[m] > first[m + 1]) first[m] = first[m + 1];
  (void)mt_off;
  int64_t total = pixels ? npix : (int64_t)cam->width * cam->height;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t p = 0; p < total; ++p) {
    int32_t x, y;
    if (pixels) { x = pixels[2 * p]; y = pixels[2 * p + 1]; }
    else { x = (int32_t)(p % cam->width); y = (int32_t)(p / cam->width); }
    int32_t m = (y / OC_MT_H) * nmx + (x / OC_MT_W);
    double Cacc[3] = {0.0, 0.0, 0.0}, Tacc = 1.0;
    uint8_t a = 0;
    for (int64_t bi = first[m]; bi < first[m + 1]; ++bi) {
      if (Tacc < prm->t_eps) break;
      double Cb[3], Tb;
      batch_partial(geo, sorted_gid, batch_tab + 3 * bi, x + 0.5, y + 0.5, prm, Cb, &Tb, &a);
      for (int ch = 0; ch < 3; ++ch) Cacc[ch] += Tacc * Cb[ch];
      Tacc = Tacc * Tb;
      flag_t(Tacc, prm, &a);
    }
    for (int ch = 0; ch < 3; ++ch) image[3 * p + ch] = Cacc[ch] + Tacc * (double)cam->background[ch];
    Tout[p] = Tacc;
    amb[p] = a;
  }
  free(first);
}

/* Pixel-gaussian evaluations the batched form needs (the rasteriser's work
 * count).  Per (macro-tile, batch) unit and render tile, in the unit's depth
 * order, a gaussian is evaluated at the tile's 64 pixels when its level
 * ellipse {q <= tau} contains at least one of the tile's pixel centres (the
 * per-tile visibility of Alg. 1, taken exactly), until every in-image pixel
 * of the tile has local T < t_eps (the unanimous early-out of Alg. 2).
 *   out[0] = 64 x those evaluations over every unit and tile;
 *   out[1] = the same over the (unit, tile) pairs whose partial the merge of
 *            Eq. 1 reads: some in-image pixel of the tile still has merged
 *            T >= t_eps before the batch (the product of the earlier batches'
 *            partial T, taken while it is >= t_eps).
 * The second is the work a rasteriser that skips tiles the earlier batches
 * have saturated must do at least. */
void oc_count_evals(const double* geo, const int32_t* sorted_gid, const int32_t* batch_tab,
                    int64_t nbatches, const oc_camera* cam, const oc_params* prm, int64_t out[2]) {
  int32_t nmx = (cam->width + OC_MT_W - 1) / OC_MT_W;
  int32_t nmy = (cam->height + OC_MT_H - 1) / OC_MT_H;
  int32_t nmt = nmx * nmy;
  int64_t* first = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nmt + 1));
  for (int32_t m = 0; m <= nmt; ++m) first[m] = nbatches;
  for (int64_t bi = nbatches - 1; bi >= 0; --bi) first[batch_tab[3 * bi]] = bi;
  for (int32_t m = nmt - 1; m >= 0; --m)
    if (first[m] > first[m + 1]) first[m] = first[m + 1];
  int64_t all = 0, read = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : all, read)
  for (int32_t m = 0; m < nmt; ++m) {
    int32_t x0 = (m % nmx) * OC_MT_W, y0 = (m / nmx) * OC_MT_H;
    double Tm[OC_MT_TX * OC_MT_TY][64];
    for (int t = 0; t < OC_MT_TX * OC_MT_TY; ++t)
      for (int p = 0; p < 64; ++p) Tm[t][p] = 1.0;
    for (int64_t bi = first[m]; bi < first[m + 1]; ++bi) {
      const int32_t* bt = batch_tab + 3 * bi;
      for (int t = 0; t < OC_MT_TX * OC_MT_TY; ++t) {
        int32_t tx0 = x0 + (t % OC_MT_TX) * OC_TILE, ty0 = y0 + (t / OC_MT_TX) * OC_TILE;
        if (tx0 >= cam->width || ty0 >= cam->height) continue;
        int inside[64];
        int merge_reads = 0;
        for (int p = 0; p < 64; ++p) {
          inside[p] = (tx0 + p % OC_TILE) < cam->width && (ty0 + p / OC_TILE) < cam->height;
          if (inside[p] && Tm[t][p] >= prm->t_eps) merge_reads = 1;
        }
        double T[64];
        for (int p = 0; p < 64; ++p) T[p] = 1.0;
        int64_t cnt = 0;
        for (int32_t k = 0; k < bt[2]; ++k) {
          int live = 0;
          for (int p = 0; p < 64; ++p) live |= inside[p] && T[p] >= prm->t_eps;
          if (!live) break;
          const double* rec = geo + (int64_t)sorted_gid[bt[1] + k] * G_NCOL;
          double tau = rec[G_TAU];
          /* the ellipse's bounding box against the tile's pixel centres first */
          double ex = sqrt(tau * rec[G_A]), ey = sqrt(tau * rec[G_C]);
          if (rec[G_MX] + ex < tx0 + 0.5 || rec[G_MX] - ex > tx0 + 7.5 || rec[G_MY] + ey < ty0 + 0.5 ||
              rec[G_MY] - ey > ty0 + 7.5)
            continue;
          int hit = 0;
          for (int p = 0; p < 64; ++p) {
            double dx = tx0 + p % OC_TILE + 0.5 - rec[G_MX], dy = ty0 + p / OC_TILE + 0.5 - rec[G_MY];
            double u = rec[G_L0] * dx + rec[G_L1] * dy, v = rec[G_L2] * dy;
            double q = u * u + v * v;
            if (q > tau) continue;
            hit = 1;
            if (T[p] < prm->t_eps) continue;
            double al = rec[G_OP] * exp(-0.5 * q);
            if (al > prm->alpha_max) al = prm->alpha_max;
            if (al < prm->alpha_min) continue;
            T[p] = T[p] * (1.0 - al);
          }
          cnt += hit;
        }
        all += 64 * cnt;
        if (merge_reads) read += 64 * cnt;
        for (int p = 0; p < 64; ++p)
          if (Tm[t][p] >= prm->t_eps) Tm[t][p] = Tm[t][p] * T[p];
      }
    }
  }
  free(first);
  out[0] = all;
  out[1] = read;
}

/* Per-pixel partial (C, T) of one batch over the 32 render tiles x 64 pixels
 * of its macro-tile (pixel (tx*8 + px, ty*8 + py) of the macro-tile at index
 * ((ty*8 + tx)*64 + py*8 + px)), for stage-by-stage comparisons.  Pixels
 * outside the image get (0, 0, 0, 1). */
void oc_batch_partials(const double* geo, const int32_t* sorted_gid, const int32_t* bt,
                       const oc_camera* cam, const oc_params* prm, double* out /* 2048 x 4 */,
                       uint8_t* amb /* 2048 flags, or NULL */) {
  int32_t nmx = (cam->width + OC_MT_W - 1) / OC_MT_W;
  int32_t m = bt[0];
  int32_t x0 = (m % nmx) * OC_MT_W, y0 = (m / nmx) * OC_MT_H;
  for (int32_t t = 0; t < OC_MT_TX * OC_MT_TY; ++t) {
    int32_t tx = t % OC_MT_TX, ty = t / OC_MT_TX;
    for (int32_t q = 0; q < OC_TILE * OC_TILE; ++q) {
      int32_t x = x0 + tx * OC_TILE + q % OC_TILE;
      int32_t y = y0 + ty * OC_TILE + q / OC_TILE;
      double* o = out + 4 * ((int64_t)t * 64 + q);
      if (amb) amb[(int64_t)t * 64 + q] = 0;
      if (x >= cam->width || y >= cam->height) { o[0] = o[1] = o[2] = 0.0; o[3] = 1.0; continue; }
      double C[3], T;
      uint8_t a = 0;
      batch_partial(geo, sorted_gid, bt, x + 0.5, y + 0.5, prm, C, &T, &a);
      o[0] = C[0]; o[1] = C[1]; o[2] = C[2]; o[3] = T;
      if (amb) amb[(int64_t)t * 64 + q] = a;
    }
  }
}

/* Threads of the oracle's parallel loops (timing its single-core rate). */
void oc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
