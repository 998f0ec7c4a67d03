/*
 * Plain FP64 CPU adjoint of the HiGS forward frame path: gradients of a
 * scalar loss L(image, T) with respect to the gaussian parameters (means,
 * scales, quaternions, opacities, SH coefficients).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the GPU library.
 *
 * The paper renders forward only; its limitations paragraph (Forward-only)
 * sketches the backward: the post-blend merge becomes a scan whose prefix is
 * the transmittance before each batch, and the point where transmittance
 * saturates is kept per (pixel, batch).  This file writes that adjoint out
 * directly:
 *   - The discrete structure (culls, pair lists, depth order, batches, which
 *     gaussians composite at a pixel, the alpha clamp) is held fixed, as it is
 *     piecewise constant in the parameters.
 *   - At a pixel, the batched composite of Eq. 1 equals the sequential
 *     composite over the gaussians that took part, in order:
 *       I = sum_k alpha_k T_k c_k + T_end bg,  T_k = prod_{j<k} (1 - alpha_j).
 *     With g = dL/dI and gT = dL/dT_end, walking back to front with
 *       X = g.bg + gT,   X <- alpha_k (g.c_k) + (1 - alpha_k) X
 *     gives dL/dalpha_k = T_k (g.c_k - X_k) (X_k: the value after gaussian k)
 *     and dL/dc_k = alpha_k T_k g, without dividing by (1 - alpha).
 *   - alpha = min(alpha_max, o exp(-q/2)), q = (l0 dx + l1 dy)^2 + (l2 dy)^2
 *     (sec. 3.5); the clamp has zero derivative.
 *   - The projection (the same EWA chain as the forward oracle) is
 *     differentiated by hand in reverse order.
 * Pinned by central finite differences of the forward oracle (tests).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "higs_oracle.h"

/* Columns of the per-gaussian gradient with respect to the raster record. */
enum { D_MX = 0, D_MY, D_L0, D_L1, D_L2, D_OP, D_R, D_G, D_BL, D_NCOL };

/* ---------------------------------------------------------------- SH ---- */
/* d Y_k / d(x, y, z) of the basis in oc_sh_basis, the components of the
 * direction taken as independent variables; out[3 k + axis]. */
void oc_sh_basis_grad(const double d[3], int degree, double out[48]) {
  const double pi = 3.14159265358979323846;
  double x = d[0], y = d[1], z = d[2];
  for (int k = 0; k < 48; ++k) out[k] = 0.0;
  if (degree < 1) return;
  double k1 = sqrt(3.0 / (4.0 * pi));
  out[3 * 1 + 1] = -k1;
  out[3 * 2 + 2] = k1;
  out[3 * 3 + 0] = -k1;
  if (degree < 2) return;
  double k2a = 0.5 * sqrt(15.0 / pi);
  double k2b = 0.25 * sqrt(5.0 / pi);
  double k2c = 0.25 * sqrt(15.0 / pi);
  /* 4: k2a x y */
  out[3 * 4 + 0] = k2a * y;
  out[3 * 4 + 1] = k2a * x;
  /* 5: -k2a y z */
  out[3 * 5 + 1] = -k2a * z;
  out[3 * 5 + 2] = -k2a * y;
  /* 6: k2b (2 z^2 - x^2 - y^2) */
  out[3 * 6 + 0] = -2.0 * k2b * x;
  out[3 * 6 + 1] = -2.0 * k2b * y;
  out[3 * 6 + 2] = 4.0 * k2b * z;
  /* 7: -k2a x z */
  out[3 * 7 + 0] = -k2a * z;
  out[3 * 7 + 2] = -k2a * x;
  /* 8: k2c (x^2 - y^2) */
  out[3 * 8 + 0] = 2.0 * k2c * x;
  out[3 * 8 + 1] = -2.0 * k2c * y;
  if (degree < 3) return;
  double k3a = 0.25 * sqrt(35.0 / (2.0 * pi));
  double k3b = 0.5 * sqrt(105.0 / pi);
  double k3c = 0.25 * sqrt(21.0 / (2.0 * pi));
  double k3d = 0.25 * sqrt(7.0 / pi);
  double k3e = 0.25 * sqrt(105.0 / pi);
  double xx = x * x, yy = y * y, zz = z * z;
  /* 9: -k3a (3 x^2 y - y^3) */
  out[3 * 9 + 0] = -6.0 * k3a * x * y;
  out[3 * 9 + 1] = -3.0 * k3a * (xx - yy);
  /* 10: k3b x y z */
  out[3 * 10 + 0] = k3b * y * z;
  out[3 * 10 + 1] = k3b * x * z;
  out[3 * 10 + 2] = k3b * x * y;
  /* 11: -k3c y (4 z^2 - x^2 - y^2) */
  out[3 * 11 + 0] = 2.0 * k3c * x * y;
  out[3 * 11 + 1] = -k3c * (4.0 * zz - xx - 3.0 * yy);
  out[3 * 11 + 2] = -8.0 * k3c * y * z;
  /* 12: k3d z (2 z^2 - 3 x^2 - 3 y^2) */
  out[3 * 12 + 0] = -6.0 * k3d * x * z;
  out[3 * 12 + 1] = -6.0 * k3d * y * z;
  out[3 * 12 + 2] = k3d * (6.0 * zz - 3.0 * xx - 3.0 * yy);
  /* 13: -k3c x (4 z^2 - x^2 - y^2) */
  out[3 * 13 + 0] = -k3c * (4.0 * zz - 3.0 * xx - yy);
  out[3 * 13 + 1] = 2.0 * k3c * x * y;
  out[3 * 13 + 2] = -8.0 * k3c * x * z;
  /* 14: k3e z (x^2 - y^2) */
  out[3 * 14 + 0] = 2.0 * k3e * x * z;
  out[3 * 14 + 1] = -2.0 * k3e * y * z;
  out[3 * 14 + 2] = k3e * (xx - yy);
  /* 15: -k3a (x^3 - 3 x y^2) */
  out[3 * 15 + 0] = -3.0 * k3a * (xx - yy);
  out[3 * 15 + 1] = 6.0 * k3a * x * y;
}

/* ------------------------------------------------------- projection ---- */
/* Reverse pass of one gaussian's projection.  g[D_NCOL] is dL/d(record);
 * writes dL/d(mean, scale, quat, opacity, sh).  Replays the forward chain
 * (camera transform, rotation, covariance, EWA Jacobian with its clamp,
 * dilation, Cholesky factors, pixel mean, SH colour) and walks it back. */
static void project_grad_one(const float* mean, const float* scale, const float* quat,
                             const float* sh, const oc_camera* cam, const oc_params* prm,
                             const double* g, double* dmean, double* dscale, double* dquat,
                             double* dopac, double* dsh) {
  double R[9], t[3];
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) R[r * 3 + k] = (double)cam->world_to_cam[r * 4 + k];
    t[r] = (double)cam->world_to_cam[r * 4 + 3];
  }
  double m[3] = {mean[0], mean[1], mean[2]};
  double s[3] = {scale[0], scale[1], scale[2]};
  double qv[4] = {quat[0], quat[1], quat[2], quat[3]};

  /* forward replay */
  double tc[3];
  for (int r = 0; r < 3; ++r) tc[r] = R[r * 3 + 0] * m[0] + R[r * 3 + 1] * m[1] + R[r * 3 + 2] * m[2] + t[r];
  double tx = tc[0], ty = tc[1], tz = tc[2];
  double qn = sqrt(qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3]);
  double w = qv[0] / qn, x = qv[1] / qn, y = qv[2] / qn, z = qv[3] / qn;
  double G[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z),       2.0 * (x * z + w * y),
                 2.0 * (x * y + w * z),       1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                 2.0 * (x * z - w * y),       2.0 * (y * z + w * x),       1.0 - 2.0 * (x * x + y * y)};
  double M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i * 3 + j] = G[i * 3 + j] * s[j];
  double S[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      S[i * 3 + j] = M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1] + M[i * 3 + 2] * M[j * 3 + 2];
  double fx = cam->fx, fy = cam->fy;
  double Wd = cam->width, Hd = cam->height, cx = cam->cx, cy = cam->cy;
  double tanx = Wd / (2.0 * fx), tany = Hd / (2.0 * fy);
  double xlo = -(cx / fx + 0.3 * tanx), xhi = (Wd - cx) / fx + 0.3 * tanx;
  double ylo = -(cy / fy + 0.3 * tany), yhi = (Hd - cy) / fy + 0.3 * tany;
  double xr = tx / tz, yr = ty / tz;
  int xclamp = 0, yclamp = 0;
  if (xr < xlo) { xr = xlo; xclamp = 1; }
  if (xr > xhi) { xr = xhi; xclamp = 1; }
  if (yr < ylo) { yr = ylo; yclamp = 1; }
  if (yr > yhi) { yr = yhi; yclamp = 1; }
  double xc = xr * tz, yc = yr * tz;
  double j00 = fx / tz, j02 = -(fx * xc) / (tz * tz);
  double j11 = fy / tz, j12 = -(fy * yc) / (tz * tz);
  double T0[3], T1[3];
  for (int k = 0; k < 3; ++k) {
    T0[k] = j00 * R[0 * 3 + k] + j02 * R[2 * 3 + k];
    T1[k] = j11 * R[1 * 3 + k] + j12 * R[2 * 3 + k];
  }
  double ST0[3], ST1[3]; /* S T0^T, S T1^T */
  for (int i = 0; i < 3; ++i) {
    ST0[i] = S[i * 3 + 0] * T0[0] + S[i * 3 + 1] * T0[1] + S[i * 3 + 2] * T0[2];
    ST1[i] = S[i * 3 + 0] * T1[0] + S[i * 3 + 1] * T1[1] + S[i * 3 + 2] * T1[2];
  }
  double a = T0[0] * ST0[0] + T0[1] * ST0[1] + T0[2] * ST0[2] + prm->dilation;
  double b = T0[0] * ST1[0] + T0[1] * ST1[1] + T0[2] * ST1[2];
  double c = T1[0] * ST1[0] + T1[1] * ST1[1] + T1[2] * ST1[2] + prm->dilation;
  double det = a * c - b * b;

  /* Cholesky factors: l0 = sqrt(c/det), l1 = -b/sqrt(c det), l2 = 1/sqrt(c) */
  double gl0 = g[D_L0], gl1 = g[D_L1], gl2 = g[D_L2];
  double r_cd = sqrt(c / det), r_cdet = sqrt(c * det), r_c = sqrt(c);
  double dl0_dc = 0.5 / r_cd / det, dl0_ddet = -0.5 / r_cd * c / (det * det);
  double dl1_db = -1.0 / r_cdet;
  double cdet3 = r_cdet * r_cdet * r_cdet;
  double dl1_dc = 0.5 * b * det / cdet3, dl1_ddet = 0.5 * b * c / cdet3;
  double dl2_dc = -0.5 / (r_c * r_c * r_c);
  double gdet = gl0 * dl0_ddet + gl1 * dl1_ddet;
  double ga = gdet * c;
  double gb = gl1 * dl1_db - 2.0 * b * gdet;
  double gc = gl0 * dl0_dc + gl1 * dl1_dc + gl2 * dl2_dc + gdet * a;

  /* 2D covariance: a = T0 S T0^T, b = T0 S T1^T, c = T1 S T1^T */
  double gT0[3], gT1[3], gS[9];
  for (int k = 0; k < 3; ++k) {
    gT0[k] = 2.0 * ga * ST0[k] + gb * ST1[k];
    gT1[k] = gb * ST0[k] + 2.0 * gc * ST1[k];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      gS[i * 3 + j] = ga * T0[i] * T0[j] + gb * T0[i] * T1[j] + gc * T1[i] * T1[j];
  /* S = M M^T: dL/dM = (gS + gS^T) M */
  double gM[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += (gS[i * 3 + k] + gS[k * 3 + i]) * M[k * 3 + j];
      gM[i * 3 + j] = acc;
    }
  /* M = G diag(s) */
  double gG[9];
  for (int j = 0; j < 3; ++j) {
    double acc = 0.0;
    for (int i = 0; i < 3; ++i) {
      gG[i * 3 + j] = gM[i * 3 + j] * s[j];
      acc += gM[i * 3 + j] * G[i * 3 + j];
    }
    dscale[j] = acc;
  }
  /* rotation matrix of the unit quaternion (w, x, y, z) */
  double gw = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  gy += -4.0 * y * gG[0]; gz += -4.0 * z * gG[0];
  gx += 2.0 * y * gG[1]; gy += 2.0 * x * gG[1]; gw += -2.0 * z * gG[1]; gz += -2.0 * w * gG[1];
  gx += 2.0 * z * gG[2]; gz += 2.0 * x * gG[2]; gw += 2.0 * y * gG[2]; gy += 2.0 * w * gG[2];
  gx += 2.0 * y * gG[3]; gy += 2.0 * x * gG[3]; gw += 2.0 * z * gG[3]; gz += 2.0 * w * gG[3];
  gx += -4.0 * x * gG[4]; gz += -4.0 * z * gG[4];
  gy += 2.0 * z * gG[5]; gz += 2.0 * y * gG[5]; gw += -2.0 * x * gG[5]; gx += -2.0 * w * gG[5];
  gx += 2.0 * z * gG[6]; gz += 2.0 * x * gG[6]; gw += -2.0 * y * gG[6]; gy += -2.0 * w * gG[6];
  gy += 2.0 * z * gG[7]; gz += 2.0 * y * gG[7]; gw += 2.0 * x * gG[7]; gx += 2.0 * w * gG[7];
  gx += -4.0 * x * gG[8]; gy += -4.0 * y * gG[8];
  /* normalisation u = q / |q|: dL/dq = (gu - u (u . gu)) / |q| */
  double u4[4] = {w, x, y, z}, gu4[4] = {gw, gx, gy, gz};
  double ug = u4[0] * gu4[0] + u4[1] * gu4[1] + u4[2] * gu4[2] + u4[3] * gu4[3];
  for (int k = 0; k < 4; ++k) dquat[k] = (gu4[k] - u4[k] * ug) / qn;

  /* EWA Jacobian rows T0 = j00 R0 + j02 R2, T1 = j11 R1 + j12 R2 */
  double gj00 = 0.0, gj02 = 0.0, gj11 = 0.0, gj12 = 0.0;
  for (int k = 0; k < 3; ++k) {
    gj00 += gT0[k] * R[0 * 3 + k];
    gj02 += gT0[k] * R[2 * 3 + k];
    gj11 += gT1[k] * R[1 * 3 + k];
    gj12 += gT1[k] * R[2 * 3 + k];
  }
  double gtx = 0.0, gty = 0.0, gtz = 0.0;
  gtz += -gj00 * fx / (tz * tz);
  gtz += -gj11 * fy / (tz * tz);
  /* j02 = -fx xc / tz^2, xc = xr tz, xr = tx / tz (unless clamped) */
  double gxc = -gj02 * fx / (tz * tz), gyc = -gj12 * fy / (tz * tz);
  gtz += gj02 * 2.0 * fx * xc / (tz * tz * tz) + gj12 * 2.0 * fy * yc / (tz * tz * tz);
  double gxr = gxc * tz, gyr = gyc * tz;
  gtz += gxc * xr + gyc * yr;
  if (!xclamp) { gtx += gxr / tz; gtz += -gxr * tx / (tz * tz); }
  if (!yclamp) { gty += gyr / tz; gtz += -gyr * ty / (tz * tz); }
  /* pixel mean */
  gtx += g[D_MX] * fx / tz;
  gtz += -g[D_MX] * fx * tx / (tz * tz);
  gty += g[D_MY] * fy / tz;
  gtz += -g[D_MY] * fy * ty / (tz * tz);
  /* camera transform: dL/dmean = R^T dL/dtc */
  double gtc[3] = {gtx, gty, gtz};
  for (int k = 0; k < 3; ++k)
    dmean[k] = R[0 * 3 + k] * gtc[0] + R[1 * 3 + k] * gtc[1] + R[2 * 3 + k] * gtc[2];

  *dopac = g[D_OP];

  /* SH colour rgb = max(0, 0.5 + sum_k Y_k(d) sh_k), d = (mean - campos)/|.| */
  int ncoef = (prm->sh_degree + 1) * (prm->sh_degree + 1);
  double campos[3];
  for (int k = 0; k < 3; ++k)
    campos[k] = -(R[0 * 3 + k] * t[0] + R[1 * 3 + k] * t[1] + R[2 * 3 + k] * t[2]);
  double e[3] = {m[0] - campos[0], m[1] - campos[1], m[2] - campos[2]};
  double en = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  double d[3] = {e[0], e[1], e[2]};
  if (en > 0.0) { d[0] /= en; d[1] /= en; d[2] /= en; }
  double Y[16], dY[48];
  oc_sh_basis(d, prm->sh_degree, Y);
  oc_sh_basis_grad(d, prm->sh_degree, dY);
  double gY[16] = {0};
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.0;
    for (int k = 0; k < ncoef; ++k) acc += Y[k] * (double)sh[k * 3 + ch];
    double grgb = (0.5 + acc > 0.0) ? g[D_R + ch] : 0.0;
    for (int k = 0; k < ncoef; ++k) {
      dsh[k * 3 + ch] = grgb * Y[k];
      gY[k] += grgb * (double)sh[k * 3 + ch];
    }
  }
  double gd[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < ncoef; ++k)
    for (int ax = 0; ax < 3; ++ax) gd[ax] += gY[k] * dY[3 * k + ax];
  if (en > 0.0) {
    double dg = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
    for (int k = 0; k < 3; ++k) dmean[k] += (gd[k] - d[k] * dg) / en;
  }
}

/* dgeo [n x D_NCOL] -> gradients of the inputs; culled gaussians (valid 0)
 * get zeros. */
void oc_project_grad(int64_t n, const float* means, const float* scales, const float* quats,
                     const float* sh, const oc_camera* cam, const oc_params* prm,
                     const int8_t* valid, const double* dgeo, double* dmeans, double* dscales,
                     double* dquats, double* dopac, double* dsh) {
  int ncoef = (prm->sh_degree + 1) * (prm->sh_degree + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double* dm = dmeans + 3 * i;
    double* ds = dscales + 3 * i;
    double* dq = dquats + 4 * i;
    double* dc = dsh + (int64_t)ncoef * 3 * i;
    if (!valid[i]) {
      for (int k = 0; k < 3; ++k) dm[k] = ds[k] = 0.0;
      for (int k = 0; k < 4; ++k) dq[k] = 0.0;
      for (int k = 0; k < ncoef * 3; ++k) dc[k] = 0.0;
      dopac[i] = 0.0;
      continue;
    }
    project_grad_one(means + 3 * i, scales + 3 * i, quats + 4 * i, sh + (int64_t)ncoef * 3 * i,
                     cam, prm, dgeo + i * D_NCOL, dm, ds, dq, dopac + i, dc);
  }
}

/* ----------------------------------------------------------- raster ---- */
typedef struct {
  int32_t gid;
  int32_t clamped;
  double alpha, T, e, dx, dy, u, v;
} oc_contrib;

typedef struct {
  oc_contrib* v;
  int64_t n, cap;
} oc_list;

static void list_push(oc_list* l, const oc_contrib* c) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 256;
    l->v = (oc_contrib*)realloc(l->v, sizeof(oc_contrib) * (size_t)l->cap);
  }
  l->v[l->n++] = *c;
}

/* First batch of every macro-tile (n_mt + 1 entries; batches are listed in
 * macro-tile order). */
static int64_t* first_batches(const int32_t* batch_tab, int64_t nbatches, int32_t nmt) {
  int64_t* first = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nmt + 1));
  for (int32_t m = 0; m <= nmt; ++m) first[m] = nbatches;
  for (int64_t bi = nbatches - 1; bi >= 0; --bi) first[batch_tab[3 * bi]] = bi;
  for (int32_t m = nmt - 1; m >= 0; --m)
    if (first[m] > first[m + 1]) first[m] = first[m + 1];
  return first;
}

/* The gaussians that take part at pixel centre (px, py) under the batched
 * form (per batch from T = 1 with its own early stop; batches merged in order
 * while the accumulated T >= t_eps), in compositing order, with the global
 * transmittance before each.  Returns the final transmittance. */
static double pixel_contributions(const double* geo, const int32_t* sorted_gid,
                                  const int32_t* batch_tab, int64_t b0, int64_t b1, double px,
                                  double py, const oc_params* prm, oc_list* out) {
  out->n = 0;
  double Tacc = 1.0;
  for (int64_t bi = b0; bi < b1; ++bi) {
    if (Tacc < prm->t_eps) break;
    const int32_t* bt = batch_tab + 3 * bi;
    double Tloc = 1.0;
    for (int32_t k = 0; k < bt[2]; ++k) {
      if (Tloc < prm->t_eps) break;
      int32_t gid = sorted_gid[bt[1] + k];
      const double* rec = geo + (int64_t)gid * G_NCOL;
      oc_contrib c;
      c.gid = gid;
      c.dx = px - rec[G_MX];
      c.dy = py - rec[G_MY];
      c.u = rec[G_L0] * c.dx + rec[G_L1] * c.dy;
      c.v = rec[G_L2] * c.dy;
      double q = c.u * c.u + c.v * c.v;
      c.e = exp(-0.5 * q);
      double al = rec[G_OP] * c.e;
      c.clamped = al > prm->alpha_max;
      if (c.clamped) al = prm->alpha_max;
      if (al < prm->alpha_min) continue;
      c.alpha = al;
      c.T = Tacc * Tloc;
      list_push(out, &c);
      Tloc = Tloc * (1.0 - al);
    }
    Tacc = Tacc * Tloc;
  }
  return Tacc;
}

/* dL/d(record) of every gaussian [n x D_NCOL] (accumulated: the caller
 * zeroes dgeo) from dL/dimage [H x W x 3] and dL/dT [H x W] (NULL: zero). */
void oc_render_tiled_grad(const double* geo, const int32_t* sorted_gid, const int32_t* batch_tab,
                          int64_t nbatches, const oc_camera* cam, const oc_params* prm,
                          const double* dimg, const double* dT, double* dgeo) {
  int32_t nmx = (cam->width + OC_MT_W - 1) / OC_MT_W;
  int32_t nmy = (cam->height + OC_MT_H - 1) / OC_MT_H;
  int64_t* first = first_batches(batch_tab, nbatches, nmx * nmy);
  int64_t total = (int64_t)cam->width * cam->height;
#pragma omp parallel
  {
    oc_list l = {NULL, 0, 0};
#pragma omp for schedule(dynamic, 64)
    for (int64_t p = 0; p < total; ++p) {
      int32_t x = (int32_t)(p % cam->width), y = (int32_t)(p / cam->width);
      int32_t m = (y / OC_MT_H) * nmx + (x / OC_MT_W);
      pixel_contributions(geo, sorted_gid, batch_tab, first[m], first[m + 1], x + 0.5, y + 0.5,
                          prm, &l);
      const double* g = dimg + 3 * p;
      double X = g[0] * cam->background[0] + g[1] * cam->background[1] +
                 g[2] * cam->background[2] + (dT ? dT[p] : 0.0);
      for (int64_t k = l.n - 1; k >= 0; --k) {
        const oc_contrib* c = &l.v[k];
        const double* rec = geo + (int64_t)c->gid * G_NCOL;
        double* d = dgeo + (int64_t)c->gid * D_NCOL;
        double gc = g[0] * rec[G_R] + g[1] * rec[G_G] + g[2] * rec[G_BL];
        double wgt = c->alpha * c->T;
        double dal = c->T * (gc - X);
        X = c->alpha * gc + (1.0 - c->alpha) * X;
#pragma omp atomic
        d[D_R] += wgt * g[0];
#pragma omp atomic
        d[D_G] += wgt * g[1];
#pragma omp atomic
        d[D_BL] += wgt * g[2];
        if (c->clamped) continue;
        /* alpha = o e, e = exp(-q/2), q = u^2 + v^2 */
        double dq = -0.5 * c->alpha * dal;
        double du = 2.0 * c->u * dq, dv = 2.0 * c->v * dq;
        double ddx = du * rec[G_L0], ddy = du * rec[G_L1] + dv * rec[G_L2];
#pragma omp atomic
        d[D_OP] += dal * c->e;
#pragma omp atomic
        d[D_L0] += du * c->dx;
#pragma omp atomic
        d[D_L1] += du * c->dy;
#pragma omp atomic
        d[D_L2] += dv * c->dy;
#pragma omp atomic
        d[D_MX] -= ddx;
#pragma omp atomic
        d[D_MY] -= ddy;
      }
    }
    free(l.v);
  }
  free(first);
}

/* A 64-bit digest of every discrete decision of the batched render (which
 * gaussians composite at which pixel, in which order, and whether their alpha
 * is clamped), summed over pixels.  Equal digests at two parameter values
 * mean the render is one smooth function between them. */
uint64_t oc_render_tiled_signature(const double* geo, const int32_t* sorted_gid,
                                   const int32_t* batch_tab, int64_t nbatches,
                                   const oc_camera* cam, const oc_params* prm) {
  int32_t nmx = (cam->width + OC_MT_W - 1) / OC_MT_W;
  int32_t nmy = (cam->height + OC_MT_H - 1) / OC_MT_H;
  int64_t* first = first_batches(batch_tab, nbatches, nmx * nmy);
  int64_t total = (int64_t)cam->width * cam->height;
  uint64_t sig = 0;
#pragma omp parallel
  {
    oc_list l = {NULL, 0, 0};
#pragma omp for schedule(dynamic, 64) reduction(+ : sig)
    for (int64_t p = 0; p < total; ++p) {
      int32_t x = (int32_t)(p % cam->width), y = (int32_t)(p / cam->width);
      int32_t m = (y / OC_MT_H) * nmx + (x / OC_MT_W);
      pixel_contributions(geo, sorted_gid, batch_tab, first[m], first[m + 1], x + 0.5, y + 0.5,
                          prm, &l);
      uint64_t h = 1469598103934665603ull ^ (uint64_t)p; /* FNV-1a over the sequence */
      for (int64_t k = 0; k < l.n; ++k) {
        uint64_t v = ((uint64_t)(uint32_t)l.v[k].gid << 1) | (uint64_t)l.v[k].clamped;
        for (int byte = 0; byte < 8; ++byte) {
          h ^= (v >> (8 * byte)) & 0xffu;
          h *= 1099511628211ull;
        }
      }
      sig += h;
    }
    free(l.v);
  }
  free(first);
  return sig;
}

/* Marks (gmask[gid] = 1) every gaussian with an evaluation, at some pixel
 * before that pixel's early stop, whose discrete decision float32 may take
 * the other way: alpha against alpha_min (|q - tau| within the float32 bound
 * of q), or o exp(-q/2) against the alpha_max clamp (within the same bound,
 * as a relative change of alpha of half of it).  Such a gaussian's own
 * gradient can legitimately jump between a float32 and this double adjoint.
 * Returns how many gaussians are marked. */
int64_t oc_render_tiled_ambiguous(int64_t n, const double* geo, const int32_t* sorted_gid,
                                  const int32_t* batch_tab, int64_t nbatches,
                                  const oc_camera* cam, const oc_params* prm, uint8_t* gmask) {
  int32_t nmx = (cam->width + OC_MT_W - 1) / OC_MT_W;
  int32_t nmy = (cam->height + OC_MT_H - 1) / OC_MT_H;
  int64_t* first = first_batches(batch_tab, nbatches, nmx * nmy);
  int64_t total = (int64_t)cam->width * cam->height;
  memset(gmask, 0, (size_t)n);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t p = 0; p < total; ++p) {
    int32_t x = (int32_t)(p % cam->width), y = (int32_t)(p / cam->width);
    int32_t m = (y / OC_MT_H) * nmx + (x / OC_MT_W);
    double px = x + 0.5, py = y + 0.5;
    double Tacc = 1.0;
    for (int64_t bi = first[m]; bi < first[m + 1]; ++bi) {
      if (Tacc < prm->t_eps) break;
      const int32_t* bt = batch_tab + 3 * bi;
      double Tloc = 1.0;
      for (int32_t k = 0; k < bt[2]; ++k) {
        if (Tloc < prm->t_eps) break;
        int32_t gid = sorted_gid[bt[1] + k];
        const double* rec = geo + (int64_t)gid * G_NCOL;
        double dx = px - rec[G_MX], dy = py - rec[G_MY];
        double u = rec[G_L0] * dx + rec[G_L1] * dy, v = rec[G_L2] * dy;
        double q = u * u + v * v;
        double bound = 2.0 * oc_f32_q_bound(rec, dx, dy, u, v, q) + 1e-5 * (1.0 + rec[G_TAU]);
        double raw = rec[G_OP] * exp(-0.5 * q);
        int amb = fabs(q - rec[G_TAU]) <= bound ||
                  fabs(raw - prm->alpha_max) <= prm->alpha_max * 0.5 * bound;
        if (amb) {
#pragma omp atomic write
          gmask[gid] = 1;
        }
        double al = raw > prm->alpha_max ? prm->alpha_max : raw;
        if (al < prm->alpha_min) continue;
        Tloc = Tloc * (1.0 - al);
      }
      Tacc = Tacc * Tloc;
    }
  }
  free(first);
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i) cnt += gmask[i];
  return cnt;
}
