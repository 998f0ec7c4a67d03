// Adjoint of the frame path: gradients of a loss L(image, T) with respect to
// the gaussian means, scales, quaternions, opacities and SH coefficients.
//
// The paper renders forward only; its Forward-only paragraph names what the
// backward needs on top of the same macro-tile decomposition: the post-blend
// merge becomes a scan whose prefix is the transmittance before every batch,
// the point where transmittance saturates is needed per (pixel, batch), and
// reversing the blend divides by (1 - alpha), which it recommends doing in
// float32.  Three kernels, in stream order after a forward frame:
//
// merge_backward_kernel (one wave per render tile, one pixel per lane): walks
//   the macro-tile's active batches front to back for T_before (the merged
//   transmittance before each batch, 0 once the merge had stopped), then back
//   to front for the scalar suffix
//     X_after(b) = g . (composite of the later batches over the background)
//                  + dL/dT * (their transmittance),
//   with X <- g.C_b + T_b X, from the partials the forward left in memory
//   (g = dL/dimage at the pixel).  One float2 per (batch, tile, pixel).
// raster_backward_kernel (persistent, one workgroup per (macro-tile, batch)
//   unit, staged exactly as the forward): per tile and pixel a forward pass
//   re-runs the batch's compositing to find the pixel's final transmittance
//   and last contributing gaussian; a backward pass from there walks the
//   gaussians back to front, recovering T before each one as T / (1 - alpha)
//   (alpha <= alpha_max keeps the divisor >= 0.01), with
//     dL/dc_k = alpha_k T_k g,  dL/dalpha_k = T_k (g.c_k - X),
//     X <- alpha_k (g.c_k) + (1 - alpha_k) X,   T_k = T_before(batch) * T_local.
//   alpha = min(alpha_max, o 2^-q') (q' the prescaled quadratic form); the
//   clamp has zero derivative.  The nine record gradients of a gaussian are
//   summed over the wave's 64 pixels and added to a per-gaussian row with one
//   atomic instruction (nine lanes).
// project_backward_kernel (one thread per gaussian): reverse pass of the
//   projection in double precision (camera transform, quaternion rotation,
//   3D covariance, EWA Jacobian with its frustum clamp, dilation, Cholesky
//   factors, pixel centre) and of the float32 SH colour.
#include "raster_common.h"

namespace higs {

// per-gaussian record-gradient row (64 bytes; 9 used)
constexpr int kGradStride = 16;
enum { kGMx = 0, kGMy, kGL0, kGL1, kGL2, kGOp, kGR, kGG, kGB, kGradUsed };
constexpr float kLn2f = 0.6931471805599453f;

// ------------------------------------------------------------------ clear --
__global__ void bwd_clear_kernel(int64_t n_words, float* __restrict__ dgeo,
                                 DeviceCounters* __restrict__ dc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) dc->bwd_next = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n_words; k += stride)
    reinterpret_cast<float4*>(dgeo)[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// ---------------------------------------------------------- merge adjoint --
constexpr int kMergeBwdThreads = 256;
__global__ void __launch_bounds__(kMergeBwdThreads)
merge_backward_kernel(CamArgs cam, ParamArgs prm, const uint32_t* __restrict__ batch_first,
                      const uint32_t* __restrict__ active, const float4* __restrict__ partials,
                      const DeviceCounters* __restrict__ dc, const float* __restrict__ dimg,
                      const float* __restrict__ dT, float2* __restrict__ state) {
  const int tiles_x = (cam.width + kTile - 1) / kTile;
  const int tiles_y = (cam.height + kTile - 1) / kTile;
  const int tile = blockIdx.x * (kMergeBwdThreads / 64) + (threadIdx.x >> 6);
  if (tile >= tiles_x * tiles_y) return;
  const int lane = threadIdx.x & 63;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const uint32_t mt = (uint32_t)((ty / kMtTilesY) * cam.n_mt_x + tx / kMtTilesX);
  const uint32_t t = (uint32_t)((ty % kMtTilesY) * kMtTilesX + tx % kMtTilesX);
  const uint32_t nb = dc->overflow ? 0u : dc->n_batches;  // no batches after an overflow
  const uint32_t b0 = min(batch_first[mt], nb), b1 = min(batch_first[mt + 1], nb);
  const int x = tx * kTile + (lane & 7), y = ty * kTile + (lane >> 3);
  float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, gT = 0.0f;
  if (x < cam.width && y < cam.height) {
    const size_t pix = (size_t)y * cam.width + x;
    g0 = dimg[3 * pix + 0];
    g1 = dimg[3 * pix + 1];
    g2 = dimg[3 * pix + 2];
    if (dT) gT = dT[pix];
  }
  const float eps = prm.t_eps;
  // front to back: transmittance before each active batch
  float T = 1.0f;
  int64_t last = -1;  // last batch the merge took at this pixel
  for (uint32_t b = b0; b < b1; ++b) {
    if (!((active[b] >> t) & 1u)) continue;
    const size_t slot = ((size_t)b * kTilesPerMt + t) * 64 + lane;
    const bool merged = T >= eps;
    state[slot].x = merged ? T : 0.0f;
    if (merged) {
      T = T * partials[slot].w;
      last = b;
    }
  }
  // back to front: the suffix after each merged batch
  float X = (g0 * cam.bg[0] + g1 * cam.bg[1] + g2 * cam.bg[2]) + gT;
  for (int64_t b = (int64_t)b1 - 1; b >= (int64_t)b0; --b) {
    if (!((active[b] >> t) & 1u)) continue;
    const size_t slot = ((size_t)b * kTilesPerMt + t) * 64 + lane;
    state[slot].y = X;
    if (b <= last) {
      const float4 p = partials[slot];
      X = (g0 * p.x + g1 * p.y + g2 * p.z) + p.w * X;
    }
  }
}

// --------------------------------------------------------- raster adjoint --
constexpr int kRasterBwdThreads = 512;
constexpr int kRasterBwdWaves = kRasterBwdThreads / 64;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

__global__ void __launch_bounds__(kRasterBwdThreads)
raster_backward_kernel(CamArgs cam, ParamArgs prm, const uint32_t* __restrict__ vals0,
                       const uint32_t* __restrict__ vals1, const RasterRecord* __restrict__ rec,
                       const uint32_t* __restrict__ batch_tab, const uint32_t* __restrict__ active,
                       DeviceCounters* __restrict__ dc, const float2* __restrict__ state,
                       const float* __restrict__ dimg, float* __restrict__ dgeo) {
  __shared__ RasterLds L;
  if (dc->overflow) return;  // the frame stopped at a capacity overflow
  const uint32_t* __restrict__ sorted = dc->sort_final ? vals1 : vals0;
  const uint32_t n_units = dc->n_batches;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float eps = prm.t_eps, amax = prm.alpha_max;
  const float pxo = (float)(lane & 7) + 0.5f, pyo = (float)(lane >> 3) + 0.5f;

  for (;;) {
    if (tid == 0) {
      L.unit = atomicAdd(&dc->bwd_next, 1u);
      L.qnext = 0;
    }
    __syncthreads();
    const uint32_t u = L.unit;
    if (u >= n_units) break;
    const UnitInfo I = unit_info(cam, batch_tab, u);
    // the tiles the forward rasterised: a tile it left out (the merge had
    // stopped reading it) has neither a partial nor a merge state
    stage_unit<kRasterBwdWaves>(L, I, sorted, rec, lane, wave, ~active[u]);

    for (;;) {
      const int t = next_tile(L, lane);
      if (t < 0) break;
      const float pxr = (float)((t & 7) * kTile) + pxo;
      const float pyr = (float)((t >> 3) * kTile) + pyo;
      const int x = I.x0 + (t & 7) * kTile + (lane & 7), y = I.y0 + (t >> 3) * kTile + (lane >> 3);
      const float2 st = state[((size_t)u * kTilesPerMt + t) * 64 + lane];
      const bool live = x < cam.width && y < cam.height && st.x >= eps;
      if (__ballot(live) == 0) continue;
      float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
      if (live) {
        const size_t pix = (size_t)y * cam.width + x;
        g0 = dimg[3 * pix + 0];
        g1 = dimg[3 * pix + 1];
        g2 = dimg[3 * pix + 2];
      }

      // forward: the pixel's final local T and its last contributing gaussian
      float T = 1.0f;
      int last = -1;
      for (int k = 0; k < I.K; ++k) {
        uint64_t m = uniform64(L.masks[k][t]);
        while (m) {
          const int j = __ffsll((unsigned long long)m) - 1;
          m &= m - 1ull;
          const int gi = k * 64 + j;
          const float al = eval_alpha(L.ga[gi], L.gb[gi], L.gb[gi].y, pxr, pyr, amax).al;
          if (T >= eps && al >= kAlphaMin) {
            T = fmaf(-al, T, T);  // the forward's update, bit for bit
            last = gi;
          }
        }
        if (__ballot(T >= eps) == 0) break;
      }
      if (!live) last = -1;
      const int wlast = wave_max_int(last);
      if (wlast < 0) continue;

      // backward: back to front from the last contributing gaussian
      float X = st.y;
      const float Tin = st.x;
      for (int k = wlast >> 6; k >= 0; --k) {
        uint64_t m = uniform64(L.masks[k][t]);
        if (k == (wlast >> 6) && (wlast & 63) != 63) m &= (2ull << (wlast & 63)) - 1ull;
        while (m) {
          const int j = 63 - __clzll((long long)m);
          m &= ~(1ull << j);
          const int gi = k * 64 + j;
          const float4 A = L.ga[gi];
          const float4 B = L.gb[gi];
          const float4 C = L.gc[gi];
          const float bb = C.x;
          const PixelEval ev = eval_alpha(A, B, B.y, pxr, pyr, amax);
          const bool take = gi <= last && ev.al >= kAlphaMin;
          if (__ballot(take) == 0) continue;
          float d0 = 0.0f, d1 = 0.0f, d2 = 0.0f, d3 = 0.0f, d4 = 0.0f, d5 = 0.0f, d6 = 0.0f,
                d7 = 0.0f, d8 = 0.0f;
          if (take) {
            const float om = 1.0f - ev.al;
            const float Tb = T / om;  // local transmittance before this gaussian
            const float Tk = Tin * Tb;
            const float gcol = (g0 * B.z + g1 * B.w) + g2 * bb;
            const float dal = Tk * (gcol - X);
            X = ev.al * gcol + om * X;
            T = Tb;
            const float w = ev.al * Tk;
            d6 = w * g0;
            d7 = w * g1;
            d8 = w * g2;
            if (ev.e < amax) {  // alpha not clamped
              d5 = dal * (ev.e / C.y);  // d alpha / d o = exp(-q/2); o > 0 for a listed gaussian
              const float dq = -dal * ev.al * kLn2f;  // dL/dq'
              const float du = 2.0f * ev.u * dq, dv = 2.0f * ev.v * dq;
              const float dx = pxr - C.z, dy = pyr - C.w;  // pixel minus centre
              d2 = du * dx;
              d3 = du * dy;
              d4 = dv * dy;
              d0 = -du * A.z;
              d1 = -(du * A.w + dv * B.x);
            }
          }
          d0 = wave_sum(d0);
          d1 = wave_sum(d1);
          d2 = wave_sum(d2);
          d3 = wave_sum(d3);
          d4 = wave_sum(d4);
          d5 = wave_sum(d5);
          d6 = wave_sum(d6);
          d7 = wave_sum(d7);
          d8 = wave_sum(d8);
          const uint32_t gid = sorted[I.start + gi];
          if (lane < kGradUsed) {
            const float v = lane == 0 ? d0 : lane == 1 ? d1 : lane == 2 ? d2 : lane == 3 ? d3
                          : lane == 4 ? d4 : lane == 5 ? d5 : lane == 6 ? d6 : lane == 7 ? d7 : d8;
            atomicAdd(dgeo + (size_t)gid * kGradStride + lane, v);
          }
        }
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------- projection adjoint --
constexpr int kProjBwdBlock = 256;

// SH basis (3DGS convention, closed-form normalisations) and its derivative
// with respect to the unnormalised direction components taken independently.
__device__ __forceinline__ void sh_basis_and_grad(float x, float y, float z, int degree, float* Y,
                                                  float* Yx, float* Yy, float* Yz) {
  const float c0 = 0.28209479177387814f;       // 1/(2 sqrt(pi))
  const float c1 = 0.4886025119029199f;        // sqrt(3/(4 pi))
  const float c2a = 1.0925484305920792f;       // sqrt(15/pi)/2
  const float c2b = 0.31539156525252005f;      // sqrt(5/pi)/4
  const float c2c = 0.5462742152960396f;       // sqrt(15/pi)/4
  const float c3a = 0.5900435899266435f;       // sqrt(35/(2 pi))/4
  const float c3b = 2.890611442640554f;        // sqrt(105/pi)/2
  const float c3c = 0.4570457994644658f;       // sqrt(21/(2 pi))/4
  const float c3d = 0.3731763325901154f;       // sqrt(7/pi)/4
  const float c3e = 1.445305721320277f;        // sqrt(105/pi)/4
#pragma unroll
  for (int k = 0; k < 16; ++k) Y[k] = Yx[k] = Yy[k] = Yz[k] = 0.0f;
  Y[0] = c0;
  if (degree < 1) return;
  Y[1] = -c1 * y;  Yy[1] = -c1;
  Y[2] = c1 * z;   Yz[2] = c1;
  Y[3] = -c1 * x;  Yx[3] = -c1;
  if (degree < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = c2a * x * y;                 Yx[4] = c2a * y;          Yy[4] = c2a * x;
  Y[5] = -c2a * y * z;                Yy[5] = -c2a * z;         Yz[5] = -c2a * y;
  Y[6] = c2b * (2.0f * zz - xx - yy); Yx[6] = -2.0f * c2b * x;  Yy[6] = -2.0f * c2b * y;
                                      Yz[6] = 4.0f * c2b * z;
  Y[7] = -c2a * x * z;                Yx[7] = -c2a * z;         Yz[7] = -c2a * x;
  Y[8] = c2c * (xx - yy);             Yx[8] = 2.0f * c2c * x;   Yy[8] = -2.0f * c2c * y;
  if (degree < 3) return;
  // 9: -c3a y (3x^2 - y^2)
  Y[9] = -c3a * y * (3.0f * xx - yy);
  Yx[9] = -6.0f * c3a * x * y;
  Yy[9] = -3.0f * c3a * (xx - yy);
  // 10: c3b x y z
  Y[10] = c3b * x * y * z;
  Yx[10] = c3b * y * z;
  Yy[10] = c3b * x * z;
  Yz[10] = c3b * x * y;
  // 11: -c3c y (4z^2 - x^2 - y^2)
  Y[11] = -c3c * y * (4.0f * zz - xx - yy);
  Yx[11] = 2.0f * c3c * x * y;
  Yy[11] = -c3c * (4.0f * zz - xx - 3.0f * yy);
  Yz[11] = -8.0f * c3c * y * z;
  // 12: c3d z (2z^2 - 3x^2 - 3y^2)
  Y[12] = c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Yx[12] = -6.0f * c3d * x * z;
  Yy[12] = -6.0f * c3d * y * z;
  Yz[12] = c3d * (6.0f * zz - 3.0f * xx - 3.0f * yy);
  // 13: -c3c x (4z^2 - x^2 - y^2)
  Y[13] = -c3c * x * (4.0f * zz - xx - yy);
  Yx[13] = -c3c * (4.0f * zz - 3.0f * xx - yy);
  Yy[13] = 2.0f * c3c * x * y;
  Yz[13] = -8.0f * c3c * x * z;
  // 14: c3e z (x^2 - y^2)
  Y[14] = c3e * z * (xx - yy);
  Yx[14] = 2.0f * c3e * x * z;
  Yy[14] = -2.0f * c3e * y * z;
  Yz[14] = c3e * (xx - yy);
  // 15: -c3a x (x^2 - 3y^2)
  Y[15] = -c3a * x * (xx - 3.0f * yy);
  Yx[15] = -3.0f * c3a * (xx - yy);
  Yy[15] = 6.0f * c3a * x * y;
}

__global__ void __launch_bounds__(kProjBwdBlock)
project_backward_kernel(int64_t n, const float* __restrict__ means, const float* __restrict__ scales,
                        const float* __restrict__ quats, const float* __restrict__ sh, CamArgs cam,
                        ParamArgs prm, float3 campos, const uint32_t* __restrict__ f_cnt,
                        const RasterRecord* __restrict__ rec, const float* __restrict__ dgeo,
                        const DeviceCounters* __restrict__ dc, float* __restrict__ dmeans,
                        float* __restrict__ dscales, float* __restrict__ dquats,
                        float* __restrict__ dopac, float* __restrict__ dsh) {
  const int64_t i = (int64_t)blockIdx.x * kProjBwdBlock + threadIdx.x;
  if (i >= n) return;
  const int ncoef = (prm.sh_degree + 1) * (prm.sh_degree + 1);
  float* gsh = dsh + (int64_t)ncoef * 3 * i;
  // culled or off-screen: no pixel depends on it (0); after a capacity
  // overflow the frame has no gradient (NaN)
  const bool ovf = dc->overflow != 0;
  if (ovf || f_cnt[i] == 0) {
    const float z = ovf ? __builtin_nanf("") : 0.0f;
    for (int k = 0; k < 3; ++k) dmeans[3 * i + k] = dscales[3 * i + k] = z;
    for (int k = 0; k < 4; ++k) dquats[4 * i + k] = z;
    for (int k = 0; k < ncoef * 3; ++k) gsh[k] = z;
    dopac[i] = z;
    return;
  }
  const float* gr = dgeo + (size_t)i * kGradStride;
  // the rasteriser worked with l' = l sqrt(log2(e)/2)
  const double ks = (double)kSqrtHalfLog2e;
  const double g_px = gr[kGMx], g_py = gr[kGMy];
  const double g_l0 = gr[kGL0] * ks, g_l1 = gr[kGL1] * ks, g_l2 = gr[kGL2] * ks;
  dopac[i] = gr[kGOp];

  // ---- replay of the geometry (double) ----
  const double m[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
  const double sc[3] = {scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]};
  const double q4[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
  double R[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = cam.R[k];
  double p[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) p[r] = R[3 * r] * m[0] + R[3 * r + 1] * m[1] + R[3 * r + 2] * m[2] + (double)cam.t[r];
  const double qn = sqrt(q4[0] * q4[0] + q4[1] * q4[1] + q4[2] * q4[2] + q4[3] * q4[3]);
  const double w = q4[0] / qn, qx = q4[1] / qn, qy = q4[2] / qn, qz = q4[3] / qn;
  const double Rg[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - w * qz), 2.0 * (qx * qz + w * qy),
                        2.0 * (qx * qy + w * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - w * qx),
                        2.0 * (qx * qz - w * qy), 2.0 * (qy * qz + w * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
  double Ms[9];  // Rg diag(s)
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Ms[3 * r + c] = Rg[3 * r + c] * sc[c];
  double Sg[9];  // Ms Ms^T
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Sg[3 * r + c] = Ms[3 * r] * Ms[3 * c] + Ms[3 * r + 1] * Ms[3 * c + 1] + Ms[3 * r + 2] * Ms[3 * c + 2];
  const double fx = cam.fx, fy = cam.fy;
  const double Wd = cam.width, Hd = cam.height;
  const double limx = 0.3 * Wd / (2.0 * fx), limy = 0.3 * Hd / (2.0 * fy);
  const double xlo = -((double)cam.cx / fx + limx), xhi = (Wd - (double)cam.cx) / fx + limx;
  const double ylo = -((double)cam.cy / fy + limy), yhi = (Hd - (double)cam.cy) / fy + limy;
  const double rx = p[0] / p[2], ry = p[1] / p[2];
  const bool free_x = rx >= xlo && rx <= xhi, free_y = ry >= ylo && ry <= yhi;
  const double xr = free_x ? rx : (rx < xlo ? xlo : xhi);
  const double yr = free_y ? ry : (ry < ylo ? ylo : yhi);
  const double iz = 1.0 / p[2];
  // Jacobian rows: J0 = (fx/z, 0, -fx xr / z), J1 = (0, fy/z, -fy yr / z); V = J R
  const double a00 = fx * iz, a02 = -fx * xr * iz, a11 = fy * iz, a12 = -fy * yr * iz;
  double V0[3], V1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    V0[k] = a00 * R[k] + a02 * R[6 + k];
    V1[k] = a11 * R[3 + k] + a12 * R[6 + k];
  }
  double SV0[3], SV1[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    SV0[r] = Sg[3 * r] * V0[0] + Sg[3 * r + 1] * V0[1] + Sg[3 * r + 2] * V0[2];
    SV1[r] = Sg[3 * r] * V1[0] + Sg[3 * r + 1] * V1[1] + Sg[3 * r + 2] * V1[2];
  }
  const double ca = V0[0] * SV0[0] + V0[1] * SV0[1] + V0[2] * SV0[2] + (double)prm.dilation;
  const double cb = V0[0] * SV1[0] + V0[1] * SV1[1] + V0[2] * SV1[2];
  const double cc = V1[0] * SV1[0] + V1[1] * SV1[1] + V1[2] * SV1[2] + (double)prm.dilation;
  const double det = ca * cc - cb * cb;

  // ---- reverse ----
  // l0 = sqrt(c/det), l1 = -b / sqrt(c det), l2 = c^-1/2
  const double l0 = sqrt(cc / det), s_cd = sqrt(cc * det), l2 = 1.0 / sqrt(cc);
  const double g_det = g_l0 * (-0.5 * l0 / det) + g_l1 * (0.5 * cb * cc / (s_cd * s_cd * s_cd));
  const double g_ca = g_det * cc;
  const double g_cb = -g_l1 / s_cd - 2.0 * cb * g_det;
  const double g_cc = g_l0 * (0.5 / (l0 * det)) + g_l1 * (0.5 * cb * det / (s_cd * s_cd * s_cd)) +
                      g_l2 * (-0.5 * l2 * l2 * l2) + g_det * ca;
  // covariance entries a = V0 S V0', b = V0 S V1', c = V1 S V1'
  double gV0[3], gV1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gV0[k] = 2.0 * g_ca * SV0[k] + g_cb * SV1[k];
    gV1[k] = g_cb * SV0[k] + 2.0 * g_cc * SV1[k];
  }
  // dL/dS (symmetrised) = g_a V0 V0' + g_b (V0 V1' + V1 V0')/2 + g_c V1 V1'; S = Ms Ms'
  // -> dL/dMs = 2 dL/dS Ms
  double gMs[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double gs = g_ca * V0[r] * V0[k] + 0.5 * g_cb * (V0[r] * V1[k] + V1[r] * V0[k]) +
                          g_cc * V1[r] * V1[k];
        acc += gs * Ms[3 * k + c];
      }
      gMs[3 * r + c] = 2.0 * acc;
    }
  double gRg[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      gRg[3 * r + c] = gMs[3 * r + c] * sc[c];
      acc += gMs[3 * r + c] * Rg[3 * r + c];
    }
    dscales[3 * i + c] = (float)acc;
  }
  // rotation matrix entries as polynomials of the unit quaternion (w, x, y, z)
  const double gw = 2.0 * (-qz * gRg[1] + qy * gRg[2] + qz * gRg[3] - qx * gRg[5] - qy * gRg[6] + qx * gRg[7]);
  const double gx = 2.0 * (-2.0 * qx * gRg[4] - 2.0 * qx * gRg[8] + qy * gRg[1] + qz * gRg[2] + qy * gRg[3] -
                           w * gRg[5] + qz * gRg[6] + w * gRg[7]);
  const double gy = 2.0 * (-2.0 * qy * gRg[0] - 2.0 * qy * gRg[8] + qx * gRg[1] + w * gRg[2] + qx * gRg[3] +
                           qz * gRg[5] - w * gRg[6] + qz * gRg[7]);
  const double gz = 2.0 * (-2.0 * qz * gRg[0] - 2.0 * qz * gRg[4] - w * gRg[1] + qx * gRg[2] + w * gRg[3] +
                           qy * gRg[5] + qx * gRg[6] + qy * gRg[7]);
  const double dotq = w * gw + qx * gx + qy * gy + qz * gz;
  dquats[4 * i + 0] = (float)((gw - w * dotq) / qn);
  dquats[4 * i + 1] = (float)((gx - qx * dotq) / qn);
  dquats[4 * i + 2] = (float)((gy - qy * dotq) / qn);
  dquats[4 * i + 3] = (float)((gz - qz * dotq) / qn);
  // V = J R: dL/dJ entries
  double g_a00 = 0.0, g_a02 = 0.0, g_a11 = 0.0, g_a12 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g_a00 += gV0[k] * R[k];
    g_a02 += gV0[k] * R[6 + k];
    g_a11 += gV1[k] * R[3 + k];
    g_a12 += gV1[k] * R[6 + k];
  }
  // a00 = fx/z, a02 = -fx xr/z, a11 = fy/z, a12 = -fy yr/z, xr = x/z unless clamped;
  // plus the pixel centre u = fx x/z + cx, v = fy y/z + cy
  double gpx = g_px * fx * iz, gpy = g_py * fy * iz;
  double gpz = -(g_px * fx * p[0] + g_py * fy * p[1]) * iz * iz;
  gpz += -(g_a00 * fx + g_a11 * fy) * iz * iz;
  const double g_xr = -g_a02 * fx * iz, g_yr = -g_a12 * fy * iz;
  gpz += (g_a02 * fx * xr + g_a12 * fy * yr) * iz * iz;
  if (free_x) {
    gpx += g_xr * iz;
    gpz -= g_xr * p[0] * iz * iz;
  }
  if (free_y) {
    gpy += g_yr * iz;
    gpz -= g_yr * p[1] * iz * iz;
  }
  double gm[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gm[k] = R[k] * gpx + R[3 + k] * gpy + R[6 + k] * gpz;

  // ---- SH colour (float32, as the forward) ----
  float ex = (float)m[0] - campos.x, ey = (float)m[1] - campos.y, ez = (float)m[2] - campos.z;
  const float en2 = ex * ex + ey * ey + ez * ez;
  const float inv = en2 > 0.0f ? 1.0f / sqrtf(en2) : 0.0f;
  const float dx = en2 > 0.0f ? ex * inv : ex, dy = en2 > 0.0f ? ey * inv : ey,
              dz = en2 > 0.0f ? ez * inv : ez;
  float Y[16], Yx[16], Yy[16], Yz[16];
  sh_basis_and_grad(dx, dy, dz, prm.sh_degree, Y, Yx, Yy, Yz);
  const float* shi = sh + (int64_t)ncoef * 3 * i;
  const RasterRecord& rr = rec[i];
  // a channel clamped at 0 in the forward passes no gradient
  const float gc[3] = {rr.r > 0.0f ? gr[kGR] : 0.0f, rr.g > 0.0f ? gr[kGG] : 0.0f,
                       rr.b > 0.0f ? gr[kGB] : 0.0f};
  float gdx = 0.0f, gdy = 0.0f, gdz = 0.0f;
  for (int k = 0; k < ncoef; ++k) {
    float gy_k = 0.0f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      gsh[3 * k + ch] = gc[ch] * Y[k];
      gy_k += gc[ch] * shi[3 * k + ch];
    }
    gdx += gy_k * Yx[k];
    gdy += gy_k * Yy[k];
    gdz += gy_k * Yz[k];
  }
  if (en2 > 0.0f) {
    const float dd = dx * gdx + dy * gdy + dz * gdz;
    gm[0] += (double)((gdx - dx * dd) * inv);
    gm[1] += (double)((gdy - dy * dd) * inv);
    gm[2] += (double)((gdz - dz * dd) * inv);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) dmeans[3 * i + k] = (float)gm[k];
}

// ---------------------------------------------------------------- launch --
static int g_bwd_per_cu = 0;

hipError_t launch_backward(int64_t n, const float* means, const float* scales, const float* quats,
                           const float* sh, CamArgs cam, ParamArgs prm,
                           const uint32_t* const* vals2, const RasterRecord* rec,
                           const uint32_t* f_cnt, const uint32_t* batch_tab,
                           const uint32_t* batch_first, const uint32_t* active,
                           const float4* partials, DeviceCounters* dc, const float* dimg,
                           const float* dT, float2* state, float* dgeo, float* dmeans,
                           float* dscales, float* dquats, float* dopac, float* dsh, int n_cus,
                           hipStream_t s) {
  if (g_bwd_per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, raster_backward_kernel, kRasterBwdThreads,
                                                     0) != hipSuccess ||
        nb < 1)
      nb = 1;
    g_bwd_per_cu = nb;
  }
  const int64_t words = (n > 0 ? n : 0) * (kGradStride / 4);
  const int64_t want = (words + 255) / 256 + 1;
  const unsigned cblocks = (unsigned)(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(bwd_clear_kernel, dim3(cblocks), dim3(256), 0, s, words, dgeo, dc);
  const int tiles = ((cam.width + kTile - 1) / kTile) * ((cam.height + kTile - 1) / kTile);
  const int mblocks = (tiles + (kMergeBwdThreads / 64) - 1) / (kMergeBwdThreads / 64);
  if (mblocks > 0)
    hipLaunchKernelGGL(merge_backward_kernel, dim3(mblocks), dim3(kMergeBwdThreads), 0, s, cam, prm,
                       batch_first, active, partials, dc, dimg, dT, state);
  hipLaunchKernelGGL(raster_backward_kernel, dim3(n_cus * g_bwd_per_cu), dim3(kRasterBwdThreads), 0,
                     s, cam, prm, vals2[0], vals2[1], rec, batch_tab, active, dc, state, dimg, dgeo);
  if (n > 0) {
    float3 campos;
    campos.x = -(cam.R[0] * cam.t[0] + cam.R[3] * cam.t[1] + cam.R[6] * cam.t[2]);
    campos.y = -(cam.R[1] * cam.t[0] + cam.R[4] * cam.t[1] + cam.R[7] * cam.t[2]);
    campos.z = -(cam.R[2] * cam.t[0] + cam.R[5] * cam.t[1] + cam.R[8] * cam.t[2]);
    const unsigned pblocks = (unsigned)((n + kProjBwdBlock - 1) / kProjBwdBlock);
    hipLaunchKernelGGL(project_backward_kernel, dim3(pblocks), dim3(kProjBwdBlock), 0, s, n, means,
                       scales, quats, sh, cam, prm, campos, f_cnt, rec, dgeo, dc, dmeans,
                       dscales, dquats, dopac, dsh);
  }
  return hipGetLastError();
}

}  // namespace higs
