// Stage 1: fused projection + SH (sec. 4.2, Projection and SH evaluation).
//
// One thread per gaussian, 256 per block.  The geometry (camera transform,
// 3D covariance from scale and rotation, EWA Jacobian with the frustum clamp,
// 2D covariance with dilation, Cholesky factors of its inverse, opacity level)
// runs in double precision with a fixed operation order and no contraction,
// then every stored field is the float32 rounding of its double value: the
// discrete decisions downstream (pair lists, depth order, batches) depend only
// on these fields, so they can be reproduced bit for bit.  The SH colour runs
// in float32.  The same thread counts the gaussian's macro-tile pairs
// (predicate.h); the block writes the sums of its pair counts and visible
// gaussians for the emission scan and folds the depth bits of its visible
// gaussians into the frame's [min, max] (used to compress the sort keys).
//
// Outputs: SoA binning fields (coalesced), a 48-byte raster record per
// visible gaussian, per-gaussian pair counts, the compact form of each visible
// gaussian's macro-tile list (predicate.h, SpanTracker) and per-block count
// sums.
#include "higs_internal.h"
#include "predicate.h"
#include "shcodec.h"

namespace higs {

// Real SH normalisations from their closed forms, 3DGS sign convention
// (Condon-Shortley phase kept): Y_lm for m<0 is sqrt2 Im Y_l^|m|, m>0 sqrt2 Re.
constexpr float kY00 = 0.28209479177387814f;  // 1/(2 sqrt(pi))
constexpr float kY1 = 0.4886025119029199f;    // sqrt(3/(4 pi))
constexpr float kY2a = 1.0925484305920792f;   // sqrt(15/pi)/2
constexpr float kY2b = 0.31539156525252005f;  // sqrt(5/pi)/4
constexpr float kY2c = 0.5462742152960396f;   // sqrt(15/pi)/4
constexpr float kY3a = 0.5900435899266435f;   // sqrt(35/(2 pi))/4
constexpr float kY3b = 2.890611442640554f;    // sqrt(105/pi)/2
constexpr float kY3c = 0.4570457994644658f;   // sqrt(21/(2 pi))/4
constexpr float kY3d = 0.3731763325901154f;   // sqrt(7/pi)/4
constexpr float kY3e = 1.445305721320277f;    // sqrt(105/pi)/4

struct Geo {
  double tz, px, py, a, b, c, tau, l0, l1, l2;
};

// Double-precision geometry; false when the gaussian is culled.
__device__ __forceinline__ bool geometry(float3 mean, float3 scale, float4 quat, float opac,
                                         const CamArgs& cam, const ParamArgs& prm, Geo& g) {
#pragma clang fp contract(off)
  const double mx = mean.x, my = mean.y, mz = mean.z;
  const double s0 = scale.x, s1 = scale.y, s2 = scale.z;
  const double qw = quat.x, qx = quat.y, qy = quat.z, qz = quat.w;
  const double o = opac;
  if (!(isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(s0) && isfinite(s1) &&
        isfinite(s2) && isfinite(qw) && isfinite(qx) && isfinite(qy) && isfinite(qz) &&
        isfinite(o)))
    return false;
  double R[9], t[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = (double)cam.R[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) t[k] = (double)cam.t[k];

  // camera-space mean
  const double tx = ((R[0] * mx + R[1] * my) + R[2] * mz) + t[0];
  const double ty = ((R[3] * mx + R[4] * my) + R[5] * mz) + t[1];
  const double tz = ((R[6] * mx + R[7] * my) + R[8] * mz) + t[2];
  if (!(tz > (double)prm.near_z)) return false;

  // rotation of the unit quaternion
  const double n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  if (!(n2 > 0.0)) return false;
  const double nrm = sqrt(n2);
  const double w = qw / nrm, x = qx / nrm, y = qy / nrm, z = qz / nrm;
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

  // Sigma_3D = (G S)(G S)^T
  double M[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    M[i * 3 + 0] = G[i * 3 + 0] * s0;
    M[i * 3 + 1] = G[i * 3 + 1] * s1;
    M[i * 3 + 2] = G[i * 3 + 2] * s2;
  }
  double S[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      S[i * 3 + j] =
          (M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1]) + M[i * 3 + 2] * M[j * 3 + 2];

  // EWA: Jacobian of the perspective map at the (frustum-clamped) mean
  const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
  const double W = (double)cam.width, H = (double)cam.height;
  const double tanx = W / (2.0 * fx), tany = H / (2.0 * fy);
  const double xlo = -(cx / fx + 0.3 * tanx), xhi = (W - cx) / fx + 0.3 * tanx;
  const double ylo = -(cy / fy + 0.3 * tany), yhi = (H - cy) / fy + 0.3 * tany;
  double xr = tx / tz, yr = ty / tz;
  if (xr < xlo) xr = xlo;
  if (xr > xhi) xr = xhi;
  if (yr < ylo) yr = ylo;
  if (yr > yhi) yr = yhi;
  const double xc = xr * tz, yc = yr * tz;
  const double j00 = fx / tz, j02 = -(fx * xc) / (tz * tz);
  const double j11 = fy / tz, j12 = -(fy * yc) / (tz * tz);
  double T0[3], T1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T0[k] = j00 * R[0 * 3 + k] + j02 * R[2 * 3 + k];
    T1[k] = j11 * R[1 * 3 + k] + j12 * R[2 * 3 + k];
  }
  double U0[3], U1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    U0[k] = (T0[0] * S[0 * 3 + k] + T0[1] * S[1 * 3 + k]) + T0[2] * S[2 * 3 + k];
    U1[k] = (T1[0] * S[0 * 3 + k] + T1[1] * S[1 * 3 + k]) + T1[2] * S[2 * 3 + k];
  }
  const double s00 = (U0[0] * T0[0] + U0[1] * T0[1]) + U0[2] * T0[2];
  const double s01 = (U0[0] * T1[0] + U0[1] * T1[1]) + U0[2] * T1[2];
  const double s11 = (U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2];
  const double a = s00 + (double)prm.dilation, b = s01, c = s11 + (double)prm.dilation;
  const double det = a * c - b * b;
  if (!(det > 0.0)) return false;

  // opacity level: o exp(-q/2) >= 1/255 <=> q <= 2 ln(255 o); 255 o is exact
  if (!(255.0 * o >= 1.0)) return false;
  g.tau = 2.0 * log(255.0 * o);

  // Cholesky factors of the inverse covariance (sec. 3.5)
  g.l0 = sqrt(c / det);
  g.l1 = -b / sqrt(c * det);
  g.l2 = 1.0 / sqrt(c);
  g.px = (fx * tx) / tz + cx;
  g.py = (fy * ty) / tz + cy;
  g.tz = tz;
  g.a = a;
  g.b = b;
  g.c = c;
  return true;
}

__device__ __forceinline__ float3 operator*(float s, float3 v) { return make_float3(s * v.x, s * v.y, s * v.z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }

// View-dependent colour, float32: rgb = max(0, 0.5 + sum_k Y_k(d) sh_k);
// co(k) gives coefficient k.
template <class Co>
__device__ __forceinline__ float3 sh_colour(Co&& co, int degree, float x, float y, float z) {
  float3 acc = kY00 * co(0);
  if (degree >= 1) {
    acc = acc + (-kY1 * y) * co(1) + (kY1 * z) * co(2) + (-kY1 * x) * co(3);
  }
  if (degree >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    acc = acc + (kY2a * (x * y)) * co(4) + (-kY2a * (y * z)) * co(5) +
          (kY2b * (2.0f * zz - xx - yy)) * co(6) + (-kY2a * (x * z)) * co(7) +
          (kY2c * (xx - yy)) * co(8);
    if (degree >= 3) {
      acc = acc + (-kY3a * y * (3.0f * xx - yy)) * co(9) + (kY3b * x * y * z) * co(10) +
            (-kY3c * y * (4.0f * zz - xx - yy)) * co(11) +
            (kY3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy)) * co(12) +
            (-kY3c * x * (4.0f * zz - xx - yy)) * co(13) + (kY3e * z * (xx - yy)) * co(14) +
            (-kY3a * x * (xx - 3.0f * yy)) * co(15);
    }
  }
  return make_float3(fmaxf(0.0f, 0.5f + acc.x), fmaxf(0.0f, 0.5f + acc.y), fmaxf(0.0f, 0.5f + acc.z));
}

// A workgroup takes 256 gaussians of one view; the views of one range of
// gaussians are neighbouring workgroups (workgroup w: view w mod V, block
// w / V), so views of one scene find its arrays in the caches.  Every output
// sits at the virtual index v * n_pad + i.
__global__ void __launch_bounds__(kProjBlock)
project_kernel(Views views, CamArgs shape, ParamArgs prm, float* __restrict__ f_mx,
               float* __restrict__ f_my, float* __restrict__ f_a, float* __restrict__ f_b,
               float* __restrict__ f_c, float* __restrict__ f_tau, uint32_t* __restrict__ f_key,
               uint32_t* __restrict__ f_cnt, uint32_t* __restrict__ f_span,
               RasterRecord* __restrict__ rec, uint32_t* __restrict__ block_sums,
               DeviceCounters* __restrict__ dc, bool all_fields, bool sh_packed) {
  __shared__ uint32_t wave_min[kProjBlock / 64], wave_max[kProjBlock / 64];
  __shared__ uint32_t wave_sums[2][kProjBlock / 64];
  __shared__ float sh_scale[kShComps];
  // the block's 48-byte raster records, written out together after the
  // block's barrier: 16-byte stores of consecutive addresses, where each
  // thread's own three stores 48 bytes apart cost 15% of the kernel
  __shared__ float4 rec_stage[3 * kProjBlock];
  float4 rq0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), rq1 = rq0, rq2 = rq0;
  const int view = (int)(blockIdx.x % (uint32_t)views.count);
  const int64_t blk = (int64_t)(blockIdx.x / (uint32_t)views.count);
  const ViewArgs w = views.get(view);
  const float* __restrict__ means = w.means;
  const float* __restrict__ scales = w.scales;
  const float* __restrict__ quats = w.quats;
  const float* __restrict__ opac = w.opac;
  const float* __restrict__ sh = w.sh;
  const int64_t n = w.n;
  CamArgs cam = shape;
  cam.fx = w.fx;
  cam.fy = w.fy;
  cam.cx = w.cx;
  cam.cy = w.cy;
#pragma unroll
  for (int k = 0; k < 9; ++k) cam.R[k] = w.R[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) cam.t[k] = w.t[k];
  const float3 campos = make_float3(w.campos[0], w.campos[1], w.campos[2]);
  const bool sh_vec4 = (reinterpret_cast<uintptr_t>(sh) & 15u) == 0;
  const int64_t i = blk * kProjBlock + threadIdx.x;  // in the view
  const int64_t vi = view * views.n_pad + i;           // virtual
  uint32_t cnt = 0;
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  // degree 3 with a 16-byte aligned sh array: the 48 coefficients (192
  // bytes) in twelve 16-byte loads once the gaussian is known to be visible
  // (not held across the geometry: 94 VGPRs, five waves per SIMD, whose
  // interleaving hides the loads); packed SH: the 32 bytes of the gaussian
  // and, in LDS, the 48 scales of the header
  float4 shv[12];
  uint32_t shw[8];
  const bool early = !sh_packed && sh_vec4 && prm.sh_degree == 3 && i < n;
  if (sh_packed) {
    if (threadIdx.x < kShComps) sh_scale[threadIdx.x] = sh[threadIdx.x];
    if (i < n) {
      const uint4* src = reinterpret_cast<const uint4*>(
          reinterpret_cast<const char*>(sh) + kShHeaderBytes + 32 * (size_t)i);
      const uint4 w0 = src[0], w1 = src[1];
      shw[0] = w0.x, shw[1] = w0.y, shw[2] = w0.z, shw[3] = w0.w;
      shw[4] = w1.x, shw[5] = w1.y, shw[6] = w1.z, shw[7] = w1.w;
    }
    __syncthreads();
  }
  if (i < n) {
    const float3 mean = make_float3(means[3 * i + 0], means[3 * i + 1], means[3 * i + 2]);
    const float3 scale = make_float3(scales[3 * i + 0], scales[3 * i + 1], scales[3 * i + 2]);
    const float4 quat = make_float4(quats[4 * i + 0], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]);
    const float o = opac[i];
    Geo g;
    uint32_t key = 0;
    if (geometry(mean, scale, quat, o, cam, prm, g)) {
      BinFields f;
      f.mx = (float)g.px;
      f.my = (float)g.py;
      f.a = (float)g.a;
      f.b = (float)g.b;
      f.c = (float)g.c;
      f.tau = (float)g.tau;
      const float tzf = (float)g.tz;
      key = __float_as_uint(tzf);
      SpanTracker span;
      cnt = visit_macro_tiles_ji(f, cam.width, cam.height, cam.n_mt_x, cam.n_mt_y,
                                 [&](int j, int ic) { span.add(j, ic); });
      const uint32_t sw = cnt > 0 ? span.encode() : 0u;
      if (cnt > 0) f_span[vi] = sw;
      // the binning fields: read again only for a list the span word cannot
      // hold (and by the debug read-back)
      if (all_fields || (cnt > 0 && sw == 0)) {
        f_mx[vi] = f.mx;
        f_my[vi] = f.my;
        f_a[vi] = f.a;
        f_b[vi] = f.b;
        f_c[vi] = f.c;
        f_tau[vi] = f.tau;
      }
      if (cnt > 0) {
        kmin = key;
        kmax = key;
        const int ncoef = (prm.sh_degree + 1) * (prm.sh_degree + 1);
        float dx = mean.x - campos.x, dy = mean.y - campos.y, dz = mean.z - campos.z;
        const float dn2 = dx * dx + dy * dy + dz * dz;
        if (dn2 > 0.0f) {
          const float inv = 1.0f / sqrtf(dn2);
          dx *= inv;
          dy *= inv;
          dz *= inv;
        }
        float3 rgb;
        if (sh_packed) {
          rgb = sh_colour([&](int k) { return sh_unpack(shw, sh_scale, k); }, 3, dx, dy, dz);
        } else if (early) {
          {
            const float4* src = reinterpret_cast<const float4*>(sh + 48 * i);
#pragma unroll
            for (int k = 0; k < 12; ++k) shv[k] = src[k];
          }
          const float* c = reinterpret_cast<const float*>(shv);
          rgb = sh_colour([&](int k) { return make_float3(c[3 * k], c[3 * k + 1], c[3 * k + 2]); },
                          3, dx, dy, dz);
        } else {
          const float* c = sh + (int64_t)ncoef * 3 * i;
          rgb = sh_colour([&](int k) { return make_float3(c[3 * k], c[3 * k + 1], c[3 * k + 2]); },
                          prm.sh_degree, dx, dy, dz);
        }
        RasterRecord r;
        r.mx = f.mx;
        r.my = f.my;
        r.l0 = (float)g.l0;
        r.l1 = (float)g.l1;
        r.l2 = (float)g.l2;
        r.o = o;
        r.r = rgb.x;
        r.g = rgb.y;
        r.b = rgb.z;
        r.tau = f.tau;
        r.pad0 = 0.0f;
        r.pad1 = 0.0f;
        rq0 = make_float4(r.mx, r.my, r.l0, r.l1);
        rq1 = make_float4(r.l2, r.o, r.r, r.g);
        rq2 = make_float4(r.b, r.tau, 0.0f, 0.0f);
      }
    }
    f_key[vi] = key;
    f_cnt[vi] = cnt;
  } else if (i < views.n_pad) {  // padding of the view's range
    f_key[vi] = 0u;
    f_cnt[vi] = 0u;
  }
  rec_stage[3 * threadIdx.x + 0] = rq0;
  rec_stage[3 * threadIdx.x + 1] = rq1;
  rec_stage[3 * threadIdx.x + 2] = rq2;
  // block sums of the pair counts and visible gaussians (emission scan) and
  // the frame-wide range of the visible depth bits
  uint32_t s = cnt;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    kmin = min(kmin, (uint32_t)__shfl_xor(kmin, off, 64));
    kmax = max(kmax, (uint32_t)__shfl_xor(kmax, off, 64));
  }
  const uint32_t vis = (uint32_t)__popcll(__ballot(cnt > 0));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    wave_min[wave] = kmin;
    wave_max[wave] = kmax;
    wave_sums[0][wave] = s;
    wave_sums[1][wave] = vis;
  }
  __syncthreads();
  {
    // the records of the block's 256 virtual gaussians (zero where culled)
    float4* __restrict__ dst =
        reinterpret_cast<float4*>(rec + (view * views.n_pad + blk * kProjBlock));
#pragma unroll
    for (int k = 0; k < 3; ++k) dst[threadIdx.x + k * kProjBlock] = rec_stage[threadIdx.x + k * kProjBlock];
  }
  if (threadIdx.x == 1) {
    uint32_t tp = 0, tv = 0;
#pragma unroll
    for (int w = 0; w < kProjBlock / 64; ++w) {
      tp += wave_sums[0][w];
      tv += wave_sums[1][w];
    }
    const int64_t vb = view * (views.n_pad / kProjBlock) + blk;  // virtual block
    block_sums[2 * vb] = tp;
    block_sums[2 * vb + 1] = tv;
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < kProjBlock / 64; ++w) {
      kmin = min(kmin, wave_min[w]);
      kmax = max(kmax, wave_max[w]);
    }
    // only blocks that widen the range so far touch the shared words: with
    // gaussians in random order that is a few dozen of them, not every block
    if (kmin <= kmax) {
      if (kmin < __hip_atomic_load(&dc->key_min, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin(&dc->key_min, kmin);
      if (kmax > __hip_atomic_load(&dc->key_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&dc->key_max, kmax);
    }
  }
}

hipError_t launch_project(const Views& views, CamArgs shape, ParamArgs prm, float* f_mx,
                          float* f_my, float* f_a, float* f_b, float* f_c, float* f_tau,
                          uint32_t* f_key, uint32_t* f_cnt, uint32_t* f_span, RasterRecord* rec,
                          uint32_t* block_sums, DeviceCounters* dc, bool all_fields,
                          bool sh_packed, hipStream_t s) {
  if (views.n_pad <= 0 || views.count <= 0) return hipSuccess;
  const int64_t blocks = (views.n_pad / kProjBlock) * views.count;
  hipLaunchKernelGGL(project_kernel, dim3((unsigned)blocks), dim3(kProjBlock), 0, s, views, shape,
                     prm, f_mx, f_my, f_a, f_b, f_c, f_tau, f_key, f_cnt, f_span, rec, block_sums,
                     dc, all_fields, sh_packed);
  return hipGetLastError();
}

}  // namespace higs
