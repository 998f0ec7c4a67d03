// 32-byte SH representation (sec. 4.2, the optional packed SH front end):
// per gaussian and SH basis the RGB coefficients go to YCoCg (luma and two
// chroma differences), each component is scaled by a per-basis, per-component
// factor (a high percentile of its magnitude over the gaussians that can be
// visible, opacity >= 1/255), passed through a square-root gamma and quantised.
// The paper fixes 6 bits of luma and 4 of chroma; the 32 bytes of a degree-3
// gaussian then hold the 15 higher bases (15 x 14 = 210 bits) and leave 46
// bits, which carry the DC basis at 12/10/10 bits (its error would otherwise
// dominate the colour).
//
// Layout of the packed buffer (higs_sh_packed_bytes): a 256-byte header of 48
// float32 scales (basis-major: Y, Co, Cg), then 8 words per gaussian:
//   word 0:     DC  Y (12 bits) | Co (10) << 12 | Cg (10) << 22
//   words 1..7: a 224-bit stream, basis k (1..15) at bit 14 (k - 1):
//               Y (6) | Co (4) << 6 | Cg (4) << 10
// A component c with b bits is stored as rint(sgn(x) sqrt|x| * M) + M,
// M = 2^(b-1) - 1, x = clamp(c / scale, -1, 1); decoding gives
// x = y |y|, y = (stored - M) / M.
//
// Encoding runs once per scene: the per-component maxima, a 1024-bin
// histogram of magnitudes under each maximum, the percentile bin, then the
// packing.  Decoding is inline in the projection (shcodec.h).
#include "shcodec.h"

namespace higs {

constexpr int kCodecBlock = 256;
constexpr int kCodecBins = 1024;

__global__ void shc_zero_kernel(uint32_t* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__device__ __forceinline__ void to_ycocg(float r, float g, float b, float out[3]) {
  out[0] = 0.25f * r + 0.5f * g + 0.25f * b;  // Y
  out[1] = 0.5f * r - 0.5f * b;               // Co
  out[2] = -0.25f * r + 0.5f * g - 0.25f * b; // Cg
}

// Pass 1: the largest magnitude of every (basis, component) over the
// gaussians with opacity >= 1/255 (as float bits: non-negative floats order
// like their bits).
__global__ void __launch_bounds__(kCodecBlock)
shc_max_kernel(int64_t n, const float* __restrict__ sh, const float* __restrict__ opac,
               uint32_t* __restrict__ maxbits) {
  __shared__ uint32_t m[kShComps];
  for (int k = threadIdx.x; k < kShComps; k += kCodecBlock) m[k] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kCodecBlock;
  for (int64_t i = (int64_t)blockIdx.x * kCodecBlock + threadIdx.x; i < n; i += stride) {
    if (!(opac[i] * 255.0f >= 1.0f)) continue;
    for (int k = 0; k < kShBases; ++k) {
      float c[3];
      to_ycocg(sh[48 * i + 3 * k], sh[48 * i + 3 * k + 1], sh[48 * i + 3 * k + 2], c);
      for (int q = 0; q < 3; ++q) {
        const float a = fabsf(c[q]);
        if (a == a) atomicMax(&m[3 * k + q], __float_as_uint(a));
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kShComps; k += kCodecBlock)
    if (m[k]) atomicMax(&maxbits[k], m[k]);
}

// Pass 2: histogram of |c| / max in kCodecBins bins per component.
__global__ void __launch_bounds__(kCodecBlock)
shc_hist_kernel(int64_t n, const float* __restrict__ sh, const float* __restrict__ opac,
                const uint32_t* __restrict__ maxbits, uint32_t* __restrict__ hist,
                uint32_t* __restrict__ n_valid) {
  const int64_t stride = (int64_t)gridDim.x * kCodecBlock;
  uint32_t cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * kCodecBlock + threadIdx.x; i < n; i += stride) {
    if (!(opac[i] * 255.0f >= 1.0f)) continue;
    ++cnt;
    for (int k = 0; k < kShBases; ++k) {
      float c[3];
      to_ycocg(sh[48 * i + 3 * k], sh[48 * i + 3 * k + 1], sh[48 * i + 3 * k + 2], c);
      for (int q = 0; q < 3; ++q) {
        const float mx = __uint_as_float(maxbits[3 * k + q]);
        if (!(mx > 0.0f)) continue;
        const float a = fabsf(c[q]);
        int bin = (int)(a / mx * (float)kCodecBins);
        bin = bin < 0 ? 0 : (bin >= kCodecBins ? kCodecBins - 1 : bin);
        atomicAdd(&hist[(3 * k + q) * kCodecBins + bin], 1u);
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(n_valid, cnt);
}

// Pass 3: one wave per component: the scale is the upper edge of the bin in
// which the cumulative count first reaches the percentile.
__global__ void __launch_bounds__(64)
shc_scale_kernel(const uint32_t* __restrict__ maxbits, const uint32_t* __restrict__ hist,
                 const uint32_t* __restrict__ n_valid, float* __restrict__ scales) {
  const int comp = blockIdx.x, lane = threadIdx.x;
  const float mx = __uint_as_float(maxbits[comp]);
  const uint32_t need = (uint32_t)ceil((double)kShPercentile * (double)(*n_valid));
  uint32_t run = 0;
  int found = kCodecBins - 1;
  for (int b0 = 0; b0 < kCodecBins; b0 += 64) {
    uint32_t v = hist[comp * kCodecBins + b0 + lane];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = __shfl_up(v, off, 64);
      if (lane >= off) v += o;
    }
    const uint64_t hit = __ballot(run + v >= need);
    if (hit) {
      found = b0 + __ffsll((unsigned long long)hit) - 1;
      break;
    }
    run += __shfl(v, 63, 64);
  }
  if (lane == 0) {
    const float s = mx * (float)(found + 1) / (float)kCodecBins;
    scales[comp] = s > 0.0f ? s : 1.0f;  // an all-zero component: any scale decodes 0
  }
}

__device__ __forceinline__ uint32_t quantise(float c, float scale, int bits) {
  const float m = (float)((1 << (bits - 1)) - 1);
  float x = c / scale;
  x = fminf(1.0f, fmaxf(-1.0f, x));
  const float y = copysignf(sqrtf(fabsf(x)), x);
  return (uint32_t)(int)(rintf(y * m) + m);
}

// Pass 4: the packed words of every gaussian.
__global__ void __launch_bounds__(kCodecBlock)
shc_pack_kernel(int64_t n, const float* __restrict__ sh, const float* __restrict__ scales,
                uint32_t* __restrict__ words) {
  __shared__ float s[kShComps];
  for (int k = threadIdx.x; k < kShComps; k += kCodecBlock) s[k] = scales[k];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kCodecBlock + threadIdx.x;
  if (i >= n) return;
  uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  float c[3];
  to_ycocg(sh[48 * i], sh[48 * i + 1], sh[48 * i + 2], c);
  w[0] = quantise(c[0], s[0], kDcBitsY) | (quantise(c[1], s[1], kDcBitsC) << kDcBitsY) |
         (quantise(c[2], s[2], kDcBitsC) << (kDcBitsY + kDcBitsC));
  for (int k = 1; k < kShBases; ++k) {
    to_ycocg(sh[48 * i + 3 * k], sh[48 * i + 3 * k + 1], sh[48 * i + 3 * k + 2], c);
    const uint32_t v = quantise(c[0], s[3 * k], kAcBitsY) |
                       (quantise(c[1], s[3 * k + 1], kAcBitsC) << kAcBitsY) |
                       (quantise(c[2], s[3 * k + 2], kAcBitsC) << (kAcBitsY + kAcBitsC));
    const int bit = kAcBits * (k - 1);
    const int wi = 1 + (bit >> 5), sh_ = bit & 31;
    w[wi] |= v << sh_;
    if (sh_ + kAcBits > 32) w[wi + 1] |= v >> (32 - sh_);
  }
  uint4* dst = reinterpret_cast<uint4*>(words + 8 * i);
  dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
  dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

hipError_t launch_sh_compress(int64_t n, const float* sh, const float* opac, void* packed,
                              uint32_t* work, int n_cus, hipStream_t s) {
  // work: [48] maxima, [48][1024] histogram, [1] count (cleared here)
  uint32_t* maxbits = work;
  uint32_t* hist = work + kShComps;
  uint32_t* n_valid = hist + kShComps * kCodecBins;
  const size_t words = kShComps + (size_t)kShComps * kCodecBins + 1;
  hipLaunchKernelGGL(shc_zero_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, work,
                     words);
  float* scales = reinterpret_cast<float*>(packed);
  uint32_t* out = reinterpret_cast<uint32_t*>(static_cast<char*>(packed) + kShHeaderBytes);
  if (n > 0) {
    const int64_t want = (n + kCodecBlock - 1) / kCodecBlock;
    const unsigned grid = (unsigned)(want < 8 * (int64_t)n_cus ? want : 8 * (int64_t)n_cus);
    hipLaunchKernelGGL(shc_max_kernel, dim3(grid), dim3(kCodecBlock), 0, s, n, sh, opac, maxbits);
    hipLaunchKernelGGL(shc_hist_kernel, dim3(grid), dim3(kCodecBlock), 0, s, n, sh, opac, maxbits,
                       hist, n_valid);
  }
  hipLaunchKernelGGL(shc_scale_kernel, dim3(kShComps), dim3(64), 0, s, maxbits, hist, n_valid, scales);
  if (n > 0)
    hipLaunchKernelGGL(shc_pack_kernel, dim3((unsigned)((n + kCodecBlock - 1) / kCodecBlock)),
                       dim3(kCodecBlock), 0, s, n, sh, scales, out);
  return hipGetLastError();
}

}  // namespace higs
