// The 32-byte SH representation (layout in shcodec.hip): constants and the
// inline decoder the projection uses.
#pragma once
#include "higs_internal.h"

namespace higs {

constexpr int kShBases = 16;              // degree 3
constexpr int kShComps = 3 * kShBases;    // Y, Co, Cg per basis
constexpr int kShHeaderBytes = 256;       // 48 float32 scales, padded
constexpr int kDcBitsY = 12, kDcBitsC = 10;
constexpr int kAcBitsY = 6, kAcBitsC = 4;
constexpr int kAcBits = kAcBitsY + 2 * kAcBitsC;  // 14 bits per higher basis
constexpr double kShPercentile = 0.999;   // scale = this quantile of |component|

// Component value of a stored code: x = y |y| with y = (code - M) / M, times the scale.
__device__ __forceinline__ float dequantise(uint32_t code, int bits, float scale) {
  const float m = (float)((1 << (bits - 1)) - 1);
  const float y = ((float)code - m) / m;
  return y * fabsf(y) * scale;
}

// RGB of YCoCg (the inverse of Y = (R + 2G + B) / 4, Co = (R - B) / 2,
// Cg = (-R + 2G - B) / 4).
__device__ __forceinline__ float3 from_ycocg(float y, float co, float cg) {
  return make_float3(y + co - cg, y + cg, y - co - cg);
}

// Coefficient k (RGB) of a gaussian from its 8 packed words and the 48 scales.
__device__ __forceinline__ float3 sh_unpack(const uint32_t w[8], const float* s, int k) {
  if (k == 0) {
    const uint32_t v = w[0];
    return from_ycocg(dequantise(v & ((1u << kDcBitsY) - 1u), kDcBitsY, s[0]),
                      dequantise((v >> kDcBitsY) & ((1u << kDcBitsC) - 1u), kDcBitsC, s[1]),
                      dequantise(v >> (kDcBitsY + kDcBitsC), kDcBitsC, s[2]));
  }
  const int bit = kAcBits * (k - 1);
  const int wi = 1 + (bit >> 5), sh = bit & 31;
  uint32_t v = w[wi] >> sh;
  if (sh + kAcBits > 32) v |= w[wi + 1] << (32 - sh);
  return from_ycocg(dequantise(v & ((1u << kAcBitsY) - 1u), kAcBitsY, s[3 * k]),
                    dequantise((v >> kAcBitsY) & ((1u << kAcBitsC) - 1u), kAcBitsC, s[3 * k + 1]),
                    dequantise((v >> (kAcBitsY + kAcBitsC)) & ((1u << kAcBitsC) - 1u), kAcBitsC,
                               s[3 * k + 2]));
}

hipError_t launch_sh_compress(int64_t n, const float* sh, const float* opac, void* packed,
                              uint32_t* work, int n_cus, hipStream_t s);

}  // namespace higs
