// Pieces shared by the forward rasteriser and its adjoint: the LDS image of
// one (macro-tile, batch) processing unit, the conservative gaussian-tile
// test, the staging of a unit (records gathered into LDS, per-tile gaussian
// masks by ballot transpose, queue of active tiles) and the per-pixel alpha,
// so that both kernels evaluate exactly the same float32 expression.
#pragma once
#include "higs_internal.h"

namespace higs {

constexpr int kMiniBatches = kMaxBatch / 64;  // 16
constexpr float kSqrtHalfLog2e = 0.8493218002880191f;  // sqrt(log2(e) / 2)
constexpr float kAlphaMin = 1.0f / 255.0f;
typedef float v4f __attribute__((ext_vector_type(4)));

struct RasterLds {
  float4 ga[kMaxBatch];  // c0 = l0' mx + l1' my, c1 = l2' my, l0', l1' (mx, my macro-tile relative)
  float4 gb[kMaxBatch];  // l2', log2 o, r, g
  float4 gc[kMaxBatch];  // b, o, mx, my (the stride of ga and gb: one address for all reads)
  uint64_t masks[kMiniBatches][kTilesPerMt];
  uint32_t queue[kTilesPerMt];
  uint32_t qcount;
  uint32_t qnext;
  uint32_t unit;
  // per render tile along a chain of batches: 0 = no product stored yet,
  // 1 = product of T stored, 2 = product below t_eps at every pixel
  uint32_t tstate[kTilesPerMt];
};

// Conservative test of one gaussian against the macro-tile's render tiles:
// bit (r * 8 + c) is set when the ellipse {q <= tau'} (tau' slightly above
// tau) reaches the pixel-centre rectangle of tile (c, r).  Per tile row the
// ellipse's x-extent over the row's centre range uses the branches
// x = (-l1 dy +- sqrt(tau' - (l2 dy)^2)) / l0 and their extremal points.
__device__ __forceinline__ uint32_t tile_overlap(float mx, float my, float l0, float l1, float l2,
                                                 float tau, int tiles_x, int tiles_y) {
  const float taum = tau * 1.01f + 0.01f;
  // the hardware square root, reciprocal and reciprocal square root (about
  // one ulp each) instead of correctly rounded sequences, and reciprocals
  // once per gaussian instead of divisions per tile row: these relative
  // errors of ~1e-7 are far inside the margin on tau
  const float st = __builtin_amdgcn_sqrtf(taum);
  const float inv_l0 = __builtin_amdgcn_rcpf(l0), inv_l2 = __builtin_amdgcn_rcpf(l2);
  const float ry = st * inv_l2;
  const float dys = -l1 * ry * __builtin_amdgcn_rsqf(l1 * l1 + l2 * l2);
  uint32_t mask = 0;
  for (int r = 0; r < tiles_y; ++r) {
    const float ya = (float)(r * kTile) + 0.5f - my;
    const float yb = (float)(r * kTile) + 7.5f - my;
    const float dlo = fmaxf(ya, -ry), dhi = fminf(yb, ry);
    if (!(dlo <= dhi)) continue;
    const float yp = fminf(fmaxf(dys, dlo), dhi);
    const float ym = fminf(fmaxf(-dys, dlo), dhi);
    const float sp = __builtin_amdgcn_sqrtf(fmaxf(0.0f, taum - (l2 * yp) * (l2 * yp)));
    const float sm = __builtin_amdgcn_sqrtf(fmaxf(0.0f, taum - (l2 * ym) * (l2 * ym)));
    const float xp = mx + (sp - l1 * yp) * inv_l0 + 0.5f;
    const float xm = mx - (sm + l1 * ym) * inv_l0 - 0.5f;
    // tile c spans pixel centres [8c + 0.5, 8c + 7.5]
    const float flo = fminf(fmaxf(ceilf((xm - 7.5f) * 0.125f), 0.0f), 8.0f);
    const float fhi = fminf(fmaxf(floorf((xp - 0.5f) * 0.125f), -1.0f), (float)(tiles_x - 1));
    const int clo = (int)flo, chi = (int)fhi;
    if (clo <= chi) mask |= ((0xffu >> (7 - (chi - clo))) << clo) << (r * 8);
  }
  return mask;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// alpha = min(alpha_max, o exp(-q/2)) at the pixel centre (pxr, pyr)
// relative to the macro-tile, from the prescaled factors in LDS:
// q' = u^2 + v^2 = q log2(e)/2 with u = l0' dx + l1' dy, v = l2' dy, formed as
// u = l0' pxr + l1' pyr - c0 and v = l2' pyr - c1 (three fused multiply-adds
// per pixel, no differences), and with the stored lo = log2(o),
// o exp(-q/2) = exp2(lo - q') (the opacity rides in the exponent).  e is that
// unclamped alpha.
struct PixelEval {
  float u, v, e, al;
};
__device__ __forceinline__ PixelEval eval_alpha(const float4& A, const float4& B, float lo,
                                                float pxr, float pyr, float amax) {
  PixelEval r;
  r.u = fmaf(A.z, pxr, fmaf(A.w, pyr, -A.x));
  r.v = fmaf(B.x, pyr, -A.y);
  r.e = __builtin_amdgcn_exp2f(fmaf(-r.u, r.u, fmaf(-r.v, r.v, lo)));
  r.al = fminf(amax, r.e);
  return r;
}

struct UnitInfo {
  uint32_t mt, start;
  int len, K, x0, y0, tiles_x, tiles_y;
};

// The macro-tile's pixel origin in its view and its render tiles inside the
// image (a frame of several views numbers the macro-tiles of view v after
// those of views 0 .. v-1: the position is the local number's).
__device__ __forceinline__ void mt_place(const CamArgs& cam, UnitInfo& I) {
  const uint32_t mtl = I.mt % (uint32_t)(cam.n_mt_x * cam.n_mt_y);
  const int mtx = (int)(mtl % (uint32_t)cam.n_mt_x), mty = (int)(mtl / (uint32_t)cam.n_mt_x);
  I.x0 = mtx * kMtW;
  I.y0 = mty * kMtH;
  I.tiles_x = min(kMtTilesX, (cam.width - I.x0 + kTile - 1) / kTile);
  I.tiles_y = min(kMtTilesY, (cam.height - I.y0 + kTile - 1) / kTile);
}

__device__ __forceinline__ UnitInfo unit_info(const CamArgs& cam, const uint32_t* batch_tab,
                                              uint32_t u) {
  UnitInfo I;
  I.mt = batch_tab[3 * u + 0];
  I.start = batch_tab[3 * u + 1];
  I.len = (int)batch_tab[3 * u + 2];
  mt_place(cam, I);
  I.K = (I.len + 63) >> 6;
  return I;
}

// Phase 1 of a unit, by all waves of the workgroup: wave w takes mini-batches
// k = w, w + n_waves, ... (64 gaussians, one per lane), gathers the 48-byte
// records by sorted id into LDS (macro-tile-relative, factors prescaled),
// tests each gaussian against the render tiles and transposes the 32-bit
// per-gaussian tile masks into 64-bit per-tile gaussian masks (a butterfly
// bit-matrix transpose).  Then wave 0 builds the queue of tiles with any
// gaussian, leaving out the tiles of `skip`, and returns their mask (in lane 0
// of wave 0).  Ends with a barrier.
template <int kWavesPerGroup>
__device__ __forceinline__ uint32_t stage_unit(RasterLds& L, const UnitInfo& I,
                                               const uint32_t* __restrict__ sorted,
                                               const RasterRecord* __restrict__ rec, int lane,
                                               int wave, uint32_t skip = 0u) {
  for (int k = wave; k < I.K; k += kWavesPerGroup) {
    const int j = k * 64 + lane;
    uint32_t tmask = 0;
    if (j < I.len) {
      const uint32_t gid = sorted[I.start + j];
      const float4* rp = reinterpret_cast<const float4*>(rec + gid);
      const float4 A = rp[0], B = rp[1], C = rp[2];
      const float mxr = A.x - (float)I.x0, myr = A.y - (float)I.y0;
      const float l0k = A.z * kSqrtHalfLog2e, l1k = A.w * kSqrtHalfLog2e;
      const float l2k = B.x * kSqrtHalfLog2e;
      L.ga[j] = make_float4(fmaf(l0k, mxr, l1k * myr), l2k * myr, l0k, l1k);
      L.gb[j] = make_float4(l2k, __builtin_amdgcn_logf(B.y), B.z, B.w);  // l2', log2 o, r, g
      L.gc[j] = make_float4(C.x, B.y, mxr, myr);                         // b, o, centre
      tmask = tile_overlap(mxr, myr, A.z, A.w, B.x, C.y, I.tiles_x, I.tiles_y);
    }
    // the 64 x 32 bit matrix (lane = gaussian, bit = tile) transposed into
    // 32 per-tile gaussian masks: a 32 x 32 bit transpose inside each half
    // wave in five butterfly stages (stage j swaps the j-bit blocks that sit
    // off the diagonal between lanes l and l ^ j: the partner's word rotated
    // by j into place, then one bit-field insert), then lane t joins its word
    // (gaussians 0..31 on tile t) with lane t + 32's (gaussians 32..63)
    uint32_t x = tmask;
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      const int j = 16 >> s;
      const uint32_t m = s == 0 ? 0x0000FFFFu : s == 1 ? 0x00FF00FFu : s == 2 ? 0x0F0F0F0Fu
                       : s == 3 ? 0x33333333u : 0x55555555u;  // bits whose index has bit j clear
      const bool upper = (lane & j) != 0;
      const uint32_t y = (uint32_t)__shfl_xor((int)x, j, 64);
      const uint32_t ys = __builtin_amdgcn_alignbit(y, y, upper ? j : 32 - j);  // rotate right
      const uint32_t keep = upper ? ~m : m;
      x = (x & keep) | (ys & ~keep);
    }
    const uint32_t x_hi = (uint32_t)__shfl_xor((int)x, 32, 64);
    if (lane < kTilesPerMt) L.masks[k][lane] = ((uint64_t)x_hi << 32) | x;
  }
  __syncthreads();
  uint32_t act32 = 0;
  if (wave == 0) {
    uint64_t hit = 0;
    if (lane < kTilesPerMt)
      for (int k = 0; k < I.K; ++k) hit |= L.masks[k][lane];
    const bool take = lane < kTilesPerMt && hit != 0 && !((skip >> lane) & 1u);
    const uint64_t act = __ballot(take);
    if (take) L.queue[__popcll(act & ((1ull << lane) - 1ull))] = (uint32_t)lane;
    if (lane == 0) L.qcount = (uint32_t)__popcll(act);
    act32 = (uint32_t)act;
  }
  __syncthreads();
  return act32;
}

// The 64 x 32 bit matrix of a mini-batch (lane = gaussian, bit = tile)
// transposed: lane t < 32 gets tile t's 64-bit gaussian mask (the butterfly of
// stage_unit: a 32 x 32 transpose inside each half wave, then the halves
// joined).  All 64 lanes take part.
__device__ __forceinline__ uint64_t transpose_tile_masks(uint32_t tmask, int lane) {
  uint32_t x = tmask;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const int j = 16 >> s;
    const uint32_t m = s == 0 ? 0x0000FFFFu : s == 1 ? 0x00FF00FFu : s == 2 ? 0x0F0F0F0Fu
                     : s == 3 ? 0x33333333u : 0x55555555u;
    const bool upper = (lane & j) != 0;
    const uint32_t y = (uint32_t)__shfl_xor((int)x, j, 64);
    const uint32_t ys = __builtin_amdgcn_alignbit(y, y, upper ? j : 32 - j);
    const uint32_t keep = upper ? ~m : m;
    x = (x & keep) | (ys & ~keep);
  }
  const uint32_t x_hi = (uint32_t)__shfl_xor((int)x, 32, 64);
  return ((uint64_t)x_hi << 32) | x;
}

// Next tile of the unit's queue for this wave (uniform), or -1.
__device__ __forceinline__ int next_tile(RasterLds& L, int lane) {
  uint32_t qi = 0;
  if (lane == 0) qi = atomicAdd(&L.qnext, 1u);
  qi = __builtin_amdgcn_readfirstlane(qi);
  return qi < L.qcount ? (int)L.queue[qi] : -1;
}

}  // namespace higs
