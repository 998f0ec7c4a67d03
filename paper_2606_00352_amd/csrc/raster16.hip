// Half-precision rasteriser and merge (sec. 3.5 "Numerical representation",
// sec. 4.5 "Numerical format"): the reduced-precision mode of the frame path,
// selected by higs_params.raster_precision = HIGS_RASTER_FP16.
//
// The unit is staged as in the float32 kernel (the same records, tile test and
// mask transpose, raster_common.h), but each gaussian's LDS image is
// ten halves: the Cholesky factors prescaled by sqrt(log2(e)/2) (so that
// o exp(-q/2) = exp2(log2 o - q') is one half-precision exp2), c0 = l0' mx +
// l1' my and c1 = l2' my with the centre relative to the macro-tile centre
// (every coordinate within a few hundred pixels at most, far inside the half
// range; q' = u^2 + v^2 is a sum of squares, so rounding cannot make it
// negative), log2 o, and the colour.  A wave blends two vertically adjacent
// render tiles at once, one pixel of each per lane, as half2 pairs: u, v and
// the exponent are three packed fused multiply-adds and two more, the alpha
// threshold 1/255 is a clamped fused multiply-add on the exponent, and the
// colour and transmittance are packed accumulators.  As in the paper, the
// transmittance cut-off is checked per mini-batch of 64 gaussians (the wave
// leaves the tile pair once every pixel of both tiles is below t_eps) rather
// than per gaussian; pixels keep blending until then.  Partials are stored as
// four halves per pixel (8 bytes), merged in float32 — or, fused (the
// default), folded into the work item's float32 state as the merge folds them.
#include "raster_common.h"

namespace higs {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

constexpr int kR16Threads = 512;
constexpr int kR16Waves = kR16Threads / 64;
constexpr int kPairs = kTilesPerMt / 2;  // tile t with tile t + 8 (the row below)
// alpha >= 1/255 <=> exponent >= -log2(255); the clamped ramp
// t = clamp((E + log2 255) * 2048, 0, 1) is 0 below the threshold and 1 from
// 1/2048 above it (alpha within 0.04% of 1/255)
constexpr float kLog2_255 = 7.994353436858858f;
constexpr float kRamp = 2048.0f;

struct Raster16Lds {
  h4 ga[kMaxBatch];  // l0', l1', l2', log2 o
  h4 gb[kMaxBatch];  // c0, c1, r, g
  h2 gc[kMaxBatch];  // b, -
  uint64_t masks[kMiniBatches][kTilesPerMt];
  uint32_t pqueue[kPairs];
  uint32_t qcount;
  uint32_t qnext;
  uint32_t unit;
};

__device__ __forceinline__ h2 bcast(_Float16 v) { return (h2){v, v}; }

template <bool kCountEvals>
__global__ void __launch_bounds__(kR16Threads)
raster16_kernel(CamArgs cam, ParamArgs prm, const uint32_t* __restrict__ vals0,
                const uint32_t* __restrict__ vals1, const RasterRecord* __restrict__ rec,
                const uint32_t* __restrict__ batch_tab, DeviceCounters* __restrict__ dc,
                h4* __restrict__ partials, uint32_t* __restrict__ active) {
  __shared__ Raster16Lds L;
  if (dc->overflow) return;  // the frame stops at a capacity overflow
  const uint32_t* __restrict__ sorted = dc->sort_final ? vals1 : vals0;
  const uint32_t n_units = dc->n_batches;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float eps = prm.t_eps;
  const _Float16 amax = (_Float16)prm.alpha_max;
  // this lane's pixels, relative to the macro-tile centre (32, 16)
  const float pxo = (float)(lane & 7) + 0.5f - 32.0f, pyo = (float)(lane >> 3) + 0.5f - 16.0f;

  for (;;) {
    if (tid == 0) {
      L.unit = atomicAdd(&dc->raster_next, 1u);
      L.qnext = 0;
    }
    __syncthreads();
    const uint32_t u = L.unit;
    if (u >= n_units) break;
    const UnitInfo I = unit_info(cam, batch_tab, u);

    // Phase 1: gather, half-precision LDS image, tile test, mask transpose
    for (int k = wave; k < I.K; k += kR16Waves) {
      const int j = k * 64 + lane;
      uint32_t tmask = 0;
      if (j < I.len) {
        const uint32_t gid = sorted[I.start + j];
        const float4* rp = reinterpret_cast<const float4*>(rec + gid);
        const float4 A = rp[0], B = rp[1], C = rp[2];
        const float mxr = A.x - (float)I.x0, myr = A.y - (float)I.y0;
        const float cx = mxr - 32.0f, cy = myr - 16.0f;
        const float l0k = A.z * kSqrtHalfLog2e, l1k = A.w * kSqrtHalfLog2e;
        const float l2k = B.x * kSqrtHalfLog2e;
        L.ga[j] = (h4){(_Float16)l0k, (_Float16)l1k, (_Float16)l2k,
                       (_Float16)__builtin_amdgcn_logf(B.y)};
        L.gb[j] = (h4){(_Float16)fmaf(l0k, cx, l1k * cy), (_Float16)(l2k * cy), (_Float16)B.z,
                       (_Float16)B.w};
        L.gc[j] = (h2){(_Float16)C.x, (_Float16)0.0f};
        tmask = tile_overlap(mxr, myr, A.z, A.w, B.x, C.y, I.tiles_x, I.tiles_y);
      }
      const uint64_t tm = transpose_tile_masks(tmask, lane);
      if (lane < kTilesPerMt) L.masks[k][lane] = tm;
    }
    __syncthreads();
    // queue of tile pairs (tile t with t + 8) holding any gaussian; active
    // bits: the tiles with gaussians of their own
    uint32_t act = 0;
    if (wave == 0) {
      uint64_t hit = 0;
      if (lane < kTilesPerMt)
        for (int k = 0; k < I.K; ++k) hit |= L.masks[k][lane];
      const uint32_t has = (uint32_t)__ballot(lane < kTilesPerMt && hit != 0);
      const int p = lane & (kPairs - 1);
      const int t0 = (p >> 3) * 16 + (p & 7);
      const bool want = lane < kPairs && (((has >> t0) | (has >> (t0 + 8))) & 1u);
      const uint64_t pm = __ballot(want);
      if (want) L.pqueue[__popcll(pm & ((1ull << lane) - 1ull))] = (uint32_t)p;
      if (lane == 0) L.qcount = (uint32_t)__popcll(pm);
      act = has;
    }
    if (tid == 0) active[u] = act;  // lane 0 of wave 0 holds it
    __syncthreads();

    // Phase 2: waves claim tile pairs
    for (;;) {
      uint32_t qi = 0;
      if (lane == 0) qi = atomicAdd(&L.qnext, 1u);
      qi = __builtin_amdgcn_readfirstlane(qi);
      if (qi >= L.qcount) break;
      const int p = (int)L.pqueue[qi];
      const int t0 = (p >> 3) * 16 + (p & 7), t1 = t0 + 8;
      const float px = (float)((t0 & 7) * kTile) + pxo;
      const float py0 = (float)((t0 >> 3) * kTile) + pyo;
      const h2 PX = bcast((_Float16)px);
      const h2 PY = (h2){(_Float16)py0, (_Float16)(py0 + (float)kTile)};
      const h2 ramp_off = bcast((_Float16)(kLog2_255 * kRamp));
      const h2 ramp = bcast((_Float16)kRamp);
      h2 cr = {0, 0}, cg = {0, 0}, cb = {0, 0}, T = {1, 1};
      uint32_t evals = 0;
      for (int k = 0; k < I.K; ++k) {
        uint64_t m = uniform64(L.masks[k][t0] | L.masks[k][t1]);
        if (kCountEvals) evals += 2u * (uint32_t)__popcll(m);
        while (m) {
          const int j = __ffsll((unsigned long long)m) - 1;
          m &= m - 1ull;
          const int gi = k * 64 + j;
          const h4 A = L.ga[gi];  // l0', l1', l2', log2 o
          const h4 B = L.gb[gi];  // c0, c1, r, g
          const _Float16 bb = L.gc[gi].x;
          // u = l0' px + l1' py - c0, v = l2' py - c1, exponent log2 o - u^2 - v^2
          const h2 U = __builtin_elementwise_fma(bcast(A.x), PX,
                                                 __builtin_elementwise_fma(bcast(A.y), PY, -bcast(B.x)));
          const h2 V = __builtin_elementwise_fma(bcast(A.z), PY, -bcast(B.y));
          const h2 E = __builtin_elementwise_fma(-U, U, __builtin_elementwise_fma(-V, V, bcast(A.w)));
          const h2 e = __builtin_elementwise_exp2(E);
          const h2 al = __builtin_elementwise_min(e, bcast(amax));
          h2 tr = __builtin_elementwise_fma(E, ramp, ramp_off);
          tr = __builtin_elementwise_min(__builtin_elementwise_max(tr, (h2){0, 0}), (h2){1, 1});
          const h2 a = al * tr;
          const h2 w = a * T;
          cr = __builtin_elementwise_fma(w, bcast(B.z), cr);
          cg = __builtin_elementwise_fma(w, bcast(B.w), cg);
          cb = __builtin_elementwise_fma(w, bcast(bb), cb);
          T = __builtin_elementwise_fma(-a, T, T);
        }
        const bool live0 = (float)T.x >= eps, live1 = (float)T.y >= eps;
        if (__ballot(live0 || live1) == 0) break;
      }
      if (kCountEvals && lane == 0) atomicAdd(&dc->n_evals, (unsigned long long)evals);
      const size_t base = (size_t)u * kTilesPerMt;
      partials[(base + t0) * 64 + lane] = (h4){cr.x, cg.x, cb.x, T.x};
      partials[(base + t1) * 64 + lane] = (h4){cr.y, cg.y, cb.y, T.y};
    }
    __syncthreads();
  }
}

constexpr int kMerge16Threads = 256;
__global__ void __launch_bounds__(kMerge16Threads)
merge16_kernel(CamArgs cam, ParamArgs prm, Views views, const uint32_t* __restrict__ batch_first,
               const uint32_t* __restrict__ active, const h4* __restrict__ partials,
               const DeviceCounters* __restrict__ dc) {
  // grid: (tile columns / waves per block, tile rows, views); a wave per tile
  const int tiles_x = (cam.width + kTile - 1) / kTile;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tx = (int)blockIdx.x * (kMerge16Threads / 64) + wave, ty = (int)blockIdx.y;
  const int view = (int)blockIdx.z;
  if (tx >= tiles_x) return;
  const int lane = threadIdx.x & 63;
  const uint32_t mt = (uint32_t)(view * views.n_mt + (ty / kMtTilesY) * cam.n_mt_x + tx / kMtTilesX);
  const uint32_t t = (uint32_t)((ty % kMtTilesY) * kMtTilesX + tx % kMtTilesX);
  const uint32_t nb = dc->overflow ? 0u : dc->n_batches;
  const uint32_t b0 = min(batch_first[mt], nb), b1 = min(batch_first[mt + 1], nb);
  const float eps = prm.t_eps;
  float cr = 0.0f, cg = 0.0f, cb = 0.0f, T = 1.0f;
  bool stop = false;
  for (uint32_t c0 = b0; c0 < b1 && !stop; c0 += 64) {
    const uint32_t bi = c0 + (uint32_t)lane;
    uint64_t m = __ballot(bi < b1 && ((active[bi] >> t) & 1u));
    while (m) {
      const uint32_t b = c0 + (uint32_t)(__ffsll((unsigned long long)m) - 1);
      m &= m - 1ull;
      const h4 p = partials[((size_t)b * kTilesPerMt + t) * 64 + lane];
      if (T >= eps) {
        cr = fmaf(T, (float)p.x, cr);
        cg = fmaf(T, (float)p.y, cg);
        cb = fmaf(T, (float)p.z, cb);
        T = T * (float)p.w;
      }
      if (__ballot(T >= eps) == 0) {
        stop = true;
        break;
      }
    }
  }
  const int x = tx * kTile + (lane & 7), y = ty * kTile + (lane >> 3);
  if (dc->overflow) cr = cg = cb = T = __builtin_nanf("");
  if (x < cam.width && y < cam.height) {
    const ViewArgs& w = views.get(view);
    float* __restrict__ image = w.image;
    float* __restrict__ T_out = w.T;
    const size_t pix = (size_t)y * cam.width + x;
    image[3 * pix + 0] = fmaf(T, w.bg[0], cr);
    image[3 * pix + 1] = fmaf(T, w.bg[1], cg);
    image[3 * pix + 2] = fmaf(T, w.bg[2], cb);
    if (T_out) T_out[pix] = T;
  }
}

// The fused form (fuse_merge = 1): persistent workgroups of 12 waves, two per
// CU (80 VGPRs: the blend loop keeps its constants in registers; 16 waves at
// 64 VGPRs measured 2% slower), take work items of whole macro-tiles as the
// float32 kernel does, stage
// each batch as above, and fold each tile pair's half-precision partials into
// the item's float32 (C, T_acc) per pixel with merge16's operations in its
// order, leaving out a pair once both tiles are below t_eps at every pixel;
// at the item's end they write the macro-tile's pixels.
constexpr int kR16FThreads = 768;
constexpr int kR16FWaves = kR16FThreads / 64;

struct Raster16FLds {
  Raster16Lds r;
  uint32_t tstate[kTilesPerMt];  // 0 no state yet, 1 state stored, 2 below t_eps everywhere
};

template <bool kCountEvals>
__global__ void __launch_bounds__(kR16FThreads) __attribute__((amdgpu_waves_per_eu(6)))
raster16_fused_kernel(CamArgs cam, ParamArgs prm, Views views, const uint32_t* __restrict__ vals0,
                      const uint32_t* __restrict__ vals1, const RasterRecord* __restrict__ rec,
                      const uint32_t* __restrict__ batch_tab, const uint32_t* __restrict__ chain_tab,
                      DeviceCounters* __restrict__ dc, float4* __restrict__ acc) {
  __shared__ Raster16FLds LF;
  Raster16Lds& L = LF.r;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (dc->overflow) {  // no work items were made: the images say so
    const float nan = __builtin_nanf("");
    const size_t n_px = (size_t)cam.width * cam.height;
    for (int v = 0; v < views.count; ++v) {
      const ViewArgs& w = views.get(v);
      for (size_t p = (size_t)blockIdx.x * kR16FThreads + tid; p < n_px;
           p += (size_t)gridDim.x * kR16FThreads) {
        w.image[3 * p + 0] = nan;
        w.image[3 * p + 1] = nan;
        w.image[3 * p + 2] = nan;
        if (w.T) w.T[p] = nan;
      }
    }
    return;
  }
  const uint32_t* __restrict__ sorted = dc->sort_final ? vals1 : vals0;
  const uint32_t n_items = dc->n_chains;
  const float eps = prm.t_eps;
  const _Float16 amax = (_Float16)prm.alpha_max;
  // this lane's pixels, relative to the macro-tile centre (32, 16)
  const float pxo = (float)(lane & 7) + 0.5f - 32.0f, pyo = (float)(lane >> 3) + 0.5f - 16.0f;
  float4* __restrict__ my_acc = acc + (size_t)blockIdx.x * kTilesPerMt * 64;
  uint64_t evals_all = 0;

  for (;;) {
    if (tid == 0) L.unit = atomicAdd(&dc->raster_next, 1u);
    if (tid < kTilesPerMt) LF.tstate[tid] = 0u;
    __syncthreads();
    const uint32_t ch = L.unit;
    if (ch >= n_items) break;
    UnitInfo M;
    M.mt = chain_tab[3 * ch];
    const uint32_t u0 = chain_tab[3 * ch + 1], n_u = chain_tab[3 * ch + 2];
    mt_place(cam, M);
    uint32_t inside = 0;
    for (int r = 0; r < M.tiles_y; ++r) inside |= (0xffu >> (kMtTilesX - M.tiles_x)) << (r * kMtTilesX);
    for (uint32_t i = 0; i < n_u; ++i) {
      const uint32_t u = u0 + i;
      const UnitInfo I = unit_info(cam, batch_tab, u);
      const uint32_t sat = (uint32_t)__ballot(lane < kTilesPerMt && LF.tstate[lane & (kTilesPerMt - 1)] == 2u);
      if ((sat & inside) == inside) continue;  // the merge reads nothing of this unit
      if (tid == 0) L.qnext = 0;

      // Phase 1: gather, half-precision LDS image, tile test, mask transpose
      for (int k = wave; k < I.K; k += kR16FWaves) {
        const int j = k * 64 + lane;
        uint32_t tmask = 0;
        if (j < I.len) {
          const uint32_t gid = sorted[I.start + j];
          const float4* rp = reinterpret_cast<const float4*>(rec + gid);
          const float4 A = rp[0], B = rp[1], C = rp[2];
          const float mxr = A.x - (float)I.x0, myr = A.y - (float)I.y0;
          const float cx = mxr - 32.0f, cy = myr - 16.0f;
          const float l0k = A.z * kSqrtHalfLog2e, l1k = A.w * kSqrtHalfLog2e;
          const float l2k = B.x * kSqrtHalfLog2e;
          L.ga[j] = (h4){(_Float16)l0k, (_Float16)l1k, (_Float16)l2k,
                         (_Float16)__builtin_amdgcn_logf(B.y)};
          L.gb[j] = (h4){(_Float16)fmaf(l0k, cx, l1k * cy), (_Float16)(l2k * cy), (_Float16)B.z,
                         (_Float16)B.w};
          L.gc[j] = (h2){(_Float16)C.x, (_Float16)0.0f};
          tmask = tile_overlap(mxr, myr, A.z, A.w, B.x, C.y, I.tiles_x, I.tiles_y);
        }
        const uint64_t tm = transpose_tile_masks(tmask, lane);
        if (lane < kTilesPerMt) L.masks[k][lane] = tm;
      }
      __syncthreads();
      // queue of tile pairs (tile t with t + 8) holding any gaussian, but
      // not those whose two tiles are both below t_eps or outside the image
      const uint32_t done = sat | ~inside;
      if (wave == 0) {
        uint64_t hit = 0;
        if (lane < kTilesPerMt)
          for (int k = 0; k < I.K; ++k) hit |= L.masks[k][lane];
        const uint32_t has = (uint32_t)__ballot(lane < kTilesPerMt && hit != 0);
        const int p = lane & (kPairs - 1);
        const int t0 = (p >> 3) * 16 + (p & 7);
        const bool want = lane < kPairs && (((has >> t0) | (has >> (t0 + 8))) & 1u) &&
                          !((done >> t0) & (done >> (t0 + 8)) & 1u);
        const uint64_t pm = __ballot(want);
        if (want) L.pqueue[__popcll(pm & ((1ull << lane) - 1ull))] = (uint32_t)p;
        if (lane == 0) L.qcount = (uint32_t)__popcll(pm);
      }
      __syncthreads();

      // Phase 2: waves claim tile pairs
      for (;;) {
        uint32_t qi = 0;
        if (lane == 0) qi = atomicAdd(&L.qnext, 1u);
        qi = __builtin_amdgcn_readfirstlane(qi);
        if (qi >= L.qcount) break;
        const int p = (int)L.pqueue[qi];
        const int t0 = (p >> 3) * 16 + (p & 7), t1 = t0 + 8;
        const float px = (float)((t0 & 7) * kTile) + pxo;
        const float py0 = (float)((t0 >> 3) * kTile) + pyo;
        const h2 PX = bcast((_Float16)px);
        const h2 PY = (h2){(_Float16)py0, (_Float16)(py0 + (float)kTile)};
        const h2 ramp_off = bcast((_Float16)(kLog2_255 * kRamp));
        const h2 ramp = bcast((_Float16)kRamp);
        h2 cr = {0, 0}, cg = {0, 0}, cb = {0, 0}, T = {1, 1};
        for (int k = 0; k < I.K; ++k) {
          uint64_t m = uniform64(L.masks[k][t0] | L.masks[k][t1]);
          if (kCountEvals) evals_all += 2u * (uint32_t)__popcll(m);
          while (m) {
            const int j = __ffsll((unsigned long long)m) - 1;
            m &= m - 1ull;
            const int gi = k * 64 + j;
            const h4 A = L.ga[gi];  // l0', l1', l2', log2 o
            const h4 B = L.gb[gi];  // c0, c1, r, g
            const _Float16 bb = L.gc[gi].x;
            const h2 U = __builtin_elementwise_fma(bcast(A.x), PX,
                                                   __builtin_elementwise_fma(bcast(A.y), PY, -bcast(B.x)));
            const h2 V = __builtin_elementwise_fma(bcast(A.z), PY, -bcast(B.y));
            const h2 E = __builtin_elementwise_fma(-U, U, __builtin_elementwise_fma(-V, V, bcast(A.w)));
            const h2 e = __builtin_elementwise_exp2(E);
            const h2 al = __builtin_elementwise_min(e, bcast(amax));
            h2 tr = __builtin_elementwise_fma(E, ramp, ramp_off);
            tr = __builtin_elementwise_min(__builtin_elementwise_max(tr, (h2){0, 0}), (h2){1, 1});
            const h2 a = al * tr;
            const h2 w = a * T;
            cr = __builtin_elementwise_fma(w, bcast(B.z), cr);
            cg = __builtin_elementwise_fma(w, bcast(B.w), cg);
            cb = __builtin_elementwise_fma(w, bcast(bb), cb);
            T = __builtin_elementwise_fma(-a, T, T);
          }
          const bool live0 = (float)T.x >= eps, live1 = (float)T.y >= eps;
          if (__ballot(live0 || live1) == 0) break;
        }
        // merge16's step for each tile's half-precision partial (a tile
        // without gaussians in this batch has the identity partial); every
        // lane stores the same state words (no lane-0 branch in this loop)
        const uint32_t st0 = LF.tstate[t0], st1 = LF.tstate[t1];
        float4* __restrict__ pa0 = my_acc + t0 * 64 + lane;
        float4* __restrict__ pa1 = my_acc + t1 * 64 + lane;
        float4 s0 = st0 == 0u ? make_float4(0.0f, 0.0f, 0.0f, 1.0f) : *pa0;
        float4 s1 = st1 == 0u ? make_float4(0.0f, 0.0f, 0.0f, 1.0f) : *pa1;
        if (s0.w >= eps) {
          s0.x = fmaf(s0.w, (float)cr.x, s0.x);
          s0.y = fmaf(s0.w, (float)cg.x, s0.y);
          s0.z = fmaf(s0.w, (float)cb.x, s0.z);
          s0.w = s0.w * (float)T.x;
        }
        if (s1.w >= eps) {
          s1.x = fmaf(s1.w, (float)cr.y, s1.x);
          s1.y = fmaf(s1.w, (float)cg.y, s1.y);
          s1.z = fmaf(s1.w, (float)cb.y, s1.z);
          s1.w = s1.w * (float)T.y;
        }
        *pa0 = s0;
        *pa1 = s1;
        LF.tstate[t0] = __ballot(s0.w >= eps) == 0ull ? 2u : 1u;
        LF.tstate[t1] = __ballot(s1.w >= eps) == 0ull ? 2u : 1u;
      }
      __syncthreads();
    }
    // the item's pixels: C + T_acc * background and T_acc, as merge16 writes them
    const ViewArgs& w = views.get((int)(M.mt / (uint32_t)views.n_mt));
    for (int t = wave; t < kTilesPerMt; t += kR16FWaves) {
      const int x = M.x0 + (t & 7) * kTile + (lane & 7), y = M.y0 + (t >> 3) * kTile + (lane >> 3);
      const float4 s = LF.tstate[t] == 0u ? make_float4(0.0f, 0.0f, 0.0f, 1.0f) : my_acc[t * 64 + lane];
      if (x < cam.width && y < cam.height) {
        const size_t pix = (size_t)y * cam.width + x;
        w.image[3 * pix + 0] = fmaf(s.w, w.bg[0], s.x);
        w.image[3 * pix + 1] = fmaf(s.w, w.bg[1], s.y);
        w.image[3 * pix + 2] = fmaf(s.w, w.bg[2], s.z);
        if (w.T) w.T[pix] = s.w;
      }
    }
    // no wave may still read the tile states when the next item resets them
    __syncthreads();
  }
  if (kCountEvals && lane == 0) atomicAdd(&dc->n_evals, (unsigned long long)evals_all);
}

static int g_r16f_per_cu = 0;

hipError_t launch_raster16_fused(CamArgs cam, ParamArgs prm, const Views& views,
                                 const uint32_t* const* vals2, const RasterRecord* rec,
                                 const uint32_t* batch_tab, const uint32_t* chain_tab,
                                 DeviceCounters* dc, float4* acc, int n_cus, bool count_evals,
                                 hipStream_t s) {
  if (g_r16f_per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, raster16_fused_kernel<false>, kR16FThreads,
                                                     0) != hipSuccess ||
        nb < 1)
      nb = 1;
    g_r16f_per_cu = nb;
  }
  const int grid = min(n_cus * g_r16f_per_cu, kMaxRasterWorkers);
  if (count_evals)
    hipLaunchKernelGGL(raster16_fused_kernel<true>, dim3(grid), dim3(kR16FThreads), 0, s, cam, prm,
                       views, vals2[0], vals2[1], rec, batch_tab, chain_tab, dc, acc);
  else
    hipLaunchKernelGGL(raster16_fused_kernel<false>, dim3(grid), dim3(kR16FThreads), 0, s, cam, prm,
                       views, vals2[0], vals2[1], rec, batch_tab, chain_tab, dc, acc);
  return hipGetLastError();
}

static int g_r16_per_cu = 0;

int raster16_per_cu_config() {
  if (g_r16_per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, raster16_kernel<false>, kR16Threads, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    g_r16_per_cu = nb;
  }
  return g_r16_per_cu;
}

hipError_t launch_raster16(CamArgs cam, ParamArgs prm, const uint32_t* const* vals2,
                           const RasterRecord* rec, const uint32_t* batch_tab, DeviceCounters* dc,
                           void* partials, uint32_t* active, int n_cus, bool count_evals,
                           hipStream_t s) {
  raster16_per_cu_config();
  h4* p = static_cast<h4*>(partials);
  if (count_evals)
    hipLaunchKernelGGL(raster16_kernel<true>, dim3(n_cus * g_r16_per_cu), dim3(kR16Threads), 0, s,
                       cam, prm, vals2[0], vals2[1], rec, batch_tab, dc, p, active);
  else
    hipLaunchKernelGGL(raster16_kernel<false>, dim3(n_cus * g_r16_per_cu), dim3(kR16Threads), 0, s,
                       cam, prm, vals2[0], vals2[1], rec, batch_tab, dc, p, active);
  return hipGetLastError();
}

hipError_t launch_merge16(CamArgs cam, ParamArgs prm, const Views& views,
                          const uint32_t* batch_first, const uint32_t* active, const void* partials,
                          const DeviceCounters* dc, hipStream_t s) {
  const int tiles_x = (cam.width + kTile - 1) / kTile, tiles_y = (cam.height + kTile - 1) / kTile;
  const dim3 grid((tiles_x + kMerge16Threads / 64 - 1) / (kMerge16Threads / 64), tiles_y, views.count);
  if (tiles_x == 0 || tiles_y == 0 || views.count == 0) return hipSuccess;
  hipLaunchKernelGGL(merge16_kernel, grid, dim3(kMerge16Threads), 0, s, cam, prm, views,
                     batch_first, active, static_cast<const h4*>(partials), dc);
  return hipGetLastError();
}

}  // namespace higs
