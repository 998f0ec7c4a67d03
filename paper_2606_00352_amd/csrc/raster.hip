// Stage 4: macro-tile rasterisation (sec. 3.4, Algorithms 1 and 2) and the
// post-blend merge of Eq. 1.
//
// raster_kernel: persistent; each workgroup (16 waves) claims work items
// from a device counter: consecutive (macro-tile, batch) processing units of
// one macro-tile, taken in order.  Along an item it keeps per render tile the
// merge's running state, and leaves a tile out of the later units once its
// transmittance is below t_eps at every pixel.  Fused, an item holds all
// batches of its macro-tile and writes the macro-tile's pixels itself (Eq. 1
// folded as the merge folds it); otherwise each unit's partials go to memory
// for merge_kernel.  Per unit:
//   Phase 1 (load + inline visibility): wave w takes mini-batch k = w
//     (64 gaussians each, one per lane), gathers each gaussian's 48-byte record
//     by its sorted id, stores it in LDS in macro-tile-relative pixels with
//     the Cholesky factors prescaled by sqrt(log2(e)/2) (so exp(-q/2) becomes
//     one exp2), and tests it against the 32 render tiles with a conservative
//     per-tile-row ellipse scan.  The per-gaussian 32-bit tile masks become
//     per-tile 64-bit gaussian masks by a butterfly bit-matrix transpose.
//   Queue: wave 0 ORs the masks per tile and compacts the active tiles.
//   Phase 2: waves claim tiles from the queue through an LDS counter; a wave
//     owns one 8x8 tile, one pixel per lane, walks the set bits of the tile's
//     masks in depth order on the scalar unit and blends front to back in
//     float32.  A pixel stops once T < t_eps; the wave leaves the tile once
//     every pixel has stopped.  The partial (C, T) of every active tile is
//     folded into the item's state or streamed out with non-temporal stores
//     (the active-tile mask then goes to a per-unit word).
// merge_kernel: one wave per render tile walks its macro-tile's batches in
//   depth order, reads only active partials, accumulates
//   C += T_acc C_b, T_acc *= T_b while T_acc >= t_eps and writes
//   C + T_acc * background.
#include "raster_common.h"

namespace higs {

// 16 waves per workgroup and two workgroups per CU (the LDS holds two; 64
// VGPRs give the CU's 32 wave slots): a work item's tiles spread over twice
// the waves of an 8-wave workgroup, three of which shared a CU before (1080p
// raster 0.442 -> 0.387 ms: the frame waits on its heaviest items)
constexpr int kRasterThreads = 1024;
constexpr int kRasterWaves = kRasterThreads / 64;

template <bool kCountEvals, bool kFused>
__global__ void __launch_bounds__(kRasterThreads) __attribute__((amdgpu_waves_per_eu(8)))
raster_kernel(CamArgs cam, ParamArgs prm, Views views, const uint32_t* __restrict__ vals0,
              const uint32_t* __restrict__ vals1, const RasterRecord* __restrict__ rec,
              const uint32_t* __restrict__ batch_tab, const uint32_t* __restrict__ chain_tab,
              DeviceCounters* __restrict__ dc, float4* __restrict__ partials,
              uint32_t* __restrict__ active, float4* __restrict__ acc) {
  __shared__ RasterLds L;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (dc->overflow) {  // the frame stops at a capacity overflow
    if (kFused) {      // and no work items were made: the images say so
      const float nan = __builtin_nanf("");
      const size_t n_px = (size_t)cam.width * cam.height;
      for (int v = 0; v < views.count; ++v) {
        const ViewArgs& w = views.get(v);
        for (size_t p = (size_t)blockIdx.x * kRasterThreads + tid; p < n_px;
             p += (size_t)gridDim.x * kRasterThreads) {
          w.image[3 * p + 0] = nan;
          w.image[3 * p + 1] = nan;
          w.image[3 * p + 2] = nan;
          if (w.T) w.T[p] = nan;
        }
      }
    }
    return;
  }
  const uint32_t* __restrict__ sorted = dc->sort_final ? vals1 : vals0;
  const uint32_t n_chains = dc->n_chains;
  const float eps = prm.t_eps, amax = prm.alpha_max;
  const float pxo = (float)(lane & 7) + 0.5f, pyo = (float)(lane >> 3) + 0.5f;
  // this workgroup's running state along a work item, per tile and pixel:
  // fused, the merge's (C, T_acc); otherwise the product of the batches' T
  float4* __restrict__ my_acc = acc + (size_t)blockIdx.x * kTilesPerMt * 64;
  float* __restrict__ my_T = reinterpret_cast<float*>(my_acc);

  uint64_t evals_all = 0;  // this wave's evaluations (the count-evals variant)
  for (;;) {
    if (tid == 0) L.unit = atomicAdd(&dc->raster_next, 1u);
    if (tid < kTilesPerMt) L.tstate[tid] = 0u;
    __syncthreads();
    const uint32_t ch = L.unit;
    if (ch >= n_chains) break;
    UnitInfo M;  // the item's macro-tile
    M.mt = chain_tab[3 * ch];
    const uint32_t u0 = chain_tab[3 * ch + 1], n_u = chain_tab[3 * ch + 2];
    mt_place(cam, M);
    // the render tiles inside the image
    uint32_t inside = 0;
    for (int r = 0; r < M.tiles_y; ++r) inside |= (0xffu >> (kMtTilesX - M.tiles_x)) << (r * kMtTilesX);
    for (uint32_t i = 0; i < n_u; ++i) {
      const uint32_t u = u0 + i;
      const UnitInfo I = unit_info(cam, batch_tab, u);
      // the tiles the item's earlier batches saturated (read after the
      // barrier that ended the last unit)
      const uint32_t sat = (uint32_t)__ballot(lane < kTilesPerMt && L.tstate[lane & (kTilesPerMt - 1)] == 2u);
      if ((sat & inside) == inside) {  // the merge reads nothing of this unit
        if (!kFused && tid == 0) active[u] = 0u;
        continue;
      }
      if (tid == 0) L.qnext = 0;
      const uint32_t act = stage_unit<kRasterWaves>(L, I, sorted, rec, lane, wave, sat);
      if (!kFused && tid == 0) active[u] = act;

      // Phase 2: waves claim tiles
      for (;;) {
        const int t = next_tile(L, lane);
        if (t < 0) break;
        const float pxr = (float)((t & 7) * kTile) + pxo;
        const float pyr = (float)((t >> 3) * kTile) + pyo;
        float cr = 0.0f, cg = 0.0f, cb = 0.0f, T = 1.0f;
        uint32_t evals = 0;
        for (int k = 0; k < I.K; ++k) {
          uint64_t m = uniform64(L.masks[k][t]);
          if (kCountEvals) evals += (uint32_t)__popcll(m);
          while (m) {
            const int j = __ffsll((unsigned long long)m) - 1;
            m &= m - 1ull;
            const int gi = k * 64 + j;
            const float4 A = L.ga[gi];
            const float4 B = L.gb[gi];  // l2', log2 o, r, g
            const float bb = L.gc[gi].x;
            const float al = eval_alpha(A, B, B.y, pxr, pyr, amax).al;
            // branchless blend: a skipped gaussian adds w = 0 and keeps T
            // exactly; T(1 - a) is one fused T - aT, rounded once (the
            // adjoint's replay forms it the same way)
            const float a = (T >= eps && al >= kAlphaMin) ? al : 0.0f;
            const float w = a * T;
            cr += w * B.z;
            cg += w * B.w;
            cb += w * bb;
            T = fmaf(-a, T, T);
          }
          if (__ballot(T >= eps) == 0) break;
        }
        if (kCountEvals) evals_all += evals;
        // Only this wave writes the tile's state in this unit, and every lane
        // stores the same word: no lane-0 branch in this loop, which would
        // let the compiler split the wave around next_tile's readfirstlane.
        const uint32_t st = L.tstate[t];
        if (kFused) {
          // the merge's step for this batch's partial (Eq. 1), its float32
          // operations in its order; a tile without partial in a batch is the
          // identity step, so leaving it out changes nothing
          float4* __restrict__ pa = my_acc + t * 64 + lane;
          float4 s = st == 0u ? make_float4(0.0f, 0.0f, 0.0f, 1.0f) : *pa;
          if (s.w >= eps) {
            s.x = fmaf(s.w, cr, s.x);
            s.y = fmaf(s.w, cg, s.y);
            s.z = fmaf(s.w, cb, s.z);
            s.w = s.w * T;
          }
          *pa = s;
          L.tstate[t] = __ballot(s.w >= eps) == 0ull ? 2u : 1u;
        } else {
          v4f* dst = reinterpret_cast<v4f*>(partials + (((size_t)u * kTilesPerMt + t) * 64 + lane));
          const v4f val = {cr, cg, cb, T};
          __builtin_nontemporal_store(val, dst);
          if (i + 1 < n_u) {
            // the tile's product of T over the item so far, in the order and
            // the float32 arithmetic of the merge: with t_eps reached at
            // every pixel, the merge (whose own product is never larger) has
            // stopped reading this tile, and the item's later batches leave
            // it out
            float* __restrict__ pt = my_T + t * 64 + lane;
            const float prod = st == 0u ? T : *pt * T;
            *pt = prod;
            L.tstate[t] = __ballot(prod >= eps) == 0ull ? 2u : 1u;
          }
        }
      }
      __syncthreads();
    }
    if (kFused) {
      // the item's pixels (all batches of its macro-tile folded): Eq. 1's
      // C + T_acc * background and T_acc, as the merge writes them
      const ViewArgs& w = views.get((int)(M.mt / (uint32_t)views.n_mt));
      for (int t = wave; t < kTilesPerMt; t += kRasterWaves) {
        const int x = M.x0 + (t & 7) * kTile + (lane & 7), y = M.y0 + (t >> 3) * kTile + (lane >> 3);
        const float4 s = L.tstate[t] == 0u ? make_float4(0.0f, 0.0f, 0.0f, 1.0f) : my_acc[t * 64 + lane];
        if (x < cam.width && y < cam.height) {
          const size_t pix = (size_t)y * cam.width + x;
          w.image[3 * pix + 0] = fmaf(s.w, w.bg[0], s.x);
          w.image[3 * pix + 1] = fmaf(s.w, w.bg[1], s.y);
          w.image[3 * pix + 2] = fmaf(s.w, w.bg[2], s.z);
          if (w.T) w.T[pix] = s.w;
        }
      }
    }
    // an item that ended on a left-out unit has not passed the barrier above:
    // no wave may still read the tile states when the next item resets them
    __syncthreads();
  }
  if (kCountEvals && lane == 0) atomicAdd(&dc->n_evals, (unsigned long long)evals_all);
}

constexpr int kMergeThreads = 256;
__global__ void __launch_bounds__(kMergeThreads)
merge_kernel(CamArgs cam, ParamArgs prm, Views views, const uint32_t* __restrict__ batch_first,
             const uint32_t* __restrict__ active, const float4* __restrict__ partials,
             const DeviceCounters* __restrict__ dc) {
  // grid: (tile columns / waves per block, tile rows, views); a wave per tile
  const int tiles_x = (cam.width + kTile - 1) / kTile;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tx = (int)blockIdx.x * (kMergeThreads / 64) + wave, ty = (int)blockIdx.y;
  const int view = (int)blockIdx.z;
  if (tx >= tiles_x) return;
  const int lane = threadIdx.x & 63;
  const uint32_t mt = (uint32_t)(view * views.n_mt + (ty / kMtTilesY) * cam.n_mt_x + tx / kMtTilesX);
  const uint32_t t = (uint32_t)((ty % kMtTilesY) * kMtTilesX + tx % kMtTilesX);
  const uint32_t nb = dc->overflow ? 0u : dc->n_batches;
  const uint32_t b0 = min(batch_first[mt], nb), b1 = min(batch_first[mt + 1], nb);
  const float eps = prm.t_eps;
  float cr = 0.0f, cg = 0.0f, cb = 0.0f, T = 1.0f;
  auto load = [&](uint32_t b) {
    return __builtin_nontemporal_load(
        reinterpret_cast<const v4f*>(partials + (((size_t)b * kTilesPerMt + t) * 64 + lane)));
  };
  // the tile's active batches, 64 at a time (one activity word per lane);
  // the next active partial is loaded before the current one is folded in
  bool stop = false;
  for (uint32_t c0 = b0; c0 < b1 && !stop; c0 += 64) {
    const uint32_t bi = c0 + (uint32_t)lane;
    uint64_t m = __ballot(bi < b1 && ((active[bi] >> t) & 1u));
    if (!m) continue;
    uint32_t b = c0 + (uint32_t)(__ffsll((unsigned long long)m) - 1);
    m &= m - 1ull;
    v4f p = load(b);
    for (;;) {
      const bool more = m != 0ull;
      v4f pn = p;
      if (more) {
        b = c0 + (uint32_t)(__ffsll((unsigned long long)m) - 1);
        m &= m - 1ull;
        pn = load(b);
      }
      if (T >= eps) {
        cr = fmaf(T, p.x, cr);
        cg = fmaf(T, p.y, cg);
        cb = fmaf(T, p.z, cb);
        T = T * p.w;
      }
      if (__ballot(T >= eps) == 0) {
        stop = true;
        break;
      }
      if (!more) break;
      p = pn;
    }
  }
  const int x = tx * kTile + (lane & 7), y = ty * kTile + (lane >> 3);
  if (dc->overflow) {  // no partials were made: the image says so
    cr = cg = cb = T = __builtin_nanf("");
  }
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

static int g_raster_per_cu = 0;

// Resident raster workgroups per CU (queried once; the launchers read it, also
// while a stream is being captured into a graph).
int raster_per_cu_config() {
  if (g_raster_per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, raster_kernel<false, true>, kRasterThreads, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    g_raster_per_cu = nb;
  }
  return g_raster_per_cu;
}

hipError_t launch_raster(CamArgs cam, ParamArgs prm, const Views& views, const uint32_t* const* vals2,
                         const RasterRecord* rec, const uint32_t* batch_tab,
                         const uint32_t* chain_tab, DeviceCounters* dc, float4* partials,
                         uint32_t* active, float4* acc, int n_cus, bool count_evals, bool fused,
                         hipStream_t s) {
  raster_per_cu_config();
  // one running-state slice per workgroup of the grid
  const int grid = min(n_cus * g_raster_per_cu, kMaxRasterWorkers);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kRasterThreads), 0, s, cam, prm, views, vals2[0],
                       vals2[1], rec, batch_tab, chain_tab, dc, partials, active, acc);
  };
  if (count_evals)
    fused ? go(raster_kernel<true, true>) : go(raster_kernel<true, false>);
  else
    fused ? go(raster_kernel<false, true>) : go(raster_kernel<false, false>);
  return hipGetLastError();
}

__global__ void raster_rewind_kernel(DeviceCounters* dc) { dc->raster_next = 0u; }

hipError_t launch_raster_rewind(DeviceCounters* dc, hipStream_t s) {
  hipLaunchKernelGGL(raster_rewind_kernel, dim3(1), dim3(1), 0, s, dc);
  return hipGetLastError();
}

hipError_t launch_merge(CamArgs cam, ParamArgs prm, const Views& views, const uint32_t* batch_first,
                        const uint32_t* active, const float4* partials, const DeviceCounters* dc,
                        hipStream_t s) {
  const int tiles_x = (cam.width + kTile - 1) / kTile, tiles_y = (cam.height + kTile - 1) / kTile;
  const dim3 grid((tiles_x + kMergeThreads / 64 - 1) / (kMergeThreads / 64), tiles_y, views.count);
  if (tiles_x == 0 || tiles_y == 0 || views.count == 0) return hipSuccess;
  hipLaunchKernelGGL(merge_kernel, grid, dim3(kMergeThreads), 0, s, cam, prm, views,
                     batch_first, active, partials, dc);
  return hipGetLastError();
}

int raster_workers_per_cu() { return g_raster_per_cu; }

}  // namespace higs
