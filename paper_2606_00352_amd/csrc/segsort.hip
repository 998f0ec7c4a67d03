// Stages 2-3, segmented form (sec. 3.2 Gaussian partitioning, sec. 3.3
// Segmented depth sort, sec. 4.3 count / scan / fill, sec. 4.4 tiered segment
// sort with an overflow merge): pairs are binned straight into one contiguous
// segment per macro-tile, and every segment is sorted on its own by depth; no
// global composite-key sort.
//
// part_count_kernel (one workgroup per partition batch of B_p = 8,192
//   gaussians): an LDS histogram with one counter per macro-tile, filled from
//   each visible gaussian's macro-tile list (the span word the projection
//   recorded, else the exact predicate again on the stored float32 fields),
//   written out as column b of the count matrix: 16-bit counts, macro-tile
//   major (N_M rows of N_B batches; a batch puts at most 8,192 pairs in one
//   macro-tile).
// part_tile_sum_kernel / part_scan_top_kernel / part_tile_scan_kernel:
//   reduce-then-scan of 4,096-entry tiles: an exclusive scan of the
//   matrix in macro-tile-major order gives every (macro-tile, batch) its first
//   pair slot; the row starts are the segment offsets.  Past the pair capacity
//   the frame stops (offsets clamped, overflow flagged).
// part_plan_kernel (one workgroup): segments by size into the tiers T0-T3
//   of up to 1,024, 2,048, 4,096 and 8,192 pairs (one workgroup sorts the
//   whole segment in LDS: 256, 256, 512 and 1,024 threads), and longer ones,
//   cut into 8,192-pair chunks.
// part_fill_kernel (one workgroup per partition batch): LDS cursors start at
//   the batch's slots in each row; every pair takes the next slot of its
//   macro-tile (LDS atomic) and is written as the composite
//   ((depth bits - min) << g) | id, g = bits of the largest id.  The order
//   inside a (macro-tile, batch) range is whatever the atomics give; sorting
//   composites orders a segment by (depth, id) regardless.
// part_sort_kernel<threads, items, tier> (persistent, one launch per tier):
//   a workgroup loads a segment (or chunk) into registers and sorts it with
//   LSD radix passes of 8-bit digits through LDS over the depth part of the
//   composites, skipping every digit that no composite of the segment
//   changes: per pass, a wave ranks its keys stably with 8 ballots per key
//   against a wave-private digit histogram, then digit and wave prefixes give
//   each key its slot.  Equal depths, adjacent after the passes, are put in
//   id order (a run of up to 64 by one thread; a longer run sends the segment
//   through the passes again over every bit).  A whole segment writes its
//   ids; a chunk writes its sorted run.
// part_merge_kernel (persistent, one launch per level l): the runs of length
//   C * 2^l of each long segment are merged pairwise in 8,192-output blocks,
//   each found by a merge-path search and merged from LDS; a segment whose
//   merge completes writes its ids.  Levels past the frame's longest segment
//   return at once.
// Outputs: the segment offsets (mt_off) and the ids in (macro-tile, depth,
// id) order; the batch stage and the raster read them as in the onesweep
// mode.
#include "higs_internal.h"
#include "predicate.h"

namespace higs {

constexpr int kPartThreads = 1024;
constexpr int kPartPerThread = kSegBatch / kPartThreads;  // gaussians per thread
constexpr int kScanThreads = 256;
constexpr int kScanItems = kSegScanTile / kScanThreads;    // matrix entries per thread
constexpr int kPlanThreads = 1024;
constexpr int kDigitBits = 8;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kTieRun = 64;  // equal depths a thread puts in id order by insertion
static_assert(kScanItems * kScanThreads == kSegScanTile, "whole scan tiles");

// Inclusive scan of one value per lane across a wave.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread (kThreads threads);
// *total gets the sum.  wt: kThreads / 64 words of LDS.
template <int kThreads>
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* wt, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t x = wave_scan_incl(v);
  __syncthreads();
  if (lane == 63) wt[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    before += w < wave ? wt[w] : 0u;
    all += wt[w];
  }
  *total = all;
  return before + x - v;
}

// Each visible gaussian's macro-tile list: the recorded span word, else the
// exact predicate again on the stored float32 fields (identical decisions).
template <class F>
__device__ __forceinline__ void visit_pairs(uint32_t span, int64_t i, const CamArgs& cam,
                                            const float* __restrict__ f_mx,
                                            const float* __restrict__ f_my,
                                            const float* __restrict__ f_a,
                                            const float* __restrict__ f_b,
                                            const float* __restrict__ f_c,
                                            const float* __restrict__ f_tau, F&& fn) {
  if (span) {
    visit_span(span, cam.n_mt_x, fn);
  } else {
    BinFields f;
    f.mx = f_mx[i];
    f.my = f_my[i];
    f.a = f_a[i];
    f.b = f_b[i];
    f.c = f_c[i];
    f.tau = f_tau[i];
    visit_macro_tiles(f, cam.width, cam.height, cam.n_mt_x, cam.n_mt_y, fn);
  }
}

// ------------------------------------------------------------------ count --
__global__ void __launch_bounds__(kPartThreads)
part_count_kernel(int64_t n, CamArgs cam, int n_mt, uint32_t n_b, const float* __restrict__ f_mx,
                  const float* __restrict__ f_my, const float* __restrict__ f_a,
                  const float* __restrict__ f_b, const float* __restrict__ f_c,
                  const float* __restrict__ f_tau, const uint32_t* __restrict__ f_cnt,
                  const uint32_t* __restrict__ f_span, uint16_t* __restrict__ cm,
                  DeviceCounters* __restrict__ dc) {
  HIP_DYNAMIC_SHARED(uint32_t, hist)
  __shared__ uint32_t s_vis;
  for (int m = threadIdx.x; m < n_mt; m += kPartThreads) hist[m] = 0;
  if (threadIdx.x == 0) s_vis = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSegBatch;
  uint32_t cnt[kPartPerThread], span[kPartPerThread];
#pragma unroll
  for (int r = 0; r < kPartPerThread; ++r) {
    const int64_t i = base + (int64_t)r * kPartThreads + threadIdx.x;
    cnt[r] = i < n ? f_cnt[i] : 0u;
    span[r] = i < n ? f_span[i] : 0u;
  }
  uint32_t vis = 0;
  for (int r = 0; r < kPartPerThread; ++r) {
    if (cnt[r] == 0) continue;
    ++vis;
    const int64_t i = base + (int64_t)r * kPartThreads + threadIdx.x;
    visit_pairs(span[r], i, cam, f_mx, f_my, f_a, f_b, f_c, f_tau,
                [&](uint32_t mt) { atomicAdd(&hist[mt], 1u); });
  }
  if (vis) atomicAdd(&s_vis, vis);
  __syncthreads();
  // column b of the macro-tile-major matrix
  const uint32_t b = blockIdx.x;
  for (int m = threadIdx.x; m < n_mt; m += kPartThreads) cm[(size_t)m * n_b + b] = (uint16_t)hist[m];
  if (threadIdx.x == 0 && s_vis) atomicAdd(&dc->n_visible, s_vis);
}

// ------------------------------------------------------------------- scan --
// A workgroup per scan tile: the sum of its matrix entries.
__global__ void __launch_bounds__(kScanThreads)
part_tile_sum_kernel(uint64_t n_entries, const uint16_t* __restrict__ cm,
                     uint32_t* __restrict__ tile_sum) {
  __shared__ uint32_t wt[kScanThreads / 64];
  const uint64_t i0 = (uint64_t)blockIdx.x * kSegScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) sum += i0 + k < n_entries ? (uint32_t)cm[i0 + k] : 0u;
  uint32_t tot;
  (void)block_scan_excl<kScanThreads>(sum, wt, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the tile sums (in place), the pair total,
// the capacity check.
__global__ void __launch_bounds__(kPlanThreads)
part_scan_top_kernel(uint32_t n_tiles, int n_mt, uint32_t n_b, uint32_t max_pairs,
                     uint32_t* __restrict__ tile_sum, uint32_t* __restrict__ mt_off,
                     DeviceCounters* __restrict__ dc) {
  __shared__ uint32_t wt[kPlanThreads / 64];
  uint32_t carry = 0;
  for (uint32_t t0 = 0; t0 < n_tiles; t0 += kPlanThreads) {
    const uint32_t t = t0 + threadIdx.x;
    const uint32_t v = t < n_tiles ? tile_sum[t] : 0u;
    uint32_t tot;
    const uint32_t ex = block_scan_excl<kPlanThreads>(v, wt, &tot);
    if (t < n_tiles) tile_sum[t] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    const bool ovf = carry > max_pairs;
    dc->n_pairs_total = carry;
    dc->n_pairs = ovf ? max_pairs : carry;
    if (ovf) atomicOr(&dc->overflow, (uint32_t)HIGS_OVF_PAIRS);
    dc->sort_final = 0;  // the ids end in the first value buffer
    dc->sort_passes = 0;
    mt_off[n_mt] = ovf ? max_pairs : carry;
  }
  // no partition batches (no gaussians): every segment is empty
  if (n_b == 0)
    for (int m = threadIdx.x; m < n_mt; m += kPlanThreads) mt_off[m] = 0;
}

// A workgroup per scan tile: the exclusive scan of its matrix entries plus
// the tile's base -> the slot of every (macro-tile, batch); a row's first
// entry is its segment offset.
__global__ void __launch_bounds__(kScanThreads)
part_tile_scan_kernel(uint64_t n_entries, uint32_t n_b, uint32_t max_pairs,
                      const uint16_t* __restrict__ cm, const uint32_t* __restrict__ tile_base,
                      uint32_t* __restrict__ off, uint32_t* __restrict__ mt_off) {
  __shared__ uint32_t wt[kScanThreads / 64];
  const uint64_t i0 = (uint64_t)blockIdx.x * kSegScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = i0 + k < n_entries ? (uint32_t)cm[i0 + k] : 0u;
    sum += v[k];
  }
  uint32_t tot;
  uint32_t run = tile_base[blockIdx.x] + block_scan_excl<kScanThreads>(sum, wt, &tot);
  // the (row, column) of the first entry, then stepped along
  uint64_t m = i0 / n_b;
  uint32_t b = (uint32_t)(i0 - m * n_b);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (i0 + k < n_entries) {
      off[i0 + k] = run;
      if (b == 0) mt_off[m] = min(run, max_pairs);
    }
    run += v[k];
    if (++b == n_b) {
      b = 0;
      ++m;
    }
  }
}

// ------------------------------------------------------------------- plan --
// One workgroup: segments by size into the four tiers (lists of macro-tiles
// in order), the chunk table of the long ones, the longest segment.
__global__ void __launch_bounds__(kPlanThreads)
part_plan_kernel(int n_mt, const uint32_t* __restrict__ mt_off, uint32_t* __restrict__ list,
                 DeviceCounters* __restrict__ dc) {
  __shared__ uint32_t wt[kPlanThreads / 64];
  __shared__ uint32_t s_max;
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  const bool ovf = dc->overflow != 0;
  uint32_t base[kSegTiers] = {}, chunks = 0;
  uint32_t* chunk_off = list + (size_t)kSegTiers * n_mt;
  for (int m0 = 0; m0 < n_mt; m0 += kPlanThreads) {
    const int m = m0 + (int)threadIdx.x;
    const uint32_t s = (!ovf && m < n_mt) ? mt_off[m + 1] - mt_off[m] : 0u;
    int tier = s == 0 ? -1 : kSegTiers - 1;
#pragma unroll
    for (int t = kSegTiers - 2; t >= 0; --t)
      if (s && s <= kSegTierCap[t]) tier = t;
    if (s) atomicMax(&s_max, s);
#pragma unroll
    for (int t = 0; t < kSegTiers; ++t) {
      uint32_t tot;
      const uint32_t at = block_scan_excl<kPlanThreads>(tier == t ? 1u : 0u, wt, &tot);
      if (tier == t) list[(size_t)t * n_mt + base[t] + at] = (uint32_t)m;
      if (t == kSegTiers - 1) {
        // chunk table of the long segments, in list order
        uint32_t ctot;
        const uint32_t c = tier == t ? (s + kSegChunk - 1) / kSegChunk : 0u;
        const uint32_t cat = block_scan_excl<kPlanThreads>(c, wt, &ctot);
        if (tier == t) chunk_off[base[t] + at] = chunks + cat;
        chunks += ctot;
      }
      base[t] += tot;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    chunk_off[base[kSegTiers - 1]] = chunks;
#pragma unroll
    for (int t = 0; t < kSegTiers; ++t) dc->seg_tier_n[t] = base[t];
    dc->seg_chunks = chunks;
    dc->seg_max = s_max;
  }
}

// ------------------------------------------------------------------- fill --
__global__ void __launch_bounds__(kPartThreads)
part_fill_kernel(int64_t n, CamArgs cam, int n_mt, uint32_t n_b, uint32_t gbits,
                 const float* __restrict__ f_mx, const float* __restrict__ f_my,
                 const float* __restrict__ f_a, const float* __restrict__ f_b,
                 const float* __restrict__ f_c, const float* __restrict__ f_tau,
                 const uint32_t* __restrict__ f_key, const uint32_t* __restrict__ f_cnt,
                 const uint32_t* __restrict__ f_span, const uint32_t* __restrict__ off,
                 const DeviceCounters* __restrict__ dc, uint32_t max_pairs,
                 uint64_t* __restrict__ comp) {
  HIP_DYNAMIC_SHARED(uint32_t, cur)
  if (dc->overflow) return;  // the frame stops at a capacity overflow
  const uint32_t b = blockIdx.x;
  for (int m = threadIdx.x; m < n_mt; m += kPartThreads) cur[m] = off[(size_t)m * n_b + b];
  __syncthreads();
  const uint32_t dmin = dc->key_min;
  const int64_t base = (int64_t)b * kSegBatch;
  uint32_t cnt[kPartPerThread], span[kPartPerThread], key[kPartPerThread];
#pragma unroll
  for (int r = 0; r < kPartPerThread; ++r) {
    const int64_t i = base + (int64_t)r * kPartThreads + threadIdx.x;
    cnt[r] = i < n ? f_cnt[i] : 0u;
    span[r] = i < n ? f_span[i] : 0u;
    key[r] = i < n ? f_key[i] : 0u;
  }
  for (int r = 0; r < kPartPerThread; ++r) {
    if (cnt[r] == 0) continue;
    const int64_t i = base + (int64_t)r * kPartThreads + threadIdx.x;
    const uint64_t c = ((uint64_t)(key[r] - dmin) << gbits) | (uint64_t)i;
    visit_pairs(span[r], i, cam, f_mx, f_my, f_a, f_b, f_c, f_tau, [&](uint32_t mt) {
      const uint32_t at = atomicAdd(&cur[mt], 1u);
      if (at < max_pairs) comp[at] = c;
    });
  }
}

// ------------------------------------------------------------------- sort --
template <int kThreads, int kItems>
struct PartSortLds {
  uint64_t v[kThreads * kItems];             // one pass's output, in order
  uint32_t whist[kThreads / 64][kDigits];    // per-wave digit counts, then wave prefixes
  uint32_t dstart[kDigits];                  // first slot of each digit
  uint32_t dtot[kDigits / 64];
  unsigned long long diff;                   // OR of (composite ^ first composite)
  uint32_t job;
  uint32_t long_tie;                         // a run of equal depths longer than kTieRun
};

// Segment (or chunk) sort of up to kThreads * kItems composites; tiers 0-2
// take whole segments from their list, tier 3 takes chunks of long segments.
template <int kThreads, int kItems, int kTier>
__global__ void __launch_bounds__(kThreads)
part_sort_kernel(const uint32_t* __restrict__ mt_off, const uint32_t* __restrict__ list,
                 int n_mt, uint32_t gbits, const uint64_t* __restrict__ comp,
                 uint64_t* __restrict__ runs, uint32_t* __restrict__ ids,
                 DeviceCounters* __restrict__ dc) {
  static_assert(kThreads >= kDigits && kThreads % 64 == 0, "a thread per digit, whole waves");
  constexpr int kWaves = kThreads / 64;
  constexpr bool kChunks = kTier == kSegTiers - 1;  // chunks of long segments
  static_assert(kThreads * kItems >= (kChunks ? kSegChunk : (int)kSegTierCap[kChunks ? 0 : kTier]),
                "the tier's segments fit the workgroup");
  __shared__ PartSortLds<kThreads, kItems> L;
  if (dc->overflow) return;
  const uint32_t n_jobs = kChunks ? dc->seg_chunks : dc->seg_tier_n[kTier];
  const uint32_t* __restrict__ mine = list + (size_t)kTier * n_mt;
  const uint32_t* __restrict__ chunk_off = list + (size_t)kSegTiers * n_mt;
  const uint32_t n_long = dc->seg_tier_n[kSegTiers - 1];
  const uint64_t idmask = (1ull << gbits) - 1ull;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  for (;;) {
    if (tid == 0) {
      L.job = atomicAdd(&dc->seg_next[kTier], 1u);
      L.diff = 0ull;
    }
    __syncthreads();
    const uint32_t job = L.job;
    if (job >= n_jobs) break;
    uint32_t start, len;
    bool whole = true;
    if (!kChunks) {
      const uint32_t m = mine[job];
      start = mt_off[m];
      len = mt_off[m + 1] - start;
    } else {
      // the long segment k whose chunks hold this job: last k with chunk_off[k] <= job
      uint32_t lo = 0, hi = n_long - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (chunk_off[mid] <= job) lo = mid;
        else hi = mid - 1;
      }
      const uint32_t m = mine[lo];
      const uint32_t seg0 = mt_off[m], seg_end = mt_off[m + 1];
      start = seg0 + (job - chunk_off[lo]) * (uint32_t)kSegChunk;
      len = min((uint32_t)kSegChunk, seg_end - start);
      whole = false;
    }
    // load, wave-blocked: element j = wave * 64 * kItems + r * 64 + lane
    const uint64_t first = comp[start];
    uint64_t key[kItems];
    uint64_t diff = 0ull;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t j = (uint32_t)(wave * 64 * kItems + r * 64 + lane);
      key[r] = j < len ? comp[start + j] : ~0ull;  // padding sorts last
      if (j < len) diff |= key[r] ^ first;
    }
    // the digits that vary within the segment
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) diff |= __shfl_xor(diff, off, 64);
    if (lane == 0 && diff) atomicOr(&L.diff, (unsigned long long)diff);
    __syncthreads();
    const uint64_t vary = L.diff;
    uint32_t rank[kItems];
    // one stable LSD pass on the 8-bit digit at `shift`: registers -> LDS in
    // digit order -> registers
    auto radix_pass = [&](int shift) __attribute__((always_inline)) {
      for (int k = tid; k < kWaves * kDigits; k += kThreads) (&L.whist[0][0])[k] = 0;
      __syncthreads();
      // stable wave-level ranking, item order (r, lane)
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t d = (uint32_t)(key[r] >> shift) & (kDigits - 1);
        uint64_t peers = ~0ull;
#pragma unroll
        for (int bit = 0; bit < kDigitBits; ++bit) {
          const bool set = (d >> bit) & 1u;
          const uint64_t bal = __ballot(set);
          peers &= set ? bal : ~bal;
        }
        const uint32_t before = (uint32_t)__popcll(peers & lt_mask);
        const uint32_t prev = L.whist[wave][d];
        rank[r] = prev + before;
        // every lane has read its digit's count before the first lane of each
        // digit group adds the group to it (lockstep wave; the barrier keeps
        // the compiler from moving the store up)
        __builtin_amdgcn_wave_barrier();
        if (before == 0) L.whist[wave][d] = prev + (uint32_t)__popcll(peers);
      }
      __syncthreads();
      // per digit: wave prefixes, digit totals, then the digits' exclusive scan
      uint32_t tot = 0, incl = 0;
      if (tid < kDigits) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          const uint32_t c = L.whist[w][tid];
          L.whist[w][tid] = tot;
          tot += c;
        }
        incl = wave_scan_incl(tot);
        if (lane == 63) L.dtot[wave] = incl;
      }
      __syncthreads();
      if (tid < kDigits) {
        uint32_t s = incl - tot;
        for (int w = 0; w < wave; ++w) s += L.dtot[w];
        L.dstart[tid] = s;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t d = (uint32_t)(key[r] >> shift) & (kDigits - 1);
        L.v[L.dstart[d] + L.whist[wave][d] + rank[r]] = key[r];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kItems; ++r) key[r] = L.v[wave * 64 * kItems + r * 64 + lane];
      __syncthreads();
    };
    // the passes over the digits of `bits` (from bit `from` up) that vary
    auto sort_bits = [&](int from) __attribute__((always_inline)) {
      for (int shift = from; shift < 64; shift += kDigitBits) {
        if ((vary >> shift) == 0ull) break;                      // no higher digit varies
        if (((vary >> shift) & (kDigits - 1)) == 0ull) continue;  // this digit is constant
        radix_pass(shift);
      }
    };
    // sort on the depth part only (the bits above the id); then equal depths,
    // adjacent now, are put in id order: a short run by its first element's
    // thread, and a segment with a run longer than kTieRun sorts again on
    // every bit (composites are unique, so that order is exact)
    sort_bits((int)gbits);
#pragma unroll
    for (int r = 0; r < kItems; ++r) L.v[wave * 64 * kItems + r * 64 + lane] = key[r];
    if (tid == 0) L.long_tie = 0;
    __syncthreads();
    for (uint32_t j = tid; j < len; j += kThreads) {
      const uint64_t kj = L.v[j] >> gbits;
      if ((j > 0 && (L.v[j - 1] >> gbits) == kj) || j + 1 >= len || (L.v[j + 1] >> gbits) != kj)
        continue;  // not the first of a run of two or more
      uint32_t e = j + 2;
      while (e < len && (L.v[e] >> gbits) == kj && e - j <= (uint32_t)kTieRun) ++e;
      if (e - j > (uint32_t)kTieRun) {
        L.long_tie = 1;
        continue;
      }
      for (uint32_t a = j + 1; a < e; ++a) {  // insertion sort of the run
        const uint64_t x = L.v[a];
        uint32_t q = a;
        for (; q > j && L.v[q - 1] > x; --q) L.v[q] = L.v[q - 1];
        L.v[q] = x;
      }
    }
    __syncthreads();
    const bool long_tie = L.long_tie != 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) key[r] = L.v[wave * 64 * kItems + r * 64 + lane];
    __syncthreads();
    if (long_tie) sort_bits(0);
    // out: ids of a whole segment, the sorted run of a chunk
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t j = (uint32_t)(wave * 64 * kItems + r * 64 + lane);
      if (j < len) {
        if (whole) ids[start + j] = (uint32_t)(key[r] & idmask);
        else runs[start + j] = key[r];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ merge --
// Number of elements of A[0, na) that precede output position d of the merge
// of A and B (keys unique): the largest a in [max(0, d - nb), min(d, na)]
// with a == 0 or A[a - 1] < B[d - a].
__device__ __forceinline__ uint32_t merge_split(const uint64_t* __restrict__ A, uint32_t na,
                                                const uint64_t* __restrict__ B, uint32_t nb,
                                                uint32_t d) {
  uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;  // candidate a = mid: needs A[mid-1] < B[d-mid]
    if (A[mid - 1] < B[d - mid]) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

constexpr int kMergeThreads = 1024;
struct PartMergeLds {
  uint64_t v[kSegChunk];  // [0, ca) from run A, then [ca, ca + cb) from run B
  uint32_t blk;
};

__global__ void __launch_bounds__(kMergeThreads)
part_merge_kernel(int level, int n_mt, uint32_t gbits, const uint32_t* __restrict__ mt_off,
                  const uint32_t* __restrict__ list, const uint64_t* __restrict__ src,
                  uint64_t* __restrict__ dst, uint32_t* __restrict__ ids,
                  DeviceCounters* __restrict__ dc) {
  __shared__ PartMergeLds L;
  const uint64_t run = (uint64_t)kSegChunk << level;
  if (dc->overflow) return;
  if ((uint64_t)dc->seg_max <= run) return;  // every segment was finished before this level
  const uint32_t* __restrict__ longs = list + (size_t)(kSegTiers - 1) * n_mt;
  const uint32_t* __restrict__ chunk_off = list + (size_t)kSegTiers * n_mt;
  const uint32_t n_long = dc->seg_tier_n[kSegTiers - 1];
  const uint32_t total = dc->seg_chunks;  // output blocks of kSegChunk, as many as chunks
  const uint64_t idmask = (1ull << gbits) - 1ull;
  for (;;) {
    if (threadIdx.x == 0) L.blk = atomicAdd(&dc->seg_next[kSegTiers + level], 1u);
    __syncthreads();
    const uint32_t bi = L.blk;
    __syncthreads();
    if (bi >= total) break;
    uint32_t lo = 0, hi = n_long - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (chunk_off[mid] <= bi) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t m = longs[lo];
    const uint32_t seg0 = mt_off[m], seg_n = mt_off[m + 1] - seg0;
    if (seg_n <= run) continue;  // finished at an earlier level (uniform)
    // this block: output positions [p0, p1) of the segment
    const uint32_t p0 = (bi - chunk_off[lo]) * (uint32_t)kSegChunk;
    const uint32_t pair0 = (uint32_t)(p0 / (2 * run) * (2 * run));  // the merged pair of runs
    const uint32_t na = (uint32_t)min(run, (uint64_t)(seg_n - pair0));
    const uint32_t nb =
        seg_n - pair0 > run ? (uint32_t)min(run, (uint64_t)(seg_n - pair0) - run) : 0u;
    const uint32_t p1 = min(p0 + (uint32_t)kSegChunk, pair0 + na + nb);
    const uint64_t* A = src + seg0 + pair0;
    const uint64_t* B = A + na;
    const uint32_t d0 = p0 - pair0, d1 = p1 - pair0;
    const uint32_t a0 = merge_split(A, na, B, nb, d0), a1 = merge_split(A, na, B, nb, d1);
    const uint32_t b0 = d0 - a0, b1 = d1 - a1;
    const uint32_t ca = a1 - a0, cb = b1 - b0;
    for (uint32_t k = threadIdx.x; k < ca; k += kMergeThreads) L.v[k] = A[a0 + k];
    for (uint32_t k = threadIdx.x; k < cb; k += kMergeThreads) L.v[ca + k] = B[b0 + k];
    __syncthreads();
    // each thread merges its own slice of the block's outputs
    const bool last = (uint64_t)seg_n <= 2 * run;  // the segment is complete after this level
    const uint32_t cnt = ca + cb;
    const uint32_t per = (cnt + kMergeThreads - 1) / kMergeThreads;
    const uint32_t q0 = min(cnt, threadIdx.x * per), q1 = min(cnt, q0 + per);
    if (q0 < q1) {
      uint32_t ia = merge_split(L.v, ca, L.v + ca, cb, q0);
      uint32_t ib = q0 - ia;
      for (uint32_t q = q0; q < q1; ++q) {
        uint64_t x;
        if (ib >= cb || (ia < ca && L.v[ia] < L.v[ca + ib])) x = L.v[ia++];
        else x = L.v[ca + ib++];
        const uint32_t at = seg0 + p0 + q;
        if (last) ids[at] = (uint32_t)(x & idmask);
        else dst[at] = x;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launch --
static uint32_t id_bits(int64_t n) {
  uint32_t g = 0;
  for (int64_t v = n > 1 ? n - 1 : 0; v; v >>= 1) ++g;
  return g;
}

static int per_cu(const void* kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

static int g_sort_per_cu[kSegTiers] = {}, g_merge_per_cu = 0;

int seg_sort_configs() {
  if (g_merge_per_cu == 0) {
    g_sort_per_cu[0] = per_cu(reinterpret_cast<const void*>(part_sort_kernel<256, 4, 0>), 256);
    g_sort_per_cu[1] = per_cu(reinterpret_cast<const void*>(part_sort_kernel<256, 8, 1>), 256);
    g_sort_per_cu[2] = per_cu(reinterpret_cast<const void*>(part_sort_kernel<512, 8, 2>), 512);
    g_sort_per_cu[3] = per_cu(reinterpret_cast<const void*>(part_sort_kernel<1024, 8, 3>), 1024);
    g_sort_per_cu[4] = per_cu(reinterpret_cast<const void*>(part_sort_kernel<1024, 8, 4>), 1024);
    g_merge_per_cu = per_cu(reinterpret_cast<const void*>(part_merge_kernel), kMergeThreads);
  }
  return g_merge_per_cu;
}

hipError_t launch_seg_count(int64_t n, CamArgs cam, const float* f_mx, const float* f_my,
                            const float* f_a, const float* f_b, const float* f_c,
                            const float* f_tau, const uint32_t* f_cnt, const uint32_t* f_span,
                            SegBuffers sb, uint32_t max_pairs, DeviceCounters* dc, hipStream_t s) {
  const int n_mt = cam.n_mt_x * cam.n_mt_y;
  const uint32_t n_b = (uint32_t)((n + kSegBatch - 1) / kSegBatch);
  const uint64_t n_entries = (uint64_t)n_mt * n_b;
  const uint32_t n_tiles = (uint32_t)((n_entries + kSegScanTile - 1) / kSegScanTile);
  if (n_b > 0)
    hipLaunchKernelGGL(part_count_kernel, dim3(n_b), dim3(kPartThreads), n_mt * sizeof(uint32_t), s,
                       n, cam, n_mt, n_b, f_mx, f_my, f_a, f_b, f_c, f_tau, f_cnt, f_span, sb.cm, dc);
  if (n_tiles > 0)
    hipLaunchKernelGGL(part_tile_sum_kernel, dim3(n_tiles), dim3(kScanThreads), 0, s, n_entries,
                       sb.cm, sb.tile_sum);
  hipLaunchKernelGGL(part_scan_top_kernel, dim3(1), dim3(kPlanThreads), 0, s, n_tiles, n_mt, n_b,
                     max_pairs, sb.tile_sum, sb.mt_off, dc);
  if (n_tiles > 0)
    hipLaunchKernelGGL(part_tile_scan_kernel, dim3(n_tiles), dim3(kScanThreads), 0, s, n_entries,
                       n_b, max_pairs, sb.cm, sb.tile_sum, sb.off, sb.mt_off);
  hipLaunchKernelGGL(part_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, n_mt, sb.mt_off, sb.list,
                     dc);
  return hipGetLastError();
}

hipError_t launch_seg_fill(int64_t n, CamArgs cam, const float* f_mx, const float* f_my,
                           const float* f_a, const float* f_b, const float* f_c, const float* f_tau,
                           const uint32_t* f_key, const uint32_t* f_cnt, const uint32_t* f_span,
                           SegBuffers sb, uint32_t max_pairs, DeviceCounters* dc, hipStream_t s) {
  const int n_mt = cam.n_mt_x * cam.n_mt_y;
  const uint32_t n_b = (uint32_t)((n + kSegBatch - 1) / kSegBatch);
  if (n_b > 0)
    hipLaunchKernelGGL(part_fill_kernel, dim3(n_b), dim3(kPartThreads), n_mt * sizeof(uint32_t), s,
                       n, cam, n_mt, n_b, id_bits(n), f_mx, f_my, f_a, f_b, f_c, f_tau, f_key,
                       f_cnt, f_span, sb.off, dc, max_pairs, sb.comp);
  return hipGetLastError();
}

hipError_t launch_seg_sort(int64_t n, int n_mt, SegBuffers sb, uint32_t max_pairs,
                           DeviceCounters* dc, int n_cus, hipStream_t s) {
  const uint32_t gbits = id_bits(n);
  seg_sort_configs();
  hipLaunchKernelGGL((part_sort_kernel<256, 4, 0>), dim3(n_cus * g_sort_per_cu[0]), dim3(256), 0, s,
                     sb.mt_off, sb.list, n_mt, gbits, sb.comp, sb.runs, sb.ids, dc);
  hipLaunchKernelGGL((part_sort_kernel<256, 8, 1>), dim3(n_cus * g_sort_per_cu[1]), dim3(256), 0, s,
                     sb.mt_off, sb.list, n_mt, gbits, sb.comp, sb.runs, sb.ids, dc);
  hipLaunchKernelGGL((part_sort_kernel<512, 8, 2>), dim3(n_cus * g_sort_per_cu[2]), dim3(512), 0, s,
                     sb.mt_off, sb.list, n_mt, gbits, sb.comp, sb.runs, sb.ids, dc);
  hipLaunchKernelGGL((part_sort_kernel<1024, 8, 3>), dim3(n_cus * g_sort_per_cu[3]), dim3(1024), 0,
                     s, sb.mt_off, sb.list, n_mt, gbits, sb.comp, sb.runs, sb.ids, dc);
  hipLaunchKernelGGL((part_sort_kernel<1024, 8, 4>), dim3(n_cus * g_sort_per_cu[4]), dim3(1024), 0,
                     s, sb.mt_off, sb.list, n_mt, gbits, sb.comp, sb.runs, sb.ids, dc);
  // merge levels: runs of kSegChunk << l, up to the longest segment possible
  // (a gaussian puts at most one pair in a macro-tile); a level with nothing
  // left returns at once
  const int64_t longest = n < (int64_t)max_pairs ? n : (int64_t)max_pairs;
  int levels = 0;
  while (((int64_t)kSegChunk << levels) < longest && levels < kSegMaxLevels) ++levels;
  // (a level halves the runs still merging: deeper levels get fewer workers,
  // so that a level with nothing left costs little more than its launch)
  for (int l = 0; l < levels; ++l) {
    const uint64_t* src = (l & 1) ? sb.comp : sb.runs;
    uint64_t* dst = (l & 1) ? sb.runs : sb.comp;
    const int workers = (n_cus * g_merge_per_cu) >> (l < 3 ? l : 3);
    hipLaunchKernelGGL(part_merge_kernel, dim3(workers > 0 ? workers : 1), dim3(kMergeThreads), 0, s,
                       l, n_mt, gbits, sb.mt_off, sb.list, src, dst, sb.ids, dc);
  }
  return hipGetLastError();
}

}  // namespace higs
