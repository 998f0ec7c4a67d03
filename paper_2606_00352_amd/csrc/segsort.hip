// Stages 2-3, segmented form (sec. 3.2 Gaussian partitioning, sec. 3.3
// Segmented depth sort, sec. 4.3-4.4): pairs are binned straight into one
// contiguous segment per macro-tile, and every segment is sorted on its own by
// depth; no global composite-key sort.
//
// seg_count_kernel (one workgroup per partition batch of B_p = 8,192
//   gaussians): an LDS histogram with one counter per macro-tile, filled by LDS
//   atomics from each visible gaussian's macro-tile list (the compact list the
//   projection recorded, else the exact predicate again on the stored float32
//   fields), then added to the frame's per-macro-tile totals (one global
//   atomic per touched counter).
// seg_scan_kernel (one workgroup): segment offsets (exclusive scan of the
//   totals), the fill cursors, the pair total and overflow, the chunk table
//   of the segment sort and the block table of its merges.
// seg_fill_kernel (one workgroup per partition batch): counts its batch's hits
//   per macro-tile in LDS, reserves a range in each touched segment with one
//   global atomic, and writes each pair as a 64-bit composite
//   ((depth bits - min) << g) | id, g = bits of the largest id.  Sorting
//   composites orders a segment by (depth, id) whatever order the fill wrote
//   it in, so the fill may use atomics freely.
// seg_chunk_sort_kernel (persistent): chunks of at most C = 8,192 composites of
//   one segment, bitonic-sorted in LDS (64 KiB); a segment of one chunk is
//   done and its ids go to the output, longer ones leave sorted runs.
// seg_merge_kernel (persistent, once per level l): the runs of length
//   C * 2^l of each segment still unfinished are merged pairwise, in output
//   blocks of C elements; a block finds its share of the two runs by a
//   merge-path search and merges it in LDS.  A segment whose merge completes
//   at this level writes ids to the output.
// The output is the sorted list of ids in (macro-tile, depth, id) order and
// the segment offsets; the raster stage reads the ids.
#include "higs_internal.h"
#include "predicate.h"

namespace higs {

constexpr int kSegThreads = 1024;
constexpr int kSegPerThread = kSegBatch / kSegThreads;  // gaussians per thread in a partition batch
constexpr int kChunk = 8192;                            // composites per LDS sort chunk
constexpr uint64_t kPad = ~0ull;

// ------------------------------------------------------------------ count --
__global__ void __launch_bounds__(kSegThreads)
seg_count_kernel(int64_t n, CamArgs cam, int n_mt, const float* __restrict__ f_mx,
                 const float* __restrict__ f_my, const float* __restrict__ f_a,
                 const float* __restrict__ f_b, const float* __restrict__ f_c,
                 const float* __restrict__ f_tau, const uint32_t* __restrict__ f_cnt,
                 const uint32_t* __restrict__ f_span, uint32_t* __restrict__ seg_count,
                 DeviceCounters* __restrict__ dc) {
  HIP_DYNAMIC_SHARED(uint32_t, hist)
  __shared__ uint32_t s_vis;
  for (int m = threadIdx.x; m < n_mt; m += kSegThreads) hist[m] = 0;
  if (threadIdx.x == 0) s_vis = 0;
  __syncthreads();
  uint32_t vis = 0;
  const int64_t base = (int64_t)blockIdx.x * kSegBatch;
  for (int r = 0; r < kSegPerThread; ++r) {
    const int64_t i = base + (int64_t)r * kSegThreads + threadIdx.x;
    if (i >= n || f_cnt[i] == 0) continue;
    ++vis;
    auto hit = [&](uint32_t mt) { atomicAdd(&hist[mt], 1u); };
    const uint32_t w = f_span[i];
    if (w) {
      visit_span(w, cam.n_mt_x, hit);
    } else {
      BinFields f;
      f.mx = f_mx[i];
      f.my = f_my[i];
      f.a = f_a[i];
      f.b = f_b[i];
      f.c = f_c[i];
      f.tau = f_tau[i];
      visit_macro_tiles(f, cam.width, cam.height, cam.n_mt_x, cam.n_mt_y, hit);
    }
  }
  if (vis) atomicAdd(&s_vis, vis);
  __syncthreads();
  for (int m = threadIdx.x; m < n_mt; m += kSegThreads)
    if (hist[m]) atomicAdd(&seg_count[m], hist[m]);
  if (threadIdx.x == 0 && s_vis) atomicAdd(&dc->n_visible, s_vis);
}

// ------------------------------------------------------------------- scan --
constexpr int kSegScanThreads = 1024;

// Block-wide exclusive scan of one value per thread; *total gets the sum.
__device__ __forceinline__ uint32_t seg_block_scan(uint32_t v, uint32_t* wt, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(x, off, 64);
    if (lane >= off) x += o;
  }
  __syncthreads();
  if (lane == 63) wt[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < kSegScanThreads / 64; ++w) {
    before += w < wave ? wt[w] : 0u;
    all += wt[w];
  }
  *total = all;
  return before + x - v;
}

__global__ void __launch_bounds__(kSegScanThreads)
seg_scan_kernel(int n_mt, uint32_t max_pairs, const uint32_t* __restrict__ seg_count,
                uint32_t* __restrict__ mt_off, uint32_t* __restrict__ cursor,
                uint32_t* __restrict__ chunk_off, uint32_t* __restrict__ blk_off,
                DeviceCounters* __restrict__ dc) {
  __shared__ uint32_t wt[kSegScanThreads / 64];
  __shared__ uint32_t s_max;
  if (threadIdx.x == 0) s_max = 0;
  const int per = (n_mt + kSegScanThreads - 1) / kSegScanThreads;
  const int m0 = threadIdx.x * per, m1 = min(m0 + per, n_mt);
  uint32_t pairs = 0, chunks = 0, blocks = 0, mx = 0;
  for (int m = m0; m < m1; ++m) {
    const uint32_t c = seg_count[m];
    pairs += c;
    chunks += (c + kChunk - 1) / kChunk;
    blocks += c > (uint32_t)kChunk ? (c + kChunk - 1) / kChunk : 0u;
    mx = max(mx, c);
  }
  uint32_t tp, tc, tb;
  uint32_t rp = seg_block_scan(pairs, wt, &tp);
  uint32_t rc = seg_block_scan(chunks, wt, &tc);
  uint32_t rb = seg_block_scan(blocks, wt, &tb);
  if (mx) atomicMax(&s_max, mx);
  // past the capacity the frame is invalid: offsets are clamped to it and no
  // sort work is scheduled, so that nothing reads or writes beyond the buffers
  const bool ovf = tp > max_pairs;
  for (int m = m0; m < m1; ++m) {
    const uint32_t c = seg_count[m];
    mt_off[m] = min(rp, max_pairs);
    cursor[m] = rp;
    chunk_off[m] = ovf ? 0u : rc;
    blk_off[m] = ovf ? 0u : rb;
    rp += c;
    rc += (c + kChunk - 1) / kChunk;
    rb += c > (uint32_t)kChunk ? (c + kChunk - 1) / kChunk : 0u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    mt_off[n_mt] = min(tp, max_pairs);
    chunk_off[n_mt] = ovf ? 0u : tc;
    blk_off[n_mt] = ovf ? 0u : tb;
    dc->n_pairs_total = tp;
    dc->n_pairs = ovf ? max_pairs : tp;
    if (ovf) atomicOr(&dc->overflow, (uint32_t)HIGS_OVF_PAIRS);
    dc->seg_max = ovf ? 0u : s_max;
    dc->sort_final = 0;  // the ids end in the first value buffer
    dc->sort_passes = 0;
  }
}

// ------------------------------------------------------------------- fill --
__global__ void __launch_bounds__(kSegThreads)
seg_fill_kernel(int64_t n, CamArgs cam, int n_mt, uint32_t gbits, const float* __restrict__ f_mx,
                const float* __restrict__ f_my, const float* __restrict__ f_a,
                const float* __restrict__ f_b, const float* __restrict__ f_c,
                const float* __restrict__ f_tau, const uint32_t* __restrict__ f_key,
                const uint32_t* __restrict__ f_cnt, const uint32_t* __restrict__ f_span,
                uint32_t* __restrict__ cursor,
                const DeviceCounters* __restrict__ dc, uint32_t max_pairs,
                uint64_t* __restrict__ comp) {
  HIP_DYNAMIC_SHARED(uint32_t, lds)
  if (dc->overflow) return;  // the frame stops at a capacity overflow
  uint32_t* cnt = lds;          // hits of this batch per macro-tile, then the running slot
  uint32_t* base = lds + n_mt;  // reserved start of this batch's range in each segment
  for (int m = threadIdx.x; m < n_mt; m += kSegThreads) cnt[m] = 0;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kSegBatch;
  // each gaussian's macro-tile list: the recorded span, else the predicate
  auto visit = [&](int64_t i, auto&& fn) {
    const uint32_t w = f_span[i];
    if (w) {
      visit_span(w, cam.n_mt_x, fn);
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
  };
  for (int r = 0; r < kSegPerThread; ++r) {
    const int64_t i = b0 + (int64_t)r * kSegThreads + threadIdx.x;
    if (i >= n || f_cnt[i] == 0) continue;
    visit(i, [&](uint32_t mt) { atomicAdd(&cnt[mt], 1u); });
  }
  __syncthreads();
  for (int m = threadIdx.x; m < n_mt; m += kSegThreads) {
    const uint32_t c = cnt[m];
    base[m] = c ? atomicAdd(&cursor[m], c) : 0u;
    cnt[m] = 0;
  }
  __syncthreads();
  const uint32_t dmin = dc->key_min;
  for (int r = 0; r < kSegPerThread; ++r) {
    const int64_t i = b0 + (int64_t)r * kSegThreads + threadIdx.x;
    if (i >= n || f_cnt[i] == 0) continue;
    const uint64_t c = ((uint64_t)(f_key[i] - dmin) << gbits) | (uint64_t)i;
    visit(i, [&](uint32_t mt) {
      const uint32_t at = base[mt] + atomicAdd(&cnt[mt], 1u);
      if (at < max_pairs) comp[at] = c;
    });
  }
}

// --------------------------------------------------------- chunk sort --
// In-place bitonic sort of L.v[0, size) (size a power of two <= kChunk) by all
// threads of the workgroup.
__device__ __forceinline__ void bitonic_lds(uint64_t* v, int size) {
  for (int k = 2; k <= size; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < size / 2; t += kSegThreads) {
        const int lo = 2 * t - (t & (j - 1));  // index with bit j clear
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const uint64_t a = v[lo], b = v[hi];
        if ((a > b) == up) {
          v[lo] = b;
          v[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

// Segment m of the chunk with global index ci: the last m with
// chunk_off[m] <= ci (chunk_off ascending; empty segments repeat values).
__device__ __forceinline__ int seg_of(const uint32_t* __restrict__ off, int n_mt, uint32_t ci) {
  int lo = 0, hi = n_mt - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= ci) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(kSegThreads)
seg_chunk_sort_kernel(int n_mt, uint32_t gbits, const uint32_t* __restrict__ mt_off,
                      const uint32_t* __restrict__ chunk_off, const uint64_t* __restrict__ comp,
                      uint64_t* __restrict__ runs, uint32_t* __restrict__ ids,
                      DeviceCounters* __restrict__ dc) {
  HIP_DYNAMIC_SHARED(uint64_t, v)
  __shared__ uint32_t s_chunk;
  if (dc->overflow) return;
  const uint32_t total = chunk_off[n_mt];
  const uint32_t np = dc->n_pairs;
  const uint64_t idmask = (1ull << gbits) - 1ull;
  for (;;) {
    if (threadIdx.x == 0) s_chunk = atomicAdd(&dc->seg_next[0], 1u);
    __syncthreads();
    const uint32_t ci = s_chunk;
    __syncthreads();
    if (ci >= total) break;
    const int m = seg_of(chunk_off, n_mt, ci);
    const uint32_t seg0 = mt_off[m], seg_n = mt_off[m + 1] - seg0;
    const uint32_t start = seg0 + (ci - chunk_off[m]) * (uint32_t)kChunk;
    const uint32_t len = min((uint32_t)kChunk, seg0 + seg_n - start);
    int size = 1;
    while (size < (int)len) size <<= 1;
    for (int k = threadIdx.x; k < size; k += kSegThreads)
      v[k] = (k < (int)len && start + k < np) ? comp[start + k] : kPad;
    __syncthreads();
    bitonic_lds(v, size);
    if (seg_n <= (uint32_t)kChunk) {
      for (uint32_t k = threadIdx.x; k < len; k += kSegThreads)
        if (start + k < np) ids[start + k] = (uint32_t)(v[k] & idmask);
    } else {
      for (uint32_t k = threadIdx.x; k < len; k += kSegThreads)
        if (start + k < np) runs[start + k] = v[k];
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

__global__ void __launch_bounds__(kSegThreads)
seg_merge_kernel(int level, int n_mt, uint32_t gbits, const uint32_t* __restrict__ mt_off,
                 const uint32_t* __restrict__ blk_off, const uint64_t* __restrict__ src,
                 uint64_t* __restrict__ dst, uint32_t* __restrict__ ids,
                 DeviceCounters* __restrict__ dc) {
  HIP_DYNAMIC_SHARED(uint64_t, v)  // [0, na) from A, then [na, na + nb) from B
  __shared__ uint32_t s_blk;
  const uint64_t run = (uint64_t)kChunk << level;
  if ((uint64_t)dc->seg_max <= run) return;  // every segment was finished before this level
  if (dc->overflow) return;
  const uint32_t total = blk_off[n_mt];
  const uint32_t np = dc->n_pairs;
  const uint64_t idmask = (1ull << gbits) - 1ull;
  for (;;) {
    if (threadIdx.x == 0) s_blk = atomicAdd(&dc->seg_next[1 + level], 1u);
    __syncthreads();
    const uint32_t bi = s_blk;
    __syncthreads();
    if (bi >= total) break;
    const int m = seg_of(blk_off, n_mt, bi);
    const uint32_t seg0 = mt_off[m], seg_n = mt_off[m + 1] - seg0;
    if (seg_n <= run) continue;  // finished at an earlier level (uniform)
    // this block: output positions [p0, p1) of the segment
    const uint32_t p0 = (bi - blk_off[m]) * (uint32_t)kChunk;
    const uint32_t pair0 = (uint32_t)(p0 / (2 * run) * (2 * run));  // start of the merged pair of runs
    const uint32_t na = (uint32_t)min(run, (uint64_t)(seg_n - pair0));
    const uint32_t nb = seg_n - pair0 > run ? (uint32_t)min(run, (uint64_t)(seg_n - pair0) - run) : 0u;
    const uint32_t p1 = min(p0 + (uint32_t)kChunk, pair0 + na + nb);
    const uint64_t* A = src + seg0 + pair0;
    const uint64_t* B = A + na;
    const uint32_t d0 = p0 - pair0, d1 = p1 - pair0;
    const uint32_t a0 = merge_split(A, na, B, nb, d0), a1 = merge_split(A, na, B, nb, d1);
    const uint32_t b0 = d0 - a0, b1 = d1 - a1;
    const uint32_t ca = a1 - a0, cb = b1 - b0;
    for (uint32_t k = threadIdx.x; k < ca; k += kSegThreads) v[k] = A[a0 + k];
    for (uint32_t k = threadIdx.x; k < cb; k += kSegThreads) v[ca + k] = B[b0 + k];
    __syncthreads();
    // each thread merges its own slice of the block's outputs
    const bool last = (uint64_t)seg_n <= 2 * run;  // the segment is complete after this level
    const uint32_t cnt = ca + cb;
    const uint32_t per = (cnt + kSegThreads - 1) / kSegThreads;
    const uint32_t q0 = min(cnt, threadIdx.x * per), q1 = min(cnt, q0 + per);
    if (q0 < q1) {
      uint32_t ia = merge_split(v, ca, v + ca, cb, q0);
      uint32_t ib = q0 - ia;
      for (uint32_t q = q0; q < q1; ++q) {
        uint64_t x;
        if (ib >= cb || (ia < ca && v[ia] < v[ca + ib])) x = v[ia++];
        else x = v[ca + ib++];
        const uint32_t at = seg0 + p0 + q;
        if (at < np) {
          if (last) ids[at] = (uint32_t)(x & idmask);
          else dst[at] = x;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launch --
static int g_seg_chunk_per_cu = 0, g_seg_merge_per_cu = 0;

static uint32_t id_bits(int64_t n) {
  uint32_t g = 0;
  for (int64_t v = n > 1 ? n - 1 : 0; v; v >>= 1) ++g;
  return g;
}

hipError_t launch_seg_count(int64_t n, CamArgs cam, const float* f_mx, const float* f_my,
                            const float* f_a, const float* f_b, const float* f_c,
                            const float* f_tau, const uint32_t* f_cnt, const uint32_t* f_span,
                            SegBuffers sb, uint32_t max_pairs, DeviceCounters* dc, hipStream_t s) {
  const int n_mt = cam.n_mt_x * cam.n_mt_y;
  const unsigned batches = (unsigned)((n + kSegBatch - 1) / kSegBatch);
  if (batches > 0)
    hipLaunchKernelGGL(seg_count_kernel, dim3(batches), dim3(kSegThreads), n_mt * sizeof(uint32_t),
                       s, n, cam, n_mt, f_mx, f_my, f_a, f_b, f_c, f_tau, f_cnt, f_span, sb.seg_count,
                       dc);
  hipLaunchKernelGGL(seg_scan_kernel, dim3(1), dim3(kSegScanThreads), 0, s, n_mt, max_pairs,
                     sb.seg_count, sb.mt_off, sb.cursor, sb.chunk_off, sb.blk_off, dc);
  return hipGetLastError();
}

hipError_t launch_seg_fill(int64_t n, CamArgs cam, const float* f_mx, const float* f_my,
                           const float* f_a, const float* f_b, const float* f_c, const float* f_tau,
                           const uint32_t* f_key, const uint32_t* f_cnt, const uint32_t* f_span,
                           SegBuffers sb, uint32_t max_pairs, DeviceCounters* dc, hipStream_t s) {
  const int n_mt = cam.n_mt_x * cam.n_mt_y;
  const unsigned batches = (unsigned)((n + kSegBatch - 1) / kSegBatch);
  if (batches > 0)
    hipLaunchKernelGGL(seg_fill_kernel, dim3(batches), dim3(kSegThreads),
                       2 * n_mt * sizeof(uint32_t), s, n, cam, n_mt, id_bits(n), f_mx, f_my, f_a,
                       f_b, f_c, f_tau, f_key, f_cnt, f_span, sb.cursor, dc, max_pairs,
                       sb.comp);
  return hipGetLastError();
}

hipError_t launch_seg_sort(int64_t n, int n_mt, SegBuffers sb, uint32_t max_pairs,
                           DeviceCounters* dc, int n_cus, hipStream_t s) {
  const uint32_t gbits = id_bits(n);
  if (g_seg_chunk_per_cu == 0) {
    int a = 0, b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, seg_chunk_sort_kernel, kSegThreads,
                                                     kChunk * sizeof(uint64_t)) != hipSuccess ||
        a < 1)
      a = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, seg_merge_kernel, kSegThreads,
                                                     kChunk * sizeof(uint64_t)) != hipSuccess ||
        b < 1)
      b = 1;
    g_seg_chunk_per_cu = a;
    g_seg_merge_per_cu = b;
  }
  hipLaunchKernelGGL(seg_chunk_sort_kernel, dim3(n_cus * g_seg_chunk_per_cu), dim3(kSegThreads),
                     kChunk * sizeof(uint64_t), s, n_mt, gbits, sb.mt_off, sb.chunk_off, sb.comp,
                     sb.runs, sb.ids, dc);
  // merge levels: runs of kChunk << l, enough for the largest possible segment;
  // a level with nothing left returns at once
  int levels = 0;
  while (((int64_t)kChunk << levels) < (int64_t)max_pairs && levels < kSegMaxLevels) ++levels;
  for (int l = 0; l < levels; ++l) {
    const uint64_t* src = (l & 1) ? sb.comp : sb.runs;
    uint64_t* dst = (l & 1) ? sb.runs : sb.comp;
    hipLaunchKernelGGL(seg_merge_kernel, dim3(n_cus * g_seg_merge_per_cu), dim3(kSegThreads),
                       kChunk * sizeof(uint64_t), s, l, n_mt, gbits, sb.mt_off, sb.blk_off, src,
                       dst, sb.ids, dc);
  }
  return hipGetLastError();
}

}  // namespace higs
