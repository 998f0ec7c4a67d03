// Stage 2a: (macro-tile, gaussian) pair emission (sec. 3.2 and sec. 4.3:
// count, prefix sum, fill).
//
// The per-gaussian counts and compact macro-tile lists (span words) come from
// the projection kernel.  `chunk_sum_kernel` sums the per-block sums over
// chunks of kScanChunk blocks, `scan_kernel` (one workgroup) turns the chunk
// totals into exclusive chunk offsets and the frame's pair total, and chooses
// the pair layout; `fill_kernel` scans its chunk's block sums and the counts
// inside the block with wave prefix sums and writes pairs in gaussian-id
// order, macro-tiles ascending
// within a gaussian: each gaussian's macro-tiles come from its span word, or,
// for a list the word cannot hold, from the intersection re-run on the stored
// float32 fields (the count pass's exact decisions).  Waves whose 64 gaussians
// are all invisible skip their work (ballot).
//
// Key layout: (macro-tile << dbits) | (depth bits - dmin), where dmin and
// dmin + 2^dbits - 1 bracket the float32 depth bits of the frame's visible
// gaussians (found by the projection).  The map is monotone in (macro-tile,
// depth), so the sort order is unchanged, and the key has dbits + log2(n_mt)
// significant bits instead of 32 + log2(n_mt).  A pair is the one word
// key << g | id (g the id bits) when that fits 64 bits with a bit to spare,
// else a key array and an id array.
#include "higs_internal.h"
#include "predicate.h"

namespace higs {

__global__ void clear_kernel(DeviceCounters* dc, uint32_t* hist, int n_hist) {
  uint32_t* w = reinterpret_cast<uint32_t*>(dc);
  const int nw = (int)(sizeof(DeviceCounters) / 4);
  const int keep = (int)(offsetof(DeviceCounters, epoch) / 4);
  for (int k = threadIdx.x; k < nw; k += blockDim.x)
    if (k != keep) w[k] = 0;
  for (int k = threadIdx.x; k < n_hist; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    dc->key_min = 0xffffffffu;
    // this frame's sort passes publish under epochs epoch .. epoch + kMaxPasses - 1
    dc->epoch += (uint32_t)kMaxPasses;
  }
}

hipError_t launch_clear(DeviceCounters* dc, uint32_t* hist, int n_hist, hipStream_t s) {
  hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(1024), 0, s, dc, hist, n_hist);
  return hipGetLastError();
}

// Inclusive wave-wide prefix sum of 64 lanes.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

// A workgroup per chunk of kScanChunk projection blocks (a thread per block):
// the chunk's (pairs, visible) totals, stored after the n_blocks block sums.
__global__ void __launch_bounds__(kScanChunk)
chunk_sum_kernel(uint32_t n_blocks, uint32_t* __restrict__ sums) {
  __shared__ uint32_t wave_tot[2][kScanChunk / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t b = blockIdx.x * kScanChunk + threadIdx.x;
  uint32_t p = b < n_blocks ? sums[2 * (size_t)b] : 0u;
  uint32_t v = b < n_blocks ? sums[2 * (size_t)b + 1] : 0u;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    p += __shfl_xor(p, off, 64);
    v += __shfl_xor(v, off, 64);
  }
  if (lane == 0) {
    wave_tot[0][wave] = p;
    wave_tot[1][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tp = 0, tv = 0;
#pragma unroll
    for (int w = 0; w < kScanChunk / 64; ++w) {
      tp += wave_tot[0][w];
      tv += wave_tot[1][w];
    }
    sums[2 * (size_t)n_blocks + 2 * blockIdx.x] = tp;
    sums[2 * (size_t)n_blocks + 2 * blockIdx.x + 1] = tv;
  }
}

// One workgroup of 1024 threads: exclusive scan of the chunk totals of pairs
// in place, the frame totals, and the pair layout.  A thread per chunk, chunks
// in rounds of 1024 with the carry of the earlier rounds.
constexpr int kScanThreads = 1024;
__global__ void __launch_bounds__(kScanThreads)
scan_kernel(uint32_t n_chunks, uint32_t* __restrict__ chunk, uint32_t max_pairs, int mt_bits,
            int id_bits, DeviceCounters* __restrict__ dc) {
  __shared__ uint32_t wave_tot[2][kScanThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t carry_p = 0, carry_v = 0;  // same in every thread
  for (uint32_t c0 = 0; c0 < n_chunks; c0 += kScanThreads) {
    const uint32_t c = c0 + threadIdx.x;
    const uint32_t p = c < n_chunks ? chunk[2 * (size_t)c] : 0u;
    const uint32_t v = c < n_chunks ? chunk[2 * (size_t)c + 1] : 0u;
    const uint32_t ip = wave_incl_scan(p);
    const uint32_t iv = wave_incl_scan(v);
    if (lane == 63) {
      wave_tot[0][wave] = ip;
      wave_tot[1][wave] = iv;
    }
    __syncthreads();
    uint32_t base_p = carry_p, tot_p = 0, tot_v = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
      base_p += w < wave ? wave_tot[0][w] : 0u;
      tot_p += wave_tot[0][w];
      tot_v += wave_tot[1][w];
    }
    if (c < n_chunks) chunk[2 * (size_t)c] = base_p + ip - p;
    carry_p += tot_p;
    carry_v += tot_v;
    __syncthreads();  // wave_tot is rewritten by the next round
  }
  if (threadIdx.x == 0) {
    const uint32_t total = carry_p;
    dc->n_pairs_total = total;
    dc->n_pairs = total < max_pairs ? total : max_pairs;
    dc->n_visible = carry_v;
    if (total > max_pairs) dc->overflow |= HIGS_OVF_PAIRS;
    // when the key (macro-tile and depth bits, plus one bit of headroom for
    // the segment search's end target) and the gaussian id fit one 64-bit
    // word, a pair is that word alone: the sort moves 8 bytes per pair
    // instead of 12, and ties still break by id
    const int kbits = mt_bits + (int)depth_bits(dc->key_min, dc->key_max) + 1;
    dc->id_shift = (id_bits > 0 && kbits + id_bits <= 64) ? (uint32_t)id_bits : 0u;
  }
}

hipError_t launch_scan(int64_t n, const uint32_t* cnt, uint32_t* block_sums, uint32_t max_pairs,
                       int mt_bits, bool allow_one_word, DeviceCounters* dc, hipStream_t s) {
  (void)cnt;
  const int64_t n_blocks = (n + kProjBlock - 1) / kProjBlock;
  int id_bits = 0;  // bits of the largest gaussian id (0: two-array pairs)
  if (allow_one_word)
    for (int64_t v = n > 1 ? n - 1 : 0; v; v >>= 1) ++id_bits;
  const uint32_t n_chunks = (uint32_t)scan_chunks(n_blocks);
  if (n_chunks > 0)
    hipLaunchKernelGGL(chunk_sum_kernel, dim3(n_chunks), dim3(kScanChunk), 0, s,
                       (uint32_t)n_blocks, block_sums);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, s, n_chunks,
                     block_sums + 2 * n_blocks, max_pairs, mt_bits, id_bits, dc);
  return hipGetLastError();
}

// One workgroup per kFillBlocks consecutive projection blocks (256 gaussians
// each, one per thread per block): every count, span word and depth key of
// the group is loaded first; the group's block offsets are its chunk's offset
// plus a workgroup scan of the chunk's block sums (one per thread); then each
// block's pairs are written at its offset plus the wave prefix sums.
constexpr int kFillBlocks = kFillGroup;
static_assert(kScanChunk == kProjBlock && kScanChunk % kFillBlocks == 0,
              "one chunk block per fill thread; a fill group never straddles chunks");
__global__ void __launch_bounds__(kProjBlock)
fill_kernel(int64_t n, CamArgs cam, int64_t n_pad, uint32_t n_mt,
            const float* __restrict__ f_mx, const float* __restrict__ f_my,
            const float* __restrict__ f_a, const float* __restrict__ f_b,
            const float* __restrict__ f_c, const float* __restrict__ f_tau,
            const uint32_t* __restrict__ f_key, const uint32_t* __restrict__ f_cnt,
            const uint32_t* __restrict__ f_span, const uint32_t* __restrict__ block_sums,
            uint32_t max_pairs, const DeviceCounters* __restrict__ dc,
            uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ uint32_t wave_tot[kFillBlocks][kProjBlock / 64];
  __shared__ uint32_t chunk_wave[kProjBlock / 64];
  __shared__ uint32_t chunk_excl[kScanChunk];
  if (dc->overflow) return;  // the frame stops at a capacity overflow
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t blk0 = (int64_t)blockIdx.x * kFillBlocks;
  const int64_t n_blocks = (n + kProjBlock - 1) / kProjBlock;
  const int64_t ch = blk0 / kScanChunk;
  const int64_t cb = ch * kScanChunk + threadIdx.x;  // this thread's block of the chunk
  const uint32_t cp = cb < n_blocks ? block_sums[2 * cb] : 0u;
  const uint32_t chunk_base = block_sums[2 * n_blocks + 2 * ch];  // scanned chunk totals
  uint32_t cnt[kFillBlocks], span[kFillBlocks], key[kFillBlocks], incl[kFillBlocks];
#pragma unroll
  for (int k = 0; k < kFillBlocks; ++k) {
    const int64_t i = (blk0 + k) * kProjBlock + threadIdx.x;
    const bool in = i < n;
    cnt[k] = in ? f_cnt[i] : 0u;
    span[k] = in ? f_span[i] : 0u;
    key[k] = in ? f_key[i] : 0u;
  }
  // exclusive scan of the chunk's block pair counts
  const uint32_t ci = wave_incl_scan(cp);
  if (lane == 63) chunk_wave[wave] = ci;
#pragma unroll
  for (int k = 0; k < kFillBlocks; ++k) {
    incl[k] = wave_incl_scan(cnt[k]);
    if (lane == 63) wave_tot[k][wave] = incl[k];
  }
  __syncthreads();
  uint32_t ce = ci - cp;
  for (int w = 0; w < wave; ++w) ce += chunk_wave[w];
  chunk_excl[threadIdx.x] = ce;
  __syncthreads();
  uint32_t boff[kFillBlocks];
#pragma unroll
  for (int k = 0; k < kFillBlocks; ++k)
    boff[k] = chunk_base + chunk_excl[blk0 + k - ch * kScanChunk];
  const uint32_t dmin = dc->key_min;
  const uint32_t dbits = depth_bits(dmin, dc->key_max);
  const uint32_t ish = dc->id_shift;
  // the view's first macro-tile: views own whole fill groups of blocks, so
  // one uniform division serves the group
  const uint32_t mt0 = (uint32_t)(blk0 / (n_pad / kProjBlock)) * n_mt;
#pragma unroll
  for (int k = 0; k < kFillBlocks; ++k) {
    if (__ballot(cnt[k] > 0) == 0) continue;  // whole wave invisible in this block
    uint32_t at = boff[k] + incl[k] - cnt[k];
    for (int w = 0; w < wave; ++w) at += wave_tot[k][w];
    if (cnt[k] == 0) continue;
    const int64_t i = (blk0 + k) * kProjBlock + threadIdx.x;
    const uint64_t depth = (uint64_t)(key[k] - dmin);
    const uint32_t gid = (uint32_t)i;  // virtual: the view's range, then the gaussian
    auto emit = [&](uint32_t mt) {
      if (at < max_pairs) {
        const uint64_t key = ((uint64_t)(mt0 + mt) << dbits) | depth;
        if (ish) {
          keys[at] = (key << ish) | gid;
        } else {
          keys[at] = key;
          vals[at] = gid;
        }
      }
      ++at;
    };
    if (span[k]) {  // the list the projection recorded
      visit_span(span[k], cam.n_mt_x, emit);
    } else {  // a long list: the predicate again, on the same fields
      BinFields f;
      f.mx = f_mx[i];
      f.my = f_my[i];
      f.a = f_a[i];
      f.b = f_b[i];
      f.c = f_c[i];
      f.tau = f_tau[i];
      visit_macro_tiles(f, cam.width, cam.height, cam.n_mt_x, cam.n_mt_y, emit);
    }
  }
}

hipError_t launch_fill(int64_t n, CamArgs cam, int64_t n_pad, uint32_t n_mt, const float* f_mx,
                       const float* f_my,
                       const float* f_a, const float* f_b, const float* f_c, const float* f_tau,
                       const uint32_t* f_key, const uint32_t* f_cnt, const uint32_t* f_span,
                       const uint32_t* block_sums, uint32_t max_pairs,
                       const DeviceCounters* dc, uint64_t* keys, uint32_t* vals, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t n_blocks = (n + kProjBlock - 1) / kProjBlock;
  const unsigned blocks = (unsigned)((n_blocks + kFillBlocks - 1) / kFillBlocks);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(kProjBlock), 0, s, n, cam, n_pad, n_mt, f_mx,
                     f_my, f_a, f_b, f_c, f_tau, f_key, f_cnt, f_span, block_sums, max_pairs, dc,
                     keys, vals);
  return hipGetLastError();
}

}  // namespace higs
