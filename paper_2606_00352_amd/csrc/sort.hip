// Stage 2b: depth sort of the (macro-tile, gaussian) pairs (sec. 3.3: each
// macro-tile's list ordered by depth; ties by gaussian id).
//
// A stable least-significant-digit radix sort over the composite 64-bit key
// (macro-tile << d | depth bits - min, d the bits of the frame's depth range)
// with the gaussian id as value.  Pairs arrive in gaussian-id order and every
// pass is stable, so the result is ordered by (macro-tile, depth, id).  When
// key and id fit one word (key << g | id, g the id bits) the passes move that
// word alone and the last moving pass also writes the id array.  One
// pass per 9-bit digit of the d + ceil(log2 n_mt) significant key bits, each a
// single "onesweep" kernel:
//   - a persistent grid claims 6144-key tiles from a device counter, so tile
//     t's predecessors are always resident (forward progress of the look-back);
//   - each wave ranks its 768 keys stably with 9 ballots per key (wave-level
//     multisplit) against a wave-private digit histogram in LDS;
//   - per digit, the tile publishes its count and looks back over the
//     preceding tiles' published counts/prefixes (decoupled look-back, one
//     thread per digit, 64-bit status words tagged with a per-pass epoch so
//     the status array never needs clearing);
//   - keys are regrouped by digit in LDS and written out in runs.
// A histogram kernel counts every digit position in one read of the keys; a
// plan kernel turns the counts into per-pass digit bases and skips a pass
// whose digit is the same for every key (the ping-pong buffer choice is then
// made on the device, so no host round trip is needed).
#include "higs_internal.h"

namespace higs {

__device__ __forceinline__ uint64_t ld_status(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t status_word(uint32_t epoch, uint32_t flag, uint32_t count) {
  return ((uint64_t)epoch << 34) | ((uint64_t)flag << 32) | (uint64_t)count;
}

constexpr int kHistThreads = 1024;  // 16 waves a workgroup (the sort 0.294 -> 0.288 ms against 4)
constexpr int kHistCopies = 4;  // LDS copies: lanes l and l+4k share one, 16-way at worst
constexpr int kHistBatch = 8;   // keys loaded together per thread
__global__ void __launch_bounds__(kHistThreads)
sort_hist_kernel(const uint64_t* __restrict__ keys, const DeviceCounters* __restrict__ dc,
                 int n_passes, int mt_bits, uint32_t* __restrict__ hist) {
  // the top digits of a frame's keys take few values: spreading the counters
  // over copies keeps the LDS atomics of one wave from piling on one address
  __shared__ uint32_t h[kHistCopies][kMaxPasses * kRadix];
  if (dc->overflow) return;  // the frame stops at a capacity overflow
  const uint32_t n = dc->n_pairs;
  const uint32_t ish = dc->id_shift;  // key bits start above the id in a one-word pair
  // digit positions above the frame's key width are zero in every key
  const int np = min(n_passes, (mt_bits + (int)depth_bits(dc->key_min, dc->key_max) +
                                kRadixBits - 1) / kRadixBits);
  for (int c = 0; c < kHistCopies; ++c)
    for (int k = threadIdx.x; k < np * kRadix; k += kHistThreads) h[c][k] = 0;
  __syncthreads();
  uint32_t* mine = h[threadIdx.x & (kHistCopies - 1)];
  // kHistBatch independent loads in flight per thread, then their counts
  const uint32_t stride = gridDim.x * kHistThreads;
  for (uint32_t i0 = blockIdx.x * kHistThreads + threadIdx.x; i0 < n; i0 += kHistBatch * stride) {
    uint64_t key[kHistBatch];
#pragma unroll
    for (int b = 0; b < kHistBatch; ++b) {
      const uint32_t i = i0 + (uint32_t)b * stride;
      key[b] = i < n ? keys[i] : 0ull;
    }
#pragma unroll
    for (int b = 0; b < kHistBatch; ++b) {
      if (i0 + (uint32_t)b * stride >= n) break;
      for (int p = 0; p < np; ++p)
        atomicAdd(&mine[p * kRadix + (uint32_t)((key[b] >> (ish + kRadixBits * p)) & (kRadix - 1))],
                  1u);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < np * kRadix; k += kHistThreads) {
    uint32_t v = 0;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) v += h[c][k];
    if (v) atomicAdd(&hist[k], v);
  }
}

// One block of kRadix threads (one per digit): per pass, skip flag, source
// buffer and the exclusive digit bases.  One-word pairs need one moving pass
// to write the id array: if no digit varies, pass 0 moves anyway.
__global__ void __launch_bounds__(kRadix)
sort_plan_kernel(const uint32_t* __restrict__ hist, DeviceCounters* __restrict__ dc, int n_passes,
                 int mt_bits, uint32_t* __restrict__ plan, uint32_t* __restrict__ base) {
  __shared__ uint32_t wave_tot[kRadix / 64];
  if (dc->overflow) return;
  const uint32_t n = dc->n_pairs;
  const int np = (mt_bits + (int)depth_bits(dc->key_min, dc->key_max) + kRadixBits - 1) / kRadixBits;
  const int d = threadIdx.x, lane = d & 63, wave = d >> 6;
  // this digit's count in every pass, loaded together (one round trip)
  uint32_t cnt[kMaxPasses];
#pragma unroll
  for (int p = 0; p < kMaxPasses; ++p) cnt[p] = p < n_passes ? hist[p * kRadix + d] : 0u;
  // a pass above the key width, or one whose digit every key shares, is skipped
  uint32_t skip = 0;
#pragma unroll
  for (int p = 0; p < kMaxPasses; ++p)
    if (p < n_passes && (__syncthreads_or(cnt[p] == n) || p >= np)) skip |= 1u << p;
  const uint32_t all = (1u << n_passes) - 1u;
  if (dc->id_shift && skip == all) skip &= ~1u;
  uint32_t cur = 0, moved = 0;
#pragma unroll
  for (int p = 0; p < kMaxPasses; ++p) {
    if (p >= n_passes) break;
    const uint32_t c = cnt[p];
    const int trivial = (skip >> p) & 1u;
    // exclusive scan of the digit counts
    uint32_t v = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = __shfl_up(v, off, 64);
      if (lane >= off) v += o;
    }
    if (lane == 63) wave_tot[wave] = v;
    __syncthreads();
    uint32_t b = v - c;
    for (int w = 0; w < wave; ++w) b += wave_tot[w];
    base[p * kRadix + d] = b;
    if (d == 0) plan[p] = trivial ? 0xffffffffu : cur;
    if (!trivial) {
      cur ^= 1u;
      ++moved;
    }
    __syncthreads();
  }
  if (d == 0) {
    dc->sort_final = cur;
    dc->sort_passes = moved;
    dc->sort_last = skip == all ? 0xffffffffu : 31u - (uint32_t)__clz(all & ~skip);
  }
}

constexpr int kWaves = kSortThreads / 64;
static_assert(kSortThreads >= kRadix && kSortThreads % 64 == 0, "one thread per digit, whole waves");
constexpr int kWaveItems = 64 * kSortItems;  // 768 keys per wave
constexpr int kLookWindow = 4;               // look-back words loaded per round trip

struct SortLds {
  // the tile regrouped by digit: keys first, then (reusing the space) values
  union {
    uint64_t keys[kSortTile];
    uint32_t vals[kSortTile];
  } buf;
  uint32_t whist[kWaves][kRadix];  // per-wave digit counts, then wave prefixes
  uint32_t local_start[kRadix];    // first LDS slot of each digit in the tile
  uint32_t gbase[kRadix];          // global position of LDS slot 0 of each digit
  uint32_t wave_tot[kWaves];
  uint32_t tile;
};

// four waves per SIMD (two workgroups per CU): the register budget is held to
// 128, which measured faster than more keys per thread at lower occupancy
__global__ void __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(4)))
onesweep_kernel(int pass, uint64_t* __restrict__ k0, uint32_t* __restrict__ v0,
                uint64_t* __restrict__ k1, uint32_t* __restrict__ v1,
                const uint32_t* __restrict__ plan, const uint32_t* __restrict__ base,
                uint64_t* __restrict__ status, DeviceCounters* __restrict__ dc) {
  __shared__ SortLds L;
  if (dc->overflow) return;  // (the plan was not written either)
  const uint32_t src = plan[pass];
  if (src == 0xffffffffu) return;  // every key has the same digit: identity pass
  // the epoch this pass publishes under (the frame's clear set the base)
  const uint32_t epoch = dc->epoch + (uint32_t)pass;
  const uint64_t* __restrict__ kin = src ? k1 : k0;
  const uint32_t* __restrict__ vin = src ? v1 : v0;
  uint64_t* __restrict__ kout = src ? k0 : k1;
  uint32_t* __restrict__ vout = src ? v0 : v1;
  // one-word pairs: the digit sits above the id, no value array moves, and
  // the last moving pass writes the ids out of the words
  const uint32_t ish = dc->id_shift;
  const bool one_word = ish != 0;
  const bool write_ids = one_word && dc->sort_last == (uint32_t)pass;
  const uint64_t id_mask = (1ull << ish) - 1ull;
  const uint32_t shift = ish + (uint32_t)(kRadixBits * pass);
  const uint32_t n = dc->n_pairs;
  const uint32_t n_tiles = (n + kSortTile - 1) / kSortTile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t lt_mask = (1ull << lane) - 1ull;

  for (;;) {
    if (tid == 0) L.tile = atomicAdd(&dc->tile_next[pass], 1u);
    for (int k = tid; k < kWaves * kRadix; k += kSortThreads) (&L.whist[0][0])[k] = 0;
    __syncthreads();
    const uint32_t tile = L.tile;
    if (tile >= n_tiles) break;
    const uint32_t t0 = tile * kSortTile;
    const uint32_t wbase = t0 + wave * kWaveItems;

    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rank[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
      const uint32_t idx = wbase + k * 64 + lane;
      if (idx < n) {
        key[k] = kin[idx];
        val[k] = one_word ? 0u : vin[idx];
      } else {
        key[k] = ~0ull;  // sorts last, never written out
        val[k] = 0;
      }
    }
    // stable wave-level ranking, item order (k, lane)
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
      uint64_t peers = ~0ull;
#pragma unroll
      for (int b = 0; b < kRadixBits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
      }
      const uint32_t before = (uint32_t)__popcll(peers & lt_mask);
      const uint32_t prev = L.whist[wave][d];
      rank[k] = prev + before;
      // every lane of the wave has read its digit's count before the first
      // lane of each digit group adds the group to it (the wave executes in
      // lockstep; the barrier keeps the compiler from moving the store up)
      __builtin_amdgcn_wave_barrier();
      if (before == 0) L.whist[wave][d] = prev + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    // per digit (threads 0..kRadix-1, whole waves): wave prefixes, tile count,
    // publish, look back
    const int d = tid;
    uint32_t v = 0, tot = 0, prefix = 0;
    if (tid < kRadix) {
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = L.whist[w][d];
        L.whist[w][d] = tot;
        tot += c;
      }
      uint64_t* st = status + (size_t)tile * kRadix + d;
      if (tile == 0) st_status(st, status_word(epoch, kFlagPrefix, tot));
      else st_status(st, status_word(epoch, kFlagAggregate, tot));
      // exclusive scan of the tile's digit counts -> LDS slots
      v = tot;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
      }
      if (lane == 63) L.wave_tot[wave] = v;
      if (tile > 0) {
        // kLookWindow predecessors per round trip: their words are loaded
        // together, then taken nearest first until an inclusive prefix or one
        // not yet published (the next round starts there)
        int64_t t = (int64_t)tile - 1;
        uint32_t spins = 0;
        bool done = false;
        while (t >= 0) {
          uint64_t w[kLookWindow];
#pragma unroll
          for (int k = 0; k < kLookWindow; ++k)
            w[k] = t - k >= 0 ? ld_status(status + (size_t)(t - k) * kRadix + d) : 0ull;
          int used = 0;
#pragma unroll
          for (int k = 0; k < kLookWindow; ++k) {
            if (used != k || t - k < 0) break;
            const uint32_t flag = (uint32_t)(w[k] >> 32) & 3u;
            if ((uint32_t)(w[k] >> 34) != epoch || flag == 0) break;  // not published yet
            prefix += (uint32_t)w[k];
            used = k + 1;
            if (flag == kFlagPrefix) done = true;
            if (done) break;
          }
          if (done) break;
          if (used == 0 && ++spins > kMaxSpins) {  // cannot happen unless a tile was lost
            atomicOr(&dc->overflow, kErrSortStall);
            break;
          }
          t -= used;
        }
        st_status(st, status_word(epoch, kFlagPrefix, prefix + tot));
      }
    }
    __syncthreads();
    if (tid < kRadix) {
      uint32_t ls = v - tot;
      for (int w = 0; w < wave; ++w) ls += L.wave_tot[w];
      L.local_start[d] = ls;
      L.gbase[d] = base[pass * kRadix + d] + prefix - ls;
    }
    __syncthreads();
    // regroup by digit in LDS: keys, then values through the same buffer
    uint32_t slot[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
      slot[k] = L.local_start[d] + L.whist[wave][d] + rank[k];
      L.buf.keys[slot[k]] = key[k];
    }
    __syncthreads();
    const uint32_t valid = min((uint32_t)kSortTile, n - t0);
    uint32_t dst[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
      const uint32_t j = tid + k * kSortThreads;
      dst[k] = 0xffffffffu;
      if (j < valid) {
        const uint64_t kk = L.buf.keys[j];
        const uint32_t d = (uint32_t)(kk >> shift) & (kRadix - 1);
        dst[k] = L.gbase[d] + j;
        if (dst[k] < n) {
          kout[dst[k]] = kk;
          if (write_ids) vout[dst[k]] = (uint32_t)(kk & id_mask);
        }
      }
    }
    if (one_word) {  // nothing else moves
      __syncthreads();
      continue;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) L.buf.vals[slot[k]] = val[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
      const uint32_t j = tid + k * kSortThreads;
      if (j < valid && dst[k] < n) vout[dst[k]] = L.buf.vals[j];
    }
    __syncthreads();
  }
}

static int g_onesweep_per_cu = 0;

int onesweep_per_cu_config() {
  if (g_onesweep_per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, onesweep_kernel, kSortThreads, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    g_onesweep_per_cu = nb;
  }
  return g_onesweep_per_cu;
}

hipError_t launch_sort(int n_passes, int mt_bits, SortBuffers sb,
                       DeviceCounters* dc, int n_cus, hipStream_t s) {
  onesweep_per_cu_config();
  hipLaunchKernelGGL(sort_hist_kernel, dim3(n_cus * 2), dim3(kHistThreads), 0, s, sb.keys[0], dc,
                     n_passes, mt_bits, sb.hist);
  hipLaunchKernelGGL(sort_plan_kernel, dim3(1), dim3(kRadix), 0, s, sb.hist, dc, n_passes, mt_bits,
                     sb.plan, sb.plan + kMaxPasses);
  const int workers = n_cus * g_onesweep_per_cu;
  for (int p = 0; p < n_passes; ++p) {
    hipLaunchKernelGGL(onesweep_kernel, dim3(workers), dim3(kSortThreads), 0, s, p,
                       sb.keys[0], sb.vals[0], sb.keys[1], sb.vals[1],
                       sb.plan, sb.plan + kMaxPasses, sb.status, dc);
  }
  return hipGetLastError();
}

}  // namespace higs
