// Stage 2a: (macro-tile, gaussian) pair emission (sec. 3.2 and sec. 4.3:
// count, prefix sum, fill).
//
// The per-gaussian pair counts come from the projection kernel.  `fill_kernel`
// claims its 256-gaussian blocks in order from a device counter, scans the
// counts inside the block with wave prefix sums, and turns the block total
// into a global offset with a decoupled look-back over the preceding blocks
// (each block publishes its total, then its inclusive prefix, in an
// epoch-tagged 64-bit word): one pass, no separate scan kernel.  It then re-runs
// the intersection of each gaussian from the stored float32 fields (the count
// pass's exact decisions) and writes pairs in gaussian-id order, macro-tiles
// ascending within a gaussian.  Waves whose 64 gaussians are all invisible skip
// the fields entirely (ballot).
//
// Key layout: (macro-tile << dbits) | (depth bits - dmin), where dmin and
// dmin + 2^dbits - 1 bracket the float32 depth bits of the frame's visible
// gaussians (found by the projection).  The map is monotone in (macro-tile,
// depth), so the sort order is unchanged, and the key has dbits + log2(n_mt)
// significant bits instead of 32 + log2(n_mt): a 1080p frame over a depth range
// of a few units sorts in five 8-bit passes rather than six.
#include "higs_internal.h"
#include "predicate.h"

namespace higs {

__global__ void clear_kernel(DeviceCounters* dc, uint32_t* hist, int n_hist) {
  uint32_t* w = reinterpret_cast<uint32_t*>(dc);
  const int nw = (int)(sizeof(DeviceCounters) / 4);
  for (int k = threadIdx.x; k < nw; k += blockDim.x) w[k] = 0;
  for (int k = threadIdx.x; k < n_hist; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  if (threadIdx.x == 0) dc->key_min = 0xffffffffu;
}

hipError_t launch_clear(DeviceCounters* dc, uint32_t* hist, int n_hist, hipStream_t s) {
  hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(256), 0, s, dc, hist, n_hist);
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

__device__ __forceinline__ uint64_t scan_word(uint32_t epoch, uint32_t flag, uint32_t count) {
  return ((uint64_t)epoch << 34) | ((uint64_t)flag << 32) | (uint64_t)count;
}

__global__ void __launch_bounds__(kProjBlock)
fill_kernel(int64_t n, CamArgs cam, const float* __restrict__ f_mx, const float* __restrict__ f_my,
            const float* __restrict__ f_a, const float* __restrict__ f_b,
            const float* __restrict__ f_c, const float* __restrict__ f_tau,
            const uint32_t* __restrict__ f_key, const uint32_t* __restrict__ f_cnt,
            uint64_t* __restrict__ scan_status, uint32_t epoch, uint32_t max_pairs,
            DeviceCounters* __restrict__ dc, uint64_t* __restrict__ keys,
            uint32_t* __restrict__ vals) {
  __shared__ uint32_t wave_tot[kProjBlock / 64], wave_vis[kProjBlock / 64];
  __shared__ uint32_t s_bid, s_base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_bid = atomicAdd(&dc->fill_next, 1u);
  __syncthreads();
  const uint32_t bid = s_bid;
  const uint32_t n_blocks = (uint32_t)((n + kProjBlock - 1) / kProjBlock);
  const int64_t i = (int64_t)bid * kProjBlock + threadIdx.x;
  const uint32_t cnt = i < n ? f_cnt[i] : 0u;
  const uint32_t incl = wave_incl_scan(cnt);
  const uint64_t vis = __ballot(cnt > 0);
  if (lane == 63) wave_tot[wave] = incl;
  if (lane == 0) wave_vis[wave] = (uint32_t)__popcll(vis);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0, nvis = 0;
    for (int w = 0; w < kProjBlock / 64; ++w) {
      tot += wave_tot[w];
      nvis += wave_vis[w];
    }
    if (nvis) atomicAdd(&dc->n_visible, nvis);
    uint64_t* mine = scan_status + bid;
    uint32_t prefix = 0;
    if (bid == 0) {
      __hip_atomic_store(mine, scan_word(epoch, kFlagPrefix, tot), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(mine, scan_word(epoch, kFlagAggregate, tot), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      int64_t t = (int64_t)bid - 1;
      uint32_t spins = 0;
      while (t >= 0) {
        const uint64_t w = __hip_atomic_load(scan_status + t, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t flag = (uint32_t)(w >> 32) & 3u;
        if ((uint32_t)(w >> 34) != epoch || flag == 0) {  // not published yet
          if (++spins > kMaxSpins) {  // cannot happen unless a block was lost
            atomicOr(&dc->overflow, kErrSortStall);
            break;
          }
          continue;
        }
        prefix += (uint32_t)w;
        if (flag == kFlagPrefix) break;
        --t;
      }
      __hip_atomic_store(mine, scan_word(epoch, kFlagPrefix, prefix + tot), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    s_base = prefix;
    if (bid == n_blocks - 1) {
      const uint32_t total = prefix + tot;
      dc->n_pairs_total = total;
      dc->n_pairs = total < max_pairs ? total : max_pairs;
      if (total > max_pairs) atomicOr(&dc->overflow, (uint32_t)HIGS_OVF_PAIRS);
    }
  }
  __syncthreads();
  if (vis == 0) return;  // whole wave invisible
  if (cnt == 0) return;
  uint32_t at = s_base + incl - cnt;
  for (int w = 0; w < wave; ++w) at += wave_tot[w];
  BinFields f;
  f.mx = f_mx[i];
  f.my = f_my[i];
  f.a = f_a[i];
  f.b = f_b[i];
  f.c = f_c[i];
  f.tau = f_tau[i];
  const uint32_t dmin = dc->key_min;
  const uint32_t dbits = depth_bits(dc->key_min, dc->key_max);
  const uint64_t depth = (uint64_t)(f_key[i] - dmin);
  const uint32_t gid = (uint32_t)i;
  visit_macro_tiles(f, cam.width, cam.height, cam.n_mt_x, cam.n_mt_y, [&](uint32_t mt) {
    if (at < max_pairs) {
      keys[at] = ((uint64_t)mt << dbits) | depth;
      vals[at] = gid;
    }
    ++at;
  });
}

hipError_t launch_fill(int64_t n, CamArgs cam, const float* f_mx, const float* f_my,
                       const float* f_a, const float* f_b, const float* f_c, const float* f_tau,
                       const uint32_t* f_key, const uint32_t* f_cnt, uint64_t* scan_status,
                       uint32_t epoch, uint32_t max_pairs, DeviceCounters* dc, uint64_t* keys,
                       uint32_t* vals, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + kProjBlock - 1) / kProjBlock);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(kProjBlock), 0, s, n, cam, f_mx, f_my, f_a,
                     f_b, f_c, f_tau, f_key, f_cnt, scan_status, epoch, max_pairs, dc, keys, vals);
  return hipGetLastError();
}

}  // namespace higs
