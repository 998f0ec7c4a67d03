// Stage 3: macro-tile segments and the batch table (sec. 3.1: a macro-tile
// holding n gaussians spawns ceil(n / B_r) processing units).
//
// `mt_offsets_kernel`: one wave per macro-tile finds the first sorted pair of
// that macro-tile with a 64-ary search (each step probes 64 evenly spaced
// keys and keeps the bracket where the predicate flips), so a 10^7-pair list
// takes four dependent loads per macro-tile.
// `batch_table_kernel` (one workgroup): batches per macro-tile and their
// exclusive scan (first batch of every macro-tile); `batch_rows_kernel` (a
// wave per macro-tile) writes the (macro-tile, start, length) rows in
// (macro-tile, batch) order.
#include "higs_internal.h"

namespace higs {

constexpr int kOffThreads = 256;
__global__ void __launch_bounds__(kOffThreads)
mt_offsets_kernel(int n_mt, const uint64_t* __restrict__ k0, const uint64_t* __restrict__ k1,
                  const DeviceCounters* __restrict__ dc, uint32_t* __restrict__ mt_off) {
  const int m = blockIdx.x * (kOffThreads / 64) + (threadIdx.x >> 6);
  if (m > n_mt || dc->overflow) return;
  const int lane = threadIdx.x & 63;
  const uint64_t* __restrict__ keys = dc->sort_final ? k1 : k0;
  // keys are macro-tile << d | depth, shifted above the id in one-word pairs
  const uint64_t target = (uint64_t)m << (depth_bits(dc->key_min, dc->key_max) + dc->id_shift);
  uint32_t lo = 0, hi = dc->n_pairs;  // answer in [lo, hi]
  while (hi - lo > 64) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t p = lo + (uint32_t)lane * step;
    const bool below = p < hi && keys[p] < target;
    const uint32_t c = (uint32_t)__popcll(__ballot(below));
    if (c == 0) {
      hi = lo;
    } else {
      const uint32_t nlo = lo + (c - 1) * step + 1;
      const uint32_t nhi = lo + c * step;
      lo = nlo;
      hi = nhi < hi ? nhi : hi;
    }
  }
  const uint32_t p = lo + (uint32_t)lane;
  const bool below = p < hi && keys[p] < target;
  const uint32_t c = (uint32_t)__popcll(__ballot(below));
  if (lane == 0) mt_off[m] = lo + c;
}

constexpr int kBtThreads = 1024;
// Exclusive scan of one value per thread over the workgroup.
__device__ __forceinline__ uint32_t bt_scan(uint32_t mine, uint32_t* wave_tot) {
  uint32_t v = mine;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  __syncthreads();
  if (lane == 63) wave_tot[wave] = v;
  __syncthreads();
  uint32_t run = v - mine;
  for (int w = 0; w < wave; ++w) run += wave_tot[w];
  return run;
}

// The first batch of every macro-tile, and the raster work items: each
// macro-tile's batches cut into runs of `chain` and a shorter remainder, or
// (whole) every macro-tile with all its batches, empty ones included.  The
// items are counted by length (lengths above kMaxChain count as kMaxChain) and
// listed longest first (the rasteriser claims them in list order, so a long
// one does not end the frame alone); within a length the order is that of the
// LDS cursor claims, which no result depends on.
__global__ void __launch_bounds__(kBtThreads)
batch_table_kernel(int n_mt, uint32_t cap, uint32_t chain, bool whole, uint32_t max_batches,
                   const uint32_t* __restrict__ mt_off, DeviceCounters* __restrict__ dc,
                   uint32_t* __restrict__ batch_first, uint32_t* __restrict__ chain_tab) {
  __shared__ uint32_t wave_tot[kBtThreads / 64];
  __shared__ uint32_t n_len[kMaxChain + 1];  // items of each length, then their next slot
  __shared__ uint32_t total;
  if (dc->overflow) return;  // pairs were cut: no batch table for this frame
  if (threadIdx.x <= kMaxChain) n_len[threadIdx.x] = 0u;
  const int per = (n_mt + kBtThreads - 1) / kBtThreads;
  const int m0 = threadIdx.x * per;
  const int m1 = min(m0 + per, n_mt);
  uint32_t mine = 0;
  for (int m = m0; m < m1; ++m) mine += (mt_off[m + 1] - mt_off[m] + cap - 1) / cap;
  const uint32_t run0 = bt_scan(mine, wave_tot);  // (its first barrier orders n_len's clearing)
  uint32_t run = run0;
  for (int m = m0; m < m1; ++m) {
    const uint32_t nb = (mt_off[m + 1] - mt_off[m] + cap - 1) / cap;
    batch_first[m] = run;
    run += nb;
    if (whole) {
      atomicAdd(&n_len[min(nb, (uint32_t)kMaxChain)], 1u);
    } else {
      if (nb >= chain) atomicAdd(&n_len[chain], nb / chain);
      if (nb % chain) atomicAdd(&n_len[nb % chain], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x == kBtThreads - 1) {
    uint32_t at = 0;
    for (int l = whole ? kMaxChain : (int)chain; l >= (whole ? 0 : 1); --l) {
      const uint32_t c = n_len[l];
      n_len[l] = at;
      at += c;
    }
    total = run;
    batch_first[n_mt] = run;
    dc->n_batches_total = run;
    dc->n_batches = run < max_batches ? run : max_batches;
    dc->n_chains = run > max_batches ? 0u : at;
    if (run > max_batches) dc->overflow |= HIGS_OVF_BATCHES;
  }
  __syncthreads();
  if (total > max_batches) return;  // (uniform) the frame stops; no work items
  // the rows: items <= batches (+ macro-tiles when whole), the table's rows
  uint32_t first = run0;
  for (int m = m0; m < m1; ++m) {
    const uint32_t nb = (mt_off[m + 1] - mt_off[m] + cap - 1) / cap;
    if (whole) {
      const uint32_t at = atomicAdd(&n_len[min(nb, (uint32_t)kMaxChain)], 1u);
      chain_tab[3 * at + 0] = (uint32_t)m;
      chain_tab[3 * at + 1] = first;
      chain_tab[3 * at + 2] = nb;
    } else {
      const uint32_t n_full = nb / chain, rest = nb - n_full * chain;
      if (n_full) {
        const uint32_t at = atomicAdd(&n_len[chain], n_full);
        for (uint32_t c = 0; c < n_full; ++c) {
          chain_tab[3 * (at + c) + 0] = (uint32_t)m;
          chain_tab[3 * (at + c) + 1] = first + c * chain;
          chain_tab[3 * (at + c) + 2] = chain;
        }
      }
      if (rest) {
        const uint32_t at = atomicAdd(&n_len[rest], 1u);
        chain_tab[3 * at + 0] = (uint32_t)m;
        chain_tab[3 * at + 1] = first + n_full * chain;
        chain_tab[3 * at + 2] = rest;
      }
    }
    first += nb;
  }
}

// The (macro-tile, start, length) rows: one wave per macro-tile, a lane per
// batch.
__global__ void __launch_bounds__(kOffThreads)
batch_rows_kernel(int n_mt, uint32_t cap, uint32_t max_batches,
                  const uint32_t* __restrict__ mt_off, const uint32_t* __restrict__ batch_first,
                  const DeviceCounters* __restrict__ dc, uint32_t* __restrict__ tab) {
  const int m = blockIdx.x * (kOffThreads / 64) + (threadIdx.x >> 6);
  if (m >= n_mt || dc->overflow) return;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t off = mt_off[m];
  const uint32_t len = mt_off[m + 1] - off;
  const uint32_t nb = (len + cap - 1) / cap;
  const uint32_t first = batch_first[m];
  for (uint32_t b = lane; b < nb; b += 64) {
    const uint32_t idx = first + b;
    if (idx < max_batches) {
      tab[3 * idx + 0] = (uint32_t)m;
      tab[3 * idx + 1] = off + b * cap;
      tab[3 * idx + 2] = min(cap, len - b * cap);
    }
  }
}

// batch_first and the work items by one workgroup, then the batch rows by a
// wave per macro-tile
static void launch_table(int n_mt, uint32_t batch_cap, uint32_t max_batches, DeviceCounters* dc,
                         const uint32_t* mt_off, uint32_t* batch_first, uint32_t* batch_tab,
                         ChainBuffers cb, hipStream_t s) {
  hipLaunchKernelGGL(batch_table_kernel, dim3(1), dim3(kBtThreads), 0, s, n_mt, batch_cap, cb.chain,
                     cb.whole, max_batches, mt_off, dc, batch_first, cb.tab);
  const int row_blocks = (n_mt + (kOffThreads / 64) - 1) / (kOffThreads / 64);
  if (row_blocks > 0)
    hipLaunchKernelGGL(batch_rows_kernel, dim3(row_blocks), dim3(kOffThreads), 0, s, n_mt,
                       batch_cap, max_batches, mt_off, batch_first, dc, batch_tab);
}

hipError_t launch_batch(int n_mt, uint32_t batch_cap, uint32_t max_batches, const uint64_t* const* keys2,
                        DeviceCounters* dc, uint32_t* mt_off, uint32_t* batch_first,
                        uint32_t* batch_tab, ChainBuffers cb, hipStream_t s) {
  const int waves = n_mt + 1;
  const int blocks = (waves + (kOffThreads / 64) - 1) / (kOffThreads / 64);
  hipLaunchKernelGGL(mt_offsets_kernel, dim3(blocks), dim3(kOffThreads), 0, s, n_mt, keys2[0],
                     keys2[1], dc, mt_off);
  launch_table(n_mt, batch_cap, max_batches, dc, mt_off, batch_first, batch_tab, cb, s);
  return hipGetLastError();
}

hipError_t launch_batch_from_offsets(int n_mt, uint32_t batch_cap, uint32_t max_batches,
                                     DeviceCounters* dc, const uint32_t* mt_off,
                                     uint32_t* batch_first, uint32_t* batch_tab, ChainBuffers cb,
                                     hipStream_t s) {
  launch_table(n_mt, batch_cap, max_batches, dc, mt_off, batch_first, batch_tab, cb, s);
  return hipGetLastError();
}

}  // namespace higs
