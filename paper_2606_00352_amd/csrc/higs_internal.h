// Internal declarations shared by the libhigs translation units (GPU side).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/higs.h"

namespace higs {

// Tile geometry (sec. 3.1): 8x8-pixel render tiles, 8x4 of them per
// 64x32-pixel macro-tile.
constexpr int kTile = 8;
constexpr int kMtTilesX = 8;
constexpr int kMtTilesY = 4;
constexpr int kMtW = kTile * kMtTilesX;  // 64
constexpr int kMtH = kTile * kMtTilesY;  // 32
constexpr int kTilesPerMt = kMtTilesX * kMtTilesY;  // 32
constexpr int kMaxBatch = 1024;  // largest B_r the rasteriser's LDS holds
constexpr int kMaxChain = 64;    // most batches of one raster work item

constexpr int kProjBlock = 256;  // gaussians per projection / emission block
constexpr int kFillGroup = 4;    // projection blocks per emission workgroup
// Projection blocks per scan chunk: a reduction writes each chunk's totals
// after the n_blocks block sums, the scan runs over the chunk totals, and a
// fill workgroup scans its chunk's block sums itself.
constexpr int kScanChunk = 256;
__host__ __device__ constexpr int64_t scan_chunks(int64_t n_blocks) {
  return (n_blocks + kScanChunk - 1) / kScanChunk;
}

// Radix sort geometry.
// 9-bit digits: a 1080p frame's keys (10 macro-tile bits, ~25 depth bits) take
// four passes instead of five 8-bit ones
constexpr int kRadixBits = 9;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortThreads = 512;
constexpr int kSortItems = 12;                         // keys per thread
constexpr int kSortTile = kSortThreads * kSortItems;  // 6144 keys per tile
constexpr int kMaxPasses = 8;

// Segmented sort geometry.
constexpr int kSegBatch = 8192;     // B_p, gaussians per partition batch (sec. 4.3)
constexpr int kSegMaxLevels = 20;   // merge levels of the largest possible segment
constexpr int kSegScanTile = 4096;  // count-matrix entries per scan tile
// Segment sort tiers (sec. 4.4): segments of up to 1,024, 2,048, 4,096 and
// 8,192 pairs, each sorted whole by one workgroup in LDS, and longer ones,
// cut into 8,192-pair chunks (sorted the same way) and merged.
constexpr int kSegTiers = 5;
constexpr uint32_t kSegTierCap[4] = {1024, 2048, 4096, 8192};
constexpr int kSegChunk = 8192;     // pairs of a chunk of a long segment
constexpr int kSegMaxMt = 20480;    // macro-tiles whose two LDS tables fit 160 KiB

// Raster record written by the projection for every visible gaussian and
// gathered by the rasteriser: 48 bytes, three 16-byte loads.
struct alignas(16) RasterRecord {
  float mx, my, l0, l1;  // centre (pixels), Cholesky factors of Sigma^-1
  float l2, o, r, g;     // ..., opacity, colour
  float b, tau, pad0, pad1;  // ..., opacity level q <= tau
};
static_assert(sizeof(RasterRecord) == 48, "record layout");

// Internal error bit in DeviceCounters::overflow: a sort look-back gave up
// waiting (reported through higs_get_counts; the frame is then invalid).
constexpr uint32_t kErrSortStall = 0x80000000u;

// Frame-wide device counters; cleared by a kernel at the start of each frame.
struct DeviceCounters {
  uint32_t n_pairs_total;   // all pairs asked for (may exceed capacity)
  uint32_t n_pairs;         // pairs stored = min(total, capacity)
  uint32_t n_visible;
  uint32_t n_batches_total;
  uint32_t n_batches;       // = min(total, capacity)
  uint32_t overflow;        // HIGS_OVF_* bits
  uint32_t sort_final;      // which key/value buffer holds the sorted pairs
  uint32_t raster_next;     // work counter of the persistent rasteriser
  uint32_t tile_next[kMaxPasses];  // work counters of the sort passes
  uint32_t sort_passes;     // radix passes that moved data (others skipped)
  uint32_t epoch;           // look-back epoch base: each frame's clear advances it by
                            //   kMaxPasses and leaves it otherwise untouched
  unsigned long long n_evals;  // gaussian-tile evaluations (when counted)
  uint32_t key_min;         // smallest / largest float32 depth bits of the
  uint32_t key_max;         //   frame's visible gaussians (key compression)
  uint32_t bwd_next;        // work counter of the persistent raster adjoint
  uint32_t seg_max;         // largest segment (segmented sort)
  uint32_t seg_next[kSegTiers + kSegMaxLevels];  // work counters: the tiers' sorts, then
                                                 //   one per merge level
  uint32_t seg_tier_n[kSegTiers];  // segments in each tier (tier 3: long segments)
  uint32_t seg_chunks;      // chunks of the long segments
  uint32_t n_chains;        // raster work items: runs of up to `chain` batches of a macro-tile
  uint32_t id_shift;        // > 0: each pair is one word key << id_shift | id (see scan_kernel)
  uint32_t sort_last;       // last radix pass that moves data (it writes the id array)
  uint32_t pad[6];
};

// Look-back status words (sort passes): 30-bit epoch,
// 2-bit flag, 32-bit count.
constexpr uint32_t kFlagAggregate = 1u;
constexpr uint32_t kFlagPrefix = 2u;
constexpr uint32_t kMaxSpins = 1u << 22;  // look-back bound: every wave exits

// Bits of (depth bits - key_min) in a pair key: enough for key_max - key_min.
__host__ __device__ __forceinline__ uint32_t depth_bits(uint32_t kmin, uint32_t kmax) {
  uint32_t d = kmax >= kmin ? kmax - kmin : 0u, b = 0;
  while (d) {
    ++b;
    d >>= 1;
  }
  return b;
}

// Camera data passed by value to kernels.
struct CamArgs {
  int32_t width, height;
  int32_t n_mt_x, n_mt_y;
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float bg[3];
};

struct ParamArgs {
  float alpha_max, t_eps, near_z, dilation;
  int32_t batch_cap, sh_degree;
  int32_t chain;  // batches of a macro-tile per raster work item
};

// Raster workgroups the chain scratch is sized for (grid bound).
constexpr int kMaxRasterWorkers = 1024;

// A frame of several views (cameras of one image size, each with its own
// scene arrays and image): view v owns the virtual gaussians
// [v * n_pad, v * n_pad + n_v) and the macro-tiles [v * n_mt, (v + 1) * n_mt),
// so that one launch of every stage serves all views: the pair keys carry the
// view in their macro-tile field, and the sort, the batch split and the
// rasteriser run unchanged over the concatenated macro-tile space.  A
// single-view frame is the case V = 1 (n_pad = the gaussian count rounded up
// to whole projection blocks).
struct ViewArgs {
  const float *means, *scales, *quats, *opac, *sh;
  int64_t n;
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float bg[3];
  float campos[3];  // camera centre -R^T t (SH view directions)
  float* image;
  float* T;
};

// The views of a frame: from a device table when there is one (several views,
// or a frame replayed from a graph, whose arguments are fixed), else the one
// view by value.
struct Views {
  int32_t count;
  int64_t n_pad;  // virtual gaussians per view: a multiple of kProjBlock * kFillGroup
  int32_t n_mt;   // macro-tiles per view
  ViewArgs v0;
  const ViewArgs* table;
  __host__ __device__ __forceinline__ const ViewArgs& get(int v) const {
    return table ? table[v] : v0;
  }
};

// ---- host-side launchers (one translation unit each) ----------------------
hipError_t launch_clear(DeviceCounters* dc, uint32_t* hist, int n_hist, hipStream_t s);

hipError_t launch_project(const Views& views, CamArgs shape, ParamArgs prm, float* f_mx,
                          float* f_my, float* f_a, float* f_b, float* f_c, float* f_tau,
                          uint32_t* f_key, uint32_t* f_cnt, uint32_t* f_span, RasterRecord* rec,
                          uint32_t* block_sums, DeviceCounters* dc, bool all_fields,
                          bool sh_packed, hipStream_t s);

hipError_t launch_scan(int64_t n, const uint32_t* cnt, uint32_t* block_sums, uint32_t max_pairs,
                       int mt_bits, bool allow_one_word, DeviceCounters* dc, hipStream_t s);

hipError_t launch_fill(int64_t n, CamArgs cam, int64_t n_pad, uint32_t n_mt, const float* f_mx,
                       const float* f_my,
                       const float* f_a, const float* f_b, const float* f_c, const float* f_tau,
                       const uint32_t* f_key, const uint32_t* f_cnt, const uint32_t* f_span,
                       const uint32_t* block_offsets, uint32_t max_pairs,
                       const DeviceCounters* dc, uint64_t* keys, uint32_t* vals, hipStream_t s);

struct SortBuffers {
  uint64_t* keys[2];
  uint32_t* vals[2];
  uint32_t* hist;        // [kMaxPasses][kRadix]
  uint32_t* plan;        // [kMaxPasses] src buffer index (~0u: pass skipped), then
                         // [kMaxPasses][kRadix] exclusive digit bases
  uint64_t* status;      // [max_tiles][kRadix] look-back words
  uint32_t max_tiles;
};
hipError_t launch_sort(int n_passes, int mt_bits, SortBuffers sb,
                       DeviceCounters* dc, int n_cus, hipStream_t s);

// Raster work items: runs of up to `chain` consecutive batches of one
// macro-tile, or (whole) every macro-tile with all its batches, empty ones
// included; tab rows are (macro-tile, first batch, batches), longest first.
struct ChainBuffers {
  uint32_t chain;
  bool whole;
  uint32_t* tab;    // [max_batches + macro-tiles][3]
};

hipError_t launch_batch(int n_mt, uint32_t batch_cap, uint32_t max_batches, const uint64_t* const* keys2,
                        DeviceCounters* dc, uint32_t* mt_off, uint32_t* batch_first,
                        uint32_t* batch_tab, ChainBuffers cb, hipStream_t s);

// fused: whole-macro-tile items fold their partials into the views' images
// (acc: per workgroup 32 x 64 float4 running sums); otherwise partials and
// active masks for the merge, and acc holds the items' products of T.
hipError_t launch_raster(CamArgs cam, ParamArgs prm, const Views& views, const uint32_t* const* vals2,
                         const RasterRecord* rec, const uint32_t* batch_tab,
                         const uint32_t* chain_tab, DeviceCounters* dc, float4* partials,
                         uint32_t* active, float4* acc, int n_cus, bool count_evals, bool fused,
                         hipStream_t s);
// Resets the rasteriser's work counter (to rasterise a frame again).
hipError_t launch_raster_rewind(DeviceCounters* dc, hipStream_t s);

// Half-precision rasteriser and merge; the partials buffer then holds four
// halves per pixel.
// Half precision, fused (whole-macro-tile work items; acc as launch_raster's).
hipError_t launch_raster16_fused(CamArgs cam, ParamArgs prm, const Views& views,
                                 const uint32_t* const* vals2, const RasterRecord* rec,
                                 const uint32_t* batch_tab, const uint32_t* chain_tab,
                                 DeviceCounters* dc, float4* acc, int n_cus, bool count_evals,
                                 hipStream_t s);
hipError_t launch_raster16(CamArgs cam, ParamArgs prm, const uint32_t* const* vals2,
                           const RasterRecord* rec, const uint32_t* batch_tab, DeviceCounters* dc,
                           void* partials, uint32_t* active, int n_cus, bool count_evals,
                           hipStream_t s);
hipError_t launch_merge16(CamArgs cam, ParamArgs prm, const Views& views,
                          const uint32_t* batch_first, const uint32_t* active, const void* partials,
                          const DeviceCounters* dc, hipStream_t s);

hipError_t launch_merge(CamArgs cam, ParamArgs prm, const Views& views, const uint32_t* batch_first,
                        const uint32_t* active, const float4* partials, const DeviceCounters* dc,
                        hipStream_t s);

// Adjoint of the frame (clear, merge, raster and projection adjoints).
// state: float2 per (batch, tile, pixel); dgeo: 16 floats per gaussian.
hipError_t launch_backward(int64_t n, const float* means, const float* scales, const float* quats,
                           const float* sh, CamArgs cam, ParamArgs prm,
                           const uint32_t* const* vals2, const RasterRecord* rec,
                           const uint32_t* f_cnt, const uint32_t* batch_tab,
                           const uint32_t* batch_first, const uint32_t* active,
                           const float4* partials, DeviceCounters* dc, const float* dimg,
                           const float* dT, float2* state, float* dgeo, float* dmeans,
                           float* dscales, float* dquats, float* dopac, float* dsh, int n_cus,
                           hipStream_t s);

struct SegBuffers {
  uint16_t* cm;         // [n_mt][n_b] pairs per (macro-tile, partition batch)
  uint32_t* tile_sum;   // [tiles + 1] scan tile sums, then their exclusive scan
  uint32_t* off;        // [n_mt][n_b] first pair slot of each (macro-tile, batch)
  uint32_t* mt_off;     // [n_mt + 1] segment offsets
  uint32_t* list;       // [4][n_mt] segments of each tier, then [n_mt + 1] chunk table
  uint64_t* comp;       // [max_pairs] composites as filled, then a merge buffer
  uint64_t* runs;       // [max_pairs] sorted runs / merge buffer
  uint32_t* ids;        // [max_pairs] output: ids in (macro-tile, depth, id) order
};
// Binning into segments: per-macro-tile counts and their scan, then the fill
// of composites; then the sort of every segment (chunk sort, merge levels).
hipError_t launch_seg_count(int64_t n, CamArgs cam, const float* f_mx, const float* f_my,
                            const float* f_a, const float* f_b, const float* f_c,
                            const float* f_tau, const uint32_t* f_cnt, const uint32_t* f_span,
                            SegBuffers sb, uint32_t max_pairs, DeviceCounters* dc, hipStream_t s);
hipError_t launch_seg_fill(int64_t n, CamArgs cam, const float* f_mx, const float* f_my,
                           const float* f_a, const float* f_b, const float* f_c, const float* f_tau,
                           const uint32_t* f_key, const uint32_t* f_cnt, const uint32_t* f_span,
                           SegBuffers sb, uint32_t max_pairs, DeviceCounters* dc, hipStream_t s);
hipError_t launch_seg_sort(int64_t n, int n_mt, SegBuffers sb, uint32_t max_pairs,
                           DeviceCounters* dc, int n_cus, hipStream_t s);

// Batch table from segment offsets already computed (segmented sort).
hipError_t launch_batch_from_offsets(int n_mt, uint32_t batch_cap, uint32_t max_batches,
                                     DeviceCounters* dc, const uint32_t* mt_off,
                                     uint32_t* batch_first, uint32_t* batch_tab, ChainBuffers cb,
                                     hipStream_t s);

int raster_workers_per_cu();
// Resident workgroups per CU of the persistent kernels, queried once per
// process (before any graph capture reads them).
int raster_per_cu_config();
int raster16_per_cu_config();
int onesweep_per_cu_config();
int seg_sort_configs();

// Enqueues a copy of the context's frame counters into pinned host memory
// (sizeof(DeviceCounters) bytes) on stream s.
int ctx_enqueue_counters(higs_ctx* c, void* pinned_dst, hipStream_t s);
// Contexts in caller-provided device memory (the render server's arena):
// ctx_arena_bytes is the size ctx_create_in lays the buffers out in (or a
// negative error for invalid capacities); ctx_create_in zeroes what must start
// at zero with kernels on stream s; ctx_release frees the host-side state only
// (no device memory, no device synchronisation: the caller has waited for the
// context's last frame).
int64_t ctx_arena_bytes(const higs_params* params, int64_t max_gaussians, int64_t max_pairs,
                        int64_t max_batches, int32_t max_width, int32_t max_height);
int ctx_create_in(int device, const higs_params* params, int64_t max_gaussians,
                  int64_t max_pairs, int64_t max_batches, int32_t max_width, int32_t max_height,
                  void* arena, size_t arena_bytes, hipStream_t s, higs_ctx** out);
int ctx_release(higs_ctx* c);

}  // namespace higs
