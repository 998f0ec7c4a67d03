// The C-ABI of libhigs: context (workspace sized up front, sec. 3.1's
// "preallocated up front"), stage entry points, counts, debug read-back,
// per-kernel timers.  Every stage only enqueues kernels on the caller's
// stream; data-dependent sizes (pairs, batches) stay on the device.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include <cstring>
#include <mutex>
#include <vector>

#include "higs_internal.h"
#include "shcodec.h"

using namespace higs;

constexpr int kViewRing = 4;
constexpr size_t kMaxGraphs = 32;  // graphs a context keeps (least recently used go)

struct higs_ctx {
  int device = 0;
  int n_cus = 0;
  higs_params params{};
  int64_t max_g = 0, max_pairs = 0, max_batches = 0;
  int32_t max_w = 0, max_h = 0, max_mt = 0;

  float *f_mx = nullptr, *f_my = nullptr, *f_a = nullptr, *f_b = nullptr, *f_c = nullptr,
        *f_tau = nullptr;
  uint32_t *f_key = nullptr, *f_cnt = nullptr;
  uint32_t* f_span = nullptr;  // compact macro-tile list of each visible gaussian
  RasterRecord* rec = nullptr;
  uint32_t* block_sums = nullptr;  // per projection block: pair count, visible count
  uint64_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint64_t* dbg_keys = nullptr;
  uint32_t* dbg_vals = nullptr;
  uint32_t* hist = nullptr;
  uint32_t* plan = nullptr;
  uint64_t* status = nullptr;
  uint32_t max_tiles = 0;
  uint32_t *mt_off = nullptr, *batch_first = nullptr, *batch_tab = nullptr, *active = nullptr;
  uint32_t* chain_tab = nullptr;  // raster work items (batches of one macro-tile)
  float4* chain_acc = nullptr;  // [kMaxRasterWorkers][32 tiles][64 px] items' running state
  float4* partials = nullptr;   // (one element when the frames fold their partials in the raster)
  DeviceCounters* dc = nullptr;
  // segmented sort: per macro-tile counts, fill cursors, chunk and block tables
  uint16_t* seg_cm = nullptr;  // [n_mt][n_b] count matrix
  uint32_t *seg_off = nullptr, *seg_tiles = nullptr, *seg_list = nullptr;
  bool segmented() const { return params.sort_mode == HIGS_SORT_SEGMENTED; }
  // adjoint buffers, allocated by the first higs_raster_backward
  float2* bwd_state = nullptr;  // [max_batches][32 tiles][64 px]: T before, suffix X
  float* dgeo = nullptr;        // [max_g][16] record gradients
  float4* partials_bwd = nullptr;  // [max_batches][32][64]: partials the adjoint has a fused
                                   //   frame rasterised again into
  bool fused_frame = false;  // the last frame folded its partials in the raster
  // frames fold the partials in the raster unless fuse_merge is 0
  bool fuses() const { return params.fuse_merge != 0; }
  // the scene arrays of the last higs_project (re-read by the adjoint)
  const float *in_means = nullptr, *in_scales = nullptr, *in_quats = nullptr,
              *in_opac = nullptr, *in_sh = nullptr;

  // frame state
  higs_camera cam{};
  CamArgs ca{};
  ParamArgs pa{};
  int64_t n = 0;
  int stage = 0;  // 1 projected, 2 sorted, 3 batched, 4 rastered
  int n_mt = 0, n_passes = 0;
  // views of the frame (a single-view frame: n_views = 1)
  int n_views = 1;
  int64_t n_pad = 0;    // virtual gaussians per view
  int64_t n_virt = 0;   // n_views * n_pad
  int n_mt_all = 0;     // n_views * n_mt
  Views views{};
  ViewArgs* view_table = nullptr;  // [max_views] device copy of the views
  ViewArgs* view_stage = nullptr;  // [kViewRing][max_views] pinned host slots
  hipEvent_t view_ev[kViewRing] = {};
  int view_slot = 0;
  uint64_t epoch_frames = 0;  // frames since the look-back words were last untagged
  // frames replayed from graphs (params.use_graphs): one graph per frame shape
  struct Graph {
    int32_t n_views = 0, width = 0, height = 0;
    int64_t n_pad = 0;
    hipGraphExec_t exec = nullptr;
    ViewArgs* stage = nullptr;  // pinned slice [n_views] of graph_stage: each replay copies
                                //   it to view_table
    hipEvent_t done = nullptr;  // after the last replay: the stage may be rewritten
    bool launched = false;
    uint64_t last_used = 0;
  };
  std::vector<Graph> graphs;
  uint64_t graph_tick = 0;
  ViewArgs* graph_stage = nullptr;  // pinned [kMaxGraphs][max_views]: the graphs' stages
  bool external = false;  // buffers carved from a caller's arena (not freed here)
  hipStream_t last_stream = nullptr;
  int debug_flags = 0;
  // timing: events of the last `ring` frames, frame f in slot f % ring
  int ring = 0;
  int64_t frames = 0;  // frames recorded since timing was set
  hipEvent_t* ev = nullptr;  // [ring][HIGS_NUM_TIMERS][2]
  bool timing() const { return ring > 0; }
  hipEvent_t event(int slot, int which) const {
    return ev[(((frames - 1) % ring) * HIGS_NUM_TIMERS + slot) * 2 + which];
  }
};

namespace {

// Fills n 64-bit words with zero (a kernel, so that a caller capturing the
// stream into a graph records no memset node).
__global__ void zero_words_kernel(uint64_t* __restrict__ p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

__global__ void epoch_reset_kernel(DeviceCounters* __restrict__ dc) { dc->epoch = 0; }

void destroy_graph(higs_ctx::Graph& g) {
  if (g.launched && g.done) (void)hipEventSynchronize(g.done);
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.done) (void)hipEventDestroy(g.done);
  g = higs_ctx::Graph();
}

hipError_t launch_zero_words(uint64_t* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t want = (n + 255) / 256;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)(want < 2048 ? want : 2048)), dim3(256), 0,
                     s, p, n);
  return hipGetLastError();
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <class T>
int dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return HIGS_E_NOMEM;
  }
  return HIGS_OK;
}

void free_events(higs_ctx* c) {
  if (c->ev) {
    for (int k = 0; k < c->ring * HIGS_NUM_TIMERS * 2; ++k)
      if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    delete[] c->ev;
  }
  c->ev = nullptr;
  c->ring = 0;
  c->frames = 0;
}

void free_all(higs_ctx* c) {
  // buffers allocated on demand (debug read-back, the adjoint's state)
  void* extra[] = {c->dbg_keys, c->dbg_vals, c->bwd_state, c->dgeo, c->partials_bwd};
  for (void* b : extra)
    if (b) (void)hipFree(b);
  if (!c->external) {
    void* bufs[] = {c->f_mx, c->f_my, c->f_a, c->f_b, c->f_c, c->f_tau, c->f_key, c->f_cnt,
                    c->f_span, c->rec, c->block_sums, c->keys[0], c->keys[1], c->vals[0],
                    c->vals[1], c->hist, c->plan, c->status, c->mt_off, c->batch_first,
                    c->batch_tab, c->active, c->partials, c->dc, c->chain_tab,
                    c->chain_acc, c->seg_cm, c->seg_off,
                    c->seg_tiles, c->seg_list, c->view_table};
    for (void* b : bufs)
      if (b) (void)hipFree(b);
  }
  for (higs_ctx::Graph& g : c->graphs) destroy_graph(g);
  c->graphs.clear();
  if (c->view_stage) (void)hipHostFree(c->view_stage);
  if (c->graph_stage) (void)hipHostFree(c->graph_stage);
  for (hipEvent_t& e : c->view_ev)
    if (e) (void)hipEventDestroy(e);
  free_events(c);
}

// Every device buffer of a context and its element count, in one place:
// higs_ctx_create allocates them, higs_ctx_footprint adds them up, and the
// allocation-free entry point lays them out in its static scratch array.
// A view's range of virtual gaussians: whole fill groups of projection blocks
// (the emission takes the view from the group's first block).
int64_t pad_blocks(int64_t n) {
  constexpr int64_t q = (int64_t)kProjBlock * kFillGroup;
  return (n + q - 1) / q * q;
}

// Needs max_g, max_pairs, max_batches, max_mt and max_tiles set.
template <class F>
void for_each_buffer(higs_ctx* c, F&& f) {
  // per-gaussian arrays hold max_views ranges of max_g, each padded
  const size_t G = (size_t)c->params.max_views * (size_t)pad_blocks(c->max_g);
  const size_t P = (size_t)c->max_pairs, B = (size_t)c->max_batches;
  const size_t nblk = (G + kProjBlock - 1) / kProjBlock;
  const size_t mt = (size_t)c->max_mt;
  f(&c->f_mx, G);
  f(&c->f_my, G);
  f(&c->f_a, G);
  f(&c->f_b, G);
  f(&c->f_c, G);
  f(&c->f_tau, G);
  f(&c->f_key, G);
  f(&c->f_cnt, G);
  f(&c->f_span, G);
  f(&c->rec, G);
  f(&c->block_sums, 2 * nblk + 2 * (size_t)scan_chunks((int64_t)nblk));
  f(&c->keys[0], P);
  f(&c->keys[1], P);
  f(&c->vals[0], P);
  f(&c->vals[1], P);
  f(&c->hist, (size_t)kMaxPasses * kRadix);
  f(&c->plan, (size_t)kMaxPasses + (size_t)kMaxPasses * kRadix);
  f(&c->status, (size_t)c->max_tiles * kRadix);
  f(&c->mt_off, mt + 1);
  f(&c->batch_first, mt + 1);
  f(&c->batch_tab, 3 * B);
  f(&c->chain_tab, 3 * (B + mt));
  f(&c->chain_acc, (size_t)kMaxRasterWorkers * kTilesPerMt * 64);
  f(&c->active, B);
  f(&c->partials, c->fuses() ? 1 : B * kTilesPerMt * 64);
  f(&c->dc, (size_t)1);
  // segmented sort (single-view contexts only): the (macro-tile, partition
  // batch) count matrix and its scan, the tile sums, the tier lists
  const size_t mat = c->segmented()
                         ? mt * (size_t)((c->max_g + kSegBatch - 1) / kSegBatch)
                         : 1;
  f(&c->seg_cm, mat);
  f(&c->seg_off, mat);
  f(&c->seg_tiles, (mat + kSegScanTile - 1) / kSegScanTile + 1);
  f(&c->seg_list, c->segmented() ? (size_t)kSegTiers * mt + mt + 1 : 1);
  f(&c->view_table, (size_t)c->params.max_views);
}

// Lays the context's buffers out in [base, base + cap), 256-byte aligned.
bool carve(higs_ctx* c, unsigned char* base, size_t cap) {
  size_t off = 0;
  bool fits = true;
  for_each_buffer(c, [&](auto** ptr, size_t count) {
    using T = typename std::remove_reference<decltype(**ptr)>::type;
    const size_t bytes = ((count ? count : 1) * sizeof(T) + 255) & ~(size_t)255;
    if (off + bytes > cap) {
      fits = false;
      *ptr = nullptr;
      return;
    }
    *ptr = reinterpret_cast<T*>(base + off);
    off += bytes;
  });
  return fits;
}

void set_capacities(higs_ctx* c, int64_t max_gaussians, int64_t max_pairs, int64_t max_batches,
                    int32_t max_width, int32_t max_height) {
  c->max_g = max_gaussians;
  c->max_pairs = max_pairs;
  c->max_batches = max_batches;
  c->max_w = max_width;
  c->max_h = max_height;
  c->max_mt = ((max_width + kMtW - 1) / kMtW) * ((max_height + kMtH - 1) / kMtH) *
              (c->params.max_views > 0 ? c->params.max_views : 1);
  c->max_tiles = (uint32_t)((max_pairs + kSortTile - 1) / kSortTile);
}

int n_bits(uint32_t v) {  // bits needed to hold 0..v
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

int hip_err(hipError_t e) {
  if (e != hipSuccess) {
    fprintf(stderr, "libhigs: HIP error %d (%s)\n", (int)e, hipGetErrorString(e));
    return HIGS_E_HIP;
  }
  return HIGS_OK;
}

struct TimerScope {
  higs_ctx* c;
  int slot;
  hipStream_t s;
  TimerScope(higs_ctx* ctx, int k, hipStream_t st) : c(ctx), slot(k), s(st) {
    if (c->timing()) (void)hipEventRecord(c->event(slot, 0), s);
  }
  ~TimerScope() {
    if (c->timing()) (void)hipEventRecord(c->event(slot, 1), s);
  }
};

}  // namespace

extern "C" {

void higs_default_params(higs_params* p) {
  if (!p) return;
  p->tile_px = 8;
  p->mt_tiles_x = 8;
  p->mt_tiles_y = 4;
  p->batch_cap = 1024;
  p->sh_degree = 3;
  p->alpha_max = 0.99f;
  p->t_eps = 1e-4f;
  p->near_z = 0.2f;
  p->dilation = 0.3f;
  p->sort_mode = HIGS_SORT_ONESWEEP;
  p->raster_precision = HIGS_RASTER_FP32;
  p->sh_format = HIGS_SH_FLOAT32;
  p->max_views = 1;
  p->use_graphs = 0;
  p->raster_chain = 64;
  p->fuse_merge = 1;
}

const char* higs_error_string(int code) {
  switch (code) {
    case HIGS_OK: return "ok";
    case HIGS_E_INVALID: return "invalid argument";
    case HIGS_E_NOMEM: return "out of device memory";
    case HIGS_E_CAPACITY: return "size exceeds the context's capacity";
    case HIGS_E_HIP: return "HIP runtime error";
    case HIGS_E_UNSUPPORTED: return "unsupported parameter";
    case HIGS_E_STATE: return "stage called before the stage it depends on";
    default: return "unknown error";
  }
}

}  // extern "C"

namespace {
int check_params(const higs_params& p, int64_t max_gaussians, int64_t max_pairs,
                 int64_t max_batches, int32_t max_width, int32_t max_height) {
  if (p.tile_px != kTile || p.mt_tiles_x != kMtTilesX || p.mt_tiles_y != kMtTilesY)
    return HIGS_E_UNSUPPORTED;
  if (p.sh_degree < 0 || p.sh_degree > 3) return HIGS_E_UNSUPPORTED;
  if (p.raster_precision != HIGS_RASTER_FP32 && p.raster_precision != HIGS_RASTER_FP16)
    return HIGS_E_INVALID;
  if (p.sh_format != HIGS_SH_FLOAT32 && p.sh_format != HIGS_SH_PACKED32) return HIGS_E_INVALID;
  if (p.sh_format == HIGS_SH_PACKED32 && p.sh_degree != 3) return HIGS_E_UNSUPPORTED;
  if (p.max_views < 1 || p.max_views > HIGS_MAX_VIEWS) return HIGS_E_INVALID;
  if (p.max_views > 1 && p.sort_mode == HIGS_SORT_SEGMENTED) return HIGS_E_UNSUPPORTED;
  if (p.sort_mode != HIGS_SORT_SEGMENTED && p.sort_mode != HIGS_SORT_ONESWEEP) return HIGS_E_INVALID;
  if (p.sort_mode == HIGS_SORT_SEGMENTED &&
      ((int64_t)((max_width + kMtW - 1) / kMtW) * ((max_height + kMtH - 1) / kMtH) > kSegMaxMt))
    return HIGS_E_UNSUPPORTED;
  if (p.batch_cap < 1 || p.batch_cap > kMaxBatch) return HIGS_E_INVALID;
  if (!(p.alpha_max > 0.0f && p.alpha_max <= 1.0f) || !(p.t_eps >= 0.0f) ||
      !(p.dilation >= 0.0f) || !(p.near_z == p.near_z))
    return HIGS_E_INVALID;
  if (max_gaussians < 1 || max_pairs < 1 || max_batches < 1 || max_width < 1 || max_height < 1)
    return HIGS_E_INVALID;
  if (max_gaussians > (int64_t)0x7fffffff || max_pairs > (int64_t)0xfffff000 ||
      max_batches > (int64_t)0x7fffffff)
    return HIGS_E_INVALID;
  // virtual gaussian ids (the view's range, then the gaussian) are 32-bit
  if ((int64_t)p.max_views * pad_blocks(max_gaussians) > (int64_t)0xffffffff) return HIGS_E_INVALID;
  if (p.use_graphs != 0 && p.use_graphs != 1) return HIGS_E_INVALID;
  if (p.raster_chain < 1 || p.raster_chain > kMaxChain) return HIGS_E_INVALID;
  if (p.fuse_merge != 0 && p.fuse_merge != 1) return HIGS_E_INVALID;
  return HIGS_OK;
}

// Device bytes of a context laid out by carve (every buffer 256-byte aligned).
int64_t carved_bytes(higs_ctx* c) {
  int64_t bytes = 0;
  for_each_buffer(c, [&](auto** ptr, size_t count) {
    bytes += (int64_t)((((count ? count : 1) * sizeof(**ptr)) + 255) & ~(size_t)255);
  });
  return bytes;
}

// Host-side state of a new context: pinned view-table slots and their events.
bool init_host_state(higs_ctx* c) {
  const higs_params& p = c->params;
  bool ok = true;
  if (p.max_views > 1) {
    ok = hipHostMalloc(reinterpret_cast<void**>(&c->view_stage),
                       sizeof(ViewArgs) * (size_t)p.max_views * kViewRing,
                       hipHostMallocDefault) == hipSuccess;
    for (int k = 0; ok && k < kViewRing; ++k)
      ok = hipEventCreateWithFlags(&c->view_ev[k], hipEventDisableTiming) == hipSuccess;
  }
  if (ok && p.use_graphs)
    ok = hipHostMalloc(reinterpret_cast<void**>(&c->graph_stage),
                       sizeof(ViewArgs) * (size_t)p.max_views * kMaxGraphs,
                       hipHostMallocDefault) == hipSuccess;
  return ok;
}

// A context with its buffers in [arena, arena + arena_bytes) (null arena:
// buffers of its own).  An arena context's look-back words and counters are
// zeroed by kernels on stream s, with no host synchronisation.
int create_ctx(int device, const higs_params* params, int64_t max_gaussians, int64_t max_pairs,
               int64_t max_batches, int32_t max_width, int32_t max_height, unsigned char* arena,
               size_t arena_bytes, hipStream_t s, higs_ctx** out) {
  if (!out) return HIGS_E_INVALID;
  *out = nullptr;
  higs_params p;
  if (params) p = *params;
  else higs_default_params(&p);
  int rc = check_params(p, max_gaussians, max_pairs, max_batches, max_width, max_height);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HIGS_E_INVALID;
  DeviceGuard g(device);
  // launch shapes of the persistent kernels, before any capture reads them
  (void)raster_per_cu_config();
  (void)raster16_per_cu_config();
  (void)onesweep_per_cu_config();
  (void)seg_sort_configs();
  higs_ctx* c = new (std::nothrow) higs_ctx();
  if (!c) return HIGS_E_NOMEM;
  c->device = device;
  c->params = p;
  set_capacities(c, max_gaussians, max_pairs, max_batches, max_width, max_height);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return HIGS_E_HIP;
  }
  c->n_cus = prop.multiProcessorCount;
  bool ok;
  if (arena) {
    c->external = true;
    ok = carve(c, arena, arena_bytes);
    if (!ok) {
      free_all(c);
      delete c;
      return HIGS_E_CAPACITY;
    }
    // look-back words start untagged (epoch 0 never matches a pass)
    ok = launch_zero_words(c->status, (size_t)c->max_tiles * kRadix, s) == hipSuccess &&
         launch_zero_words(reinterpret_cast<uint64_t*>(c->dc), sizeof(DeviceCounters) / 8, s) ==
             hipSuccess;
  } else {
    rc = HIGS_OK;
    for_each_buffer(c, [&](auto** ptr, size_t count) { rc |= dalloc(ptr, count); });
    if (rc != HIGS_OK) {
      free_all(c);
      delete c;
      return HIGS_E_NOMEM;
    }
    // look-back words start untagged (epoch 0 never matches a pass); cleared on
    // a stream of the context's own, so that creating a context does not wait for
    // work in flight on other streams
    hipStream_t init = nullptr;
    ok = hipStreamCreateWithFlags(&init, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipMemsetAsync(c->status, 0, (size_t)c->max_tiles * kRadix * sizeof(uint64_t),
                              init) == hipSuccess;
    ok = ok && hipMemsetAsync(c->dc, 0, sizeof(DeviceCounters), init) == hipSuccess;
    ok = ok && hipStreamSynchronize(init) == hipSuccess;
    if (init) (void)hipStreamDestroy(init);
  }
  ok = ok && init_host_state(c);
  if (!ok) {
    free_all(c);
    delete c;
    return HIGS_E_HIP;
  }
  *out = c;
  return HIGS_OK;
}
}  // namespace

namespace higs {
int64_t ctx_arena_bytes(const higs_params* params, int64_t max_gaussians, int64_t max_pairs,
                        int64_t max_batches, int32_t max_width, int32_t max_height) {
  higs_ctx c;
  if (params) c.params = *params;
  else higs_default_params(&c.params);
  const int rc = check_params(c.params, max_gaussians, max_pairs, max_batches, max_width, max_height);
  if (rc) return rc;
  set_capacities(&c, max_gaussians, max_pairs, max_batches, max_width, max_height);
  return carved_bytes(&c);
}

int ctx_create_in(int device, const higs_params* params, int64_t max_gaussians,
                  int64_t max_pairs, int64_t max_batches, int32_t max_width, int32_t max_height,
                  void* arena, size_t arena_bytes, hipStream_t s, higs_ctx** out) {
  if (!arena) return HIGS_E_INVALID;
  return create_ctx(device, params, max_gaussians, max_pairs, max_batches, max_width, max_height,
                    static_cast<unsigned char*>(arena), arena_bytes, s, out);
}

int ctx_release(higs_ctx* c) {
  if (!c) return HIGS_E_INVALID;
  DeviceGuard g(c->device);
  free_all(c);
  delete c;
  return HIGS_OK;
}
}  // namespace higs

extern "C" {

int higs_ctx_create(int device, const higs_params* params, int64_t max_gaussians,
                    int64_t max_pairs, int64_t max_batches, int32_t max_width,
                    int32_t max_height, higs_ctx** out) {
  return create_ctx(device, params, max_gaussians, max_pairs, max_batches, max_width, max_height,
                    nullptr, 0, nullptr, out);
}

int64_t higs_ctx_footprint(const higs_params* params, int64_t max_gaussians, int64_t max_pairs,
                           int64_t max_batches, int32_t max_width, int32_t max_height) {
  if (max_gaussians < 1 || max_pairs < 1 || max_batches < 1 || max_width < 1 || max_height < 1)
    return HIGS_E_INVALID;
  higs_ctx c;
  if (params) c.params = *params;
  else higs_default_params(&c.params);
  if (c.params.max_views < 1) return HIGS_E_INVALID;
  set_capacities(&c, max_gaussians, max_pairs, max_batches, max_width, max_height);
  int64_t bytes = 0;
  for_each_buffer(&c, [&](auto** ptr, size_t count) {
    bytes += (int64_t)((count ? count : 1) * sizeof(**ptr));
  });
  return bytes;
}

int higs_ctx_destroy(higs_ctx* c) {
  if (!c) return HIGS_E_INVALID;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  free_all(c);
  delete c;
  return HIGS_OK;
}

int higs_set_debug(higs_ctx* c, int flags) {
  if (!c) return HIGS_E_INVALID;
  DeviceGuard g(c->device);
  if ((flags & HIGS_DEBUG_KEEP_PAIRS) && !c->dbg_keys) {
    if (dalloc(&c->dbg_keys, (size_t)c->max_pairs) != HIGS_OK ||
        dalloc(&c->dbg_vals, (size_t)c->max_pairs) != HIGS_OK)
      return HIGS_E_NOMEM;
  }
  c->debug_flags = flags;
  return HIGS_OK;
}

int higs_set_timing(higs_ctx* c, int n_frames) {
  if (!c || n_frames < 0 || n_frames > 1024) return HIGS_E_INVALID;
  DeviceGuard g(c->device);
  if (c->ring) (void)hipStreamSynchronize(c->last_stream);
  free_events(c);
  if (n_frames == 0) return HIGS_OK;
  const int total = n_frames * HIGS_NUM_TIMERS * 2;
  c->ev = new (std::nothrow) hipEvent_t[total];
  if (!c->ev) return HIGS_E_NOMEM;
  for (int k = 0; k < total; ++k) c->ev[k] = nullptr;
  c->ring = n_frames;
  for (int k = 0; k < total; ++k)
    if (hipEventCreate(&c->ev[k]) != hipSuccess) {
      free_events(c);
      return HIGS_E_HIP;
    }
  return HIGS_OK;
}

}  // extern "C"

namespace {
// Camera fields of a view, and the frame's shared image geometry.
void fill_view(ViewArgs& w, const higs_camera* cam) {
  w.fx = cam->fx;
  w.fy = cam->fy;
  w.cx = cam->cx;
  w.cy = cam->cy;
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) w.R[r * 3 + k] = cam->world_to_cam[r * 4 + k];
    w.t[r] = cam->world_to_cam[r * 4 + 3];
  }
  for (int k = 0; k < 3; ++k) {
    w.bg[k] = cam->background[k];
    // camera centre -R^T t, for the SH view direction
    w.campos[k] = -(w.R[k] * w.t[0] + w.R[3 + k] * w.t[1] + w.R[6 + k] * w.t[2]);
  }
}

ViewArgs view_args(const higs_view& w) {
  ViewArgs a{};
  a.means = w.means;
  a.scales = w.scales;
  a.quats = w.quats;
  a.opac = w.opacities;
  a.sh = w.sh;
  a.n = w.n;
  a.image = w.image;
  a.T = w.T_out;
  fill_view(a, &w.camera);
  return a;
}

int check_camera(const higs_ctx* c, const higs_camera* cam) {
  if (!cam || cam->width < 1 || cam->height < 1) return HIGS_E_INVALID;
  if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f)) return HIGS_E_INVALID;
  if (cam->width > c->max_w || cam->height > c->max_h) return HIGS_E_CAPACITY;
  return HIGS_OK;
}

// The look-back status words carry 30 epoch bits and every frame advances the
// epoch by kMaxPasses (its clear kernel does): before the epoch could wrap,
// the words go back to untagged and the epoch to zero, by kernels on the
// frame's stream ahead of the frame.
int epoch_guard(higs_ctx* c, hipStream_t s) {
  constexpr uint64_t kFramesPerCycle = ((1u << 30) - 2u * kMaxPasses) / kMaxPasses;
  if (++c->epoch_frames < kFramesPerCycle) return HIGS_OK;
  c->epoch_frames = 1;
  int rc = hip_err(launch_zero_words(c->status, (size_t)c->max_tiles * kRadix, s));
  if (rc) return rc;
  hipLaunchKernelGGL(epoch_reset_kernel, dim3(1), dim3(1), 0, s, c->dc);
  return hip_err(hipGetLastError());
}

// Stage 1 for the frame's views (set in c->views): shared geometry, counters,
// the projection of every view in one launch.  capturing: the frame is being
// recorded into a graph (its replays run the epoch guard themselves).
int project_frame(higs_ctx* c, const higs_camera* cam0, hipStream_t s, bool capturing = false) {
  c->last_stream = s;
  if (!capturing) {
    const int rc = epoch_guard(c, s);
    if (rc) return rc;
  }
  c->stage = 0;
  if (c->timing()) c->frames += 1;
  c->cam = *cam0;
  CamArgs& a = c->ca;
  a.width = cam0->width;
  a.height = cam0->height;
  a.n_mt_x = (cam0->width + kMtW - 1) / kMtW;
  a.n_mt_y = (cam0->height + kMtH - 1) / kMtH;
  a.fx = cam0->fx;
  a.fy = cam0->fy;
  a.cx = cam0->cx;
  a.cy = cam0->cy;
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) a.R[r * 3 + k] = cam0->world_to_cam[r * 4 + k];
    a.t[r] = cam0->world_to_cam[r * 4 + 3];
  }
  for (int k = 0; k < 3; ++k) a.bg[k] = cam0->background[k];
  c->pa.alpha_max = c->params.alpha_max;
  c->pa.t_eps = c->params.t_eps;
  c->pa.near_z = c->params.near_z;
  c->pa.dilation = c->params.dilation;
  c->pa.batch_cap = c->params.batch_cap;
  c->pa.sh_degree = c->params.sh_degree;
  c->pa.chain = c->params.raster_chain;
  c->n_mt = a.n_mt_x * a.n_mt_y;
  c->n_mt_all = c->n_mt * c->n_views;
  c->views.n_mt = c->n_mt;
  c->views.n_pad = c->n_pad;
  c->n_virt = c->n_pad * c->n_views;
  c->n_passes = (32 + n_bits((uint32_t)(c->n_mt_all - 1)) + kRadixBits - 1) / kRadixBits;
  int rc = hip_err(launch_clear(c->dc, c->hist, kMaxPasses * kRadix, s));
  if (rc) return rc;
  {
    TimerScope ts(c, HIGS_TIMER_PROJECT, s);
    rc = hip_err(launch_project(c->views, c->ca, c->pa, c->f_mx, c->f_my, c->f_a, c->f_b, c->f_c,
                                c->f_tau, c->f_key, c->f_cnt, c->f_span, c->rec, c->block_sums,
                                c->dc, (c->debug_flags & HIGS_DEBUG_PROJ_FIELDS) != 0,
                                c->params.sh_format == HIGS_SH_PACKED32, s));
  }
  if (rc) return rc;
  c->stage = 1;
  return HIGS_OK;
}


}  // namespace

extern "C" {

int higs_project(higs_ctx* c, int64_t n, const float* means, const float* scales,
                 const float* quats, const float* opacities, const float* sh,
                 const higs_camera* cam, void* stream) {
  if (!c || !cam || n < 0) return HIGS_E_INVALID;
  if (n > 0 && (!means || !scales || !quats || !opacities || !sh)) return HIGS_E_INVALID;
  int rc = check_camera(c, cam);
  if (rc) return rc;
  if (n > c->max_g) return HIGS_E_CAPACITY;
  DeviceGuard g(c->device);
  c->in_means = means;
  c->in_scales = scales;
  c->in_quats = quats;
  c->in_opac = opacities;
  c->in_sh = sh;
  c->n = n;
  c->n_views = 1;
  c->n_pad = pad_blocks(n);
  ViewArgs& w = c->views.v0;
  w.means = means;
  w.scales = scales;
  w.quats = quats;
  w.opac = opacities;
  w.sh = sh;
  w.n = n;
  w.image = nullptr;
  w.T = nullptr;
  fill_view(w, cam);
  c->views.count = 1;
  c->views.table = nullptr;
  return project_frame(c, cam, (hipStream_t)stream);
}

}  // extern "C"

namespace {
SegBuffers seg_buffers(higs_ctx* c) {
  SegBuffers sb;
  sb.cm = c->seg_cm;
  sb.tile_sum = c->seg_tiles;
  sb.off = c->seg_off;
  sb.list = c->seg_list;
  sb.mt_off = c->mt_off;
  sb.comp = c->keys[0];
  sb.runs = c->keys[1];
  sb.ids = c->vals[0];
  return sb;
}

int keep_pairs(higs_ctx* c, hipStream_t s) {
  if (!(c->debug_flags & HIGS_DEBUG_KEEP_PAIRS) || !c->dbg_keys) return HIGS_OK;
  int rc = hip_err(hipMemcpyAsync(c->dbg_keys, c->keys[0], (size_t)c->max_pairs * 8,
                                  hipMemcpyDeviceToDevice, s));
  if (!rc && !c->segmented())
    rc = hip_err(hipMemcpyAsync(c->dbg_vals, c->vals[0], (size_t)c->max_pairs * 4,
                                hipMemcpyDeviceToDevice, s));
  return rc;
}
}  // namespace

extern "C" {

int higs_bin_sort(higs_ctx* c, void* stream) {
  if (!c) return HIGS_E_INVALID;
  if (c->stage < 1) return HIGS_E_STATE;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  int rc;
  if (c->segmented()) {
    const SegBuffers sb = seg_buffers(c);
    {
      TimerScope ts(c, HIGS_TIMER_SCAN, s);
      rc = hip_err(launch_seg_count(c->n, c->ca, c->f_mx, c->f_my, c->f_a, c->f_b, c->f_c,
                                    c->f_tau, c->f_cnt, c->f_span, sb, (uint32_t)c->max_pairs,
                                    c->dc, s));
    }
    if (rc) return rc;
    {
      TimerScope ts(c, HIGS_TIMER_FILL, s);
      rc = hip_err(launch_seg_fill(c->n, c->ca, c->f_mx, c->f_my, c->f_a, c->f_b, c->f_c,
                                   c->f_tau, c->f_key, c->f_cnt, c->f_span, sb,
                                   (uint32_t)c->max_pairs, c->dc, s));
    }
    if (rc) return rc;
    rc = keep_pairs(c, s);
    if (rc) return rc;
    {
      TimerScope ts(c, HIGS_TIMER_SORT, s);
      rc = hip_err(launch_seg_sort(c->n, c->n_mt, sb, (uint32_t)c->max_pairs, c->dc, c->n_cus, s));
    }
    if (rc) return rc;
    c->stage = 2;
    return HIGS_OK;
  }
  {
    TimerScope ts(c, HIGS_TIMER_SCAN, s);
    rc = hip_err(launch_scan(c->n_virt, c->f_cnt, c->block_sums,
                             (uint32_t)c->max_pairs, n_bits((uint32_t)(c->n_mt_all - 1)),
                             (c->debug_flags & HIGS_DEBUG_TWO_WORD_PAIRS) == 0, c->dc, s));
  }
  if (rc) return rc;
  {
    TimerScope ts(c, HIGS_TIMER_FILL, s);
    rc = hip_err(launch_fill(c->n_virt, c->ca, c->n_pad, (uint32_t)c->n_mt, c->f_mx, c->f_my,
                             c->f_a, c->f_b, c->f_c, c->f_tau,
                             c->f_key, c->f_cnt, c->f_span, c->block_sums,
                             (uint32_t)c->max_pairs, c->dc, c->keys[0], c->vals[0], s));
  }
  if (rc) return rc;
  rc = keep_pairs(c, s);
  if (rc) return rc;
  SortBuffers sb;
  sb.keys[0] = c->keys[0];
  sb.keys[1] = c->keys[1];
  sb.vals[0] = c->vals[0];
  sb.vals[1] = c->vals[1];
  sb.hist = c->hist;
  sb.plan = c->plan;
  sb.status = c->status;
  sb.max_tiles = c->max_tiles;
  {
    TimerScope ts(c, HIGS_TIMER_SORT, s);
    rc = hip_err(launch_sort(c->n_passes, n_bits((uint32_t)(c->n_mt_all - 1)), sb, c->dc,
                             c->n_cus, s));
  }
  if (rc) return rc;
  c->stage = 2;
  return HIGS_OK;
}

int higs_batch(higs_ctx* c, void* stream) {
  if (!c) return HIGS_E_INVALID;
  if (c->stage < 2) return HIGS_E_STATE;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  const uint64_t* k2[2] = {c->keys[0], c->keys[1]};
  // chains apply to the float32 rasteriser; the other keeps one batch per item
  ChainBuffers cb;
  cb.whole = c->fuses();
  cb.chain = (!cb.whole && c->params.raster_precision == HIGS_RASTER_FP32)
                 ? (uint32_t)c->params.raster_chain
                 : 1u;
  cb.tab = c->chain_tab;
  int rc;
  {
    TimerScope ts(c, HIGS_TIMER_BATCH, s);
    if (c->segmented())
      rc = hip_err(launch_batch_from_offsets(c->n_mt, (uint32_t)c->params.batch_cap,
                                             (uint32_t)c->max_batches, c->dc, c->mt_off,
                                             c->batch_first, c->batch_tab, cb, s));
    else
      rc = hip_err(launch_batch(c->n_mt_all, (uint32_t)c->params.batch_cap, (uint32_t)c->max_batches,
                                k2, c->dc, c->mt_off, c->batch_first, c->batch_tab, cb, s));
  }
  if (rc) return rc;
  c->stage = 3;
  return HIGS_OK;
}

}  // extern "C"

namespace {
// Stage 4 for the frame's views (their images are in c->views).
int raster_frame(higs_ctx* c, hipStream_t s) {
  c->last_stream = s;
  const uint32_t* v2[2] = {c->vals[0], c->vals[1]};
  int rc;
  const bool half = c->params.raster_precision == HIGS_RASTER_FP16;
  const bool count = (c->debug_flags & HIGS_DEBUG_COUNT_EVALS) != 0;
  const bool fused = c->fuses();
  c->fused_frame = fused;
  {
    TimerScope ts(c, HIGS_TIMER_RASTER, s);
    if (half && fused)
      rc = hip_err(launch_raster16_fused(c->ca, c->pa, c->views, v2, c->rec, c->batch_tab,
                                         c->chain_tab, c->dc, c->chain_acc, c->n_cus, count, s));
    else if (half)
      rc = hip_err(launch_raster16(c->ca, c->pa, v2, c->rec, c->batch_tab, c->dc, c->partials,
                                   c->active, c->n_cus, count, s));
    else
      rc = hip_err(launch_raster(c->ca, c->pa, c->views, v2, c->rec, c->batch_tab, c->chain_tab,
                                 c->dc, c->partials, c->active, c->chain_acc, c->n_cus, count,
                                 fused, s));
  }
  if (rc) return rc;
  {
    TimerScope ts(c, HIGS_TIMER_MERGE, s);
    if (fused) {
      // the raster wrote the images
    } else if (half)
      rc = hip_err(launch_merge16(c->ca, c->pa, c->views, c->batch_first, c->active, c->partials,
                                  c->dc, s));
    else
      rc = hip_err(launch_merge(c->ca, c->pa, c->views, c->batch_first, c->active, c->partials,
                                c->dc, s));
  }
  if (rc) return rc;
  c->stage = 4;
  return HIGS_OK;
}

// A frame is replayed from a graph when the context asks for it, the stream
// can be captured (not the legacy default stream) and no timers or debug
// outputs are on (their events and copies vary from frame to frame).
bool graph_frame(const higs_ctx* c, hipStream_t s) {
  return c->params.use_graphs && s != nullptr && !c->timing() && c->debug_flags == 0 &&
         !c->segmented();
}

// The frame of views va[0 .. n_views) from the graph of its shape (views,
// virtual range, image size), recorded on first use: every argument of its
// kernels is fixed, and what varies per frame (scene arrays, cameras, images)
// reaches them through the view table, which the graph's first node copies
// from the graph's pinned stage.
int render_graph(higs_ctx* c, int n_views, const ViewArgs* va, const higs_camera* cam0,
                 hipStream_t s) {
  const size_t bytes = sizeof(ViewArgs) * (size_t)n_views;
  int gi = -1;
  for (size_t k = 0; k < c->graphs.size(); ++k) {
    const higs_ctx::Graph& g = c->graphs[k];
    if (g.n_views == n_views && g.n_pad == c->n_pad && g.width == cam0->width &&
        g.height == cam0->height) {
      gi = (int)k;
      break;
    }
  }
  if (gi < 0) {
    if (c->graphs.size() >= kMaxGraphs) {
      size_t lru = 0;
      for (size_t k = 1; k < c->graphs.size(); ++k)
        if (c->graphs[k].last_used < c->graphs[lru].last_used) lru = k;
      destroy_graph(c->graphs[lru]);
      c->graphs.erase(c->graphs.begin() + (long)lru);
    }
    higs_ctx::Graph g;
    g.n_views = n_views;
    g.n_pad = c->n_pad;
    g.width = cam0->width;
    g.height = cam0->height;
    // the first stage slice no held graph uses
    for (size_t k = 0; k < kMaxGraphs && !g.stage; ++k) {
      ViewArgs* cand = c->graph_stage + k * (size_t)c->params.max_views;
      bool used = false;
      for (const higs_ctx::Graph& h : c->graphs) used = used || h.stage == cand;
      if (!used) g.stage = cand;
    }
    if (!g.stage || hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) {
      destroy_graph(g);
      return HIGS_E_NOMEM;
    }
    c->views.count = n_views;
    c->views.table = c->view_table;
    c->views.v0 = va[0];
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      destroy_graph(g);
      return HIGS_E_HIP;
    }
    int rc = hip_err(hipMemcpyAsync(c->view_table, g.stage, bytes, hipMemcpyHostToDevice, s));
    if (!rc) rc = project_frame(c, cam0, s, true);
    if (!rc) rc = higs_bin_sort(c, s);
    if (!rc) rc = higs_batch(c, s);
    if (!rc) rc = raster_frame(c, s);
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(s, &graph) != hipSuccess && !rc) rc = HIGS_E_HIP;
    if (!rc && hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess)
      rc = HIGS_E_HIP;
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) {
      destroy_graph(g);
      c->stage = 0;
      return rc;
    }
    c->graphs.push_back(g);
    gi = (int)c->graphs.size() - 1;
  }
  higs_ctx::Graph& g = c->graphs[(size_t)gi];
  // the last replay's copy has read the stage once its event completed
  if (g.launched && hipEventSynchronize(g.done) != hipSuccess) return HIGS_E_HIP;
  memcpy(g.stage, va, bytes);
  int rc = epoch_guard(c, s);
  if (rc) return rc;
  if (hipGraphLaunch(g.exec, s) != hipSuccess) return HIGS_E_HIP;
  if (hipEventRecord(g.done, s) != hipSuccess) return HIGS_E_HIP;
  g.launched = true;
  g.last_used = ++c->graph_tick;
  c->last_stream = s;
  c->stage = 4;
  return HIGS_OK;
}
}  // namespace

extern "C" {

int higs_raster(higs_ctx* c, float* image, float* T_out, void* stream) {
  if (!c || !image) return HIGS_E_INVALID;
  if (c->stage < 3 || c->n_views != 1) return HIGS_E_STATE;
  DeviceGuard g(c->device);
  c->views.v0.image = image;
  c->views.v0.T = T_out;
  return raster_frame(c, (hipStream_t)stream);
}

int higs_render(higs_ctx* c, int64_t n, const float* means, const float* scales,
                const float* quats, const float* opacities, const float* sh,
                const higs_camera* cam, float* image, float* T_out, void* stream) {
  if (!image) return HIGS_E_INVALID;
  if (c && cam && graph_frame(c, (hipStream_t)stream)) {
    higs_view v{};
    v.n = n;
    v.means = means;
    v.scales = scales;
    v.quats = quats;
    v.opacities = opacities;
    v.sh = sh;
    v.camera = *cam;
    v.image = image;
    v.T_out = T_out;
    return higs_render_views(c, 1, &v, stream);
  }
  int rc = higs_project(c, n, means, scales, quats, opacities, sh, cam, stream);
  if (rc) return rc;
  rc = higs_bin_sort(c, stream);
  if (rc) return rc;
  rc = higs_batch(c, stream);
  if (rc) return rc;
  return higs_raster(c, image, T_out, stream);
}

int higs_render_views(higs_ctx* c, int32_t n_views, const higs_view* views, void* stream) {
  if (!c || !views || n_views < 1) return HIGS_E_INVALID;
  if (n_views > c->params.max_views) return HIGS_E_CAPACITY;
  const higs_camera* cam0 = &views[0].camera;
  int64_t n_max = 0;
  for (int v = 0; v < n_views; ++v) {
    const higs_view& w = views[v];
    if (w.n < 0 || !w.image) return HIGS_E_INVALID;
    if (w.n > 0 && (!w.means || !w.scales || !w.quats || !w.opacities || !w.sh))
      return HIGS_E_INVALID;
    const int rc = check_camera(c, &w.camera);
    if (rc) return rc;
    if (w.camera.width != cam0->width || w.camera.height != cam0->height) return HIGS_E_INVALID;
    if (w.n > c->max_g) return HIGS_E_CAPACITY;
    n_max = w.n > n_max ? w.n : n_max;
  }
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  c->n = views[0].n;
  c->in_means = views[0].means;
  c->in_scales = views[0].scales;
  c->in_quats = views[0].quats;
  c->in_opac = views[0].opacities;
  c->in_sh = views[0].sh;
  c->n_views = n_views;
  c->n_pad = pad_blocks(n_max);
  if (graph_frame(c, s)) {
    ViewArgs va[HIGS_MAX_VIEWS];
    for (int v = 0; v < n_views; ++v) va[v] = view_args(views[v]);
    return render_graph(c, n_views, va, cam0, s);
  }
  ViewArgs* slot = nullptr;
  if (n_views > 1) {
    // the view table goes to the device from a pinned slot that no earlier
    // frame's copy still reads
    const int k = c->view_slot;
    c->view_slot = (c->view_slot + 1) % kViewRing;
    if (hipEventSynchronize(c->view_ev[k]) != hipSuccess) return HIGS_E_HIP;
    slot = c->view_stage + (size_t)k * c->params.max_views;
  }
  for (int v = 0; v < n_views; ++v) {
    const ViewArgs a = view_args(views[v]);
    if (v == 0) c->views.v0 = a;
    if (slot) slot[v] = a;
  }
  c->views.count = n_views;
  c->views.table = n_views > 1 ? c->view_table : nullptr;
  if (slot) {
    const int k = (c->view_slot + kViewRing - 1) % kViewRing;
    int rc = hip_err(hipMemcpyAsync(c->view_table, slot, sizeof(ViewArgs) * (size_t)n_views,
                                    hipMemcpyHostToDevice, s));
    if (!rc) rc = hip_err(hipEventRecord(c->view_ev[k], s));
    if (rc) return rc;
  }
  int rc = project_frame(c, cam0, s);
  if (rc) return rc;
  rc = higs_bin_sort(c, stream);
  if (rc) return rc;
  rc = higs_batch(c, stream);
  if (rc) return rc;
  return raster_frame(c, s);
}

int higs_raster_backward(higs_ctx* c, const float* dL_dimage, const float* dL_dT, float* dmeans,
                         float* dscales, float* dquats, float* dopacities, float* dsh,
                         void* stream) {
  if (!c || !dL_dimage) return HIGS_E_INVALID;
  if (c->n > 0 && (!dmeans || !dscales || !dquats || !dopacities || !dsh)) return HIGS_E_INVALID;
  if (c->stage < 4) return HIGS_E_STATE;
  if (c->params.raster_precision != HIGS_RASTER_FP32 || c->n_views != 1) return HIGS_E_UNSUPPORTED;
  DeviceGuard g(c->device);
  if (!c->bwd_state) {
    if (dalloc(&c->bwd_state, (size_t)c->max_batches * kTilesPerMt * 64) != HIGS_OK ||
        dalloc(&c->dgeo, (size_t)c->max_g * 16) != HIGS_OK) {
      if (c->bwd_state) (void)hipFree(c->bwd_state);
      if (c->dgeo) (void)hipFree(c->dgeo);
      c->bwd_state = nullptr;
      c->dgeo = nullptr;
      return HIGS_E_NOMEM;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  const uint32_t* v2[2] = {c->vals[0], c->vals[1]};
  float4* parts = c->partials;
  if (c->fused_frame) {
    // the frame folded its partials in the raster: rasterise it again (same
    // work items, same partials) into a buffer of the adjoint's
    if (!c->partials_bwd &&
        dalloc(&c->partials_bwd, (size_t)c->max_batches * kTilesPerMt * 64) != HIGS_OK)
      return HIGS_E_NOMEM;
    parts = c->partials_bwd;
    int rc = hip_err(launch_raster_rewind(c->dc, s));
    if (rc) return rc;
    rc = hip_err(launch_raster(c->ca, c->pa, c->views, v2, c->rec, c->batch_tab, c->chain_tab,
                               c->dc, parts, c->active, c->chain_acc, c->n_cus, false, false, s));
    if (rc) return rc;
  }
  return hip_err(launch_backward(c->n, c->in_means, c->in_scales, c->in_quats, c->in_sh, c->ca,
                                 c->pa, v2, c->rec, c->f_cnt, c->batch_tab, c->batch_first,
                                 c->active, parts, c->dc, dL_dimage, dL_dT, c->bwd_state,
                                 c->dgeo, dmeans, dscales, dquats, dopacities, dsh, c->n_cus, s));
}

int higs_get_counts(higs_ctx* c, higs_counts* out) {
  if (!c || !out) return HIGS_E_INVALID;
  DeviceGuard g(c->device);
  if (hipStreamSynchronize(c->last_stream) != hipSuccess) return HIGS_E_HIP;
  DeviceCounters h;
  if (hipMemcpy(&h, c->dc, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return HIGS_E_HIP;
  out->n_gaussians = c->n;
  out->n_visible = c->stage >= 2 ? (int64_t)h.n_visible : 0;
  out->n_pairs = c->stage >= 2 ? (int64_t)h.n_pairs_total : 0;
  out->n_batches = c->stage >= 3 ? (int64_t)h.n_batches_total : 0;
  out->overflow = h.overflow;
  out->sort_passes = c->stage >= 2 ? (int32_t)h.sort_passes : 0;
  out->n_evaluations = (c->stage >= 4 && (c->debug_flags & HIGS_DEBUG_COUNT_EVALS))
                           ? (int64_t)h.n_evals * 64
                           : -1;
  out->sort_pair_bytes = (c->stage < 2 || c->segmented()) ? 0 : (h.id_shift ? 8 : 12);
  out->graphs = (int32_t)c->graphs.size();
  return HIGS_OK;
}

namespace {
// Segmented sort read-back: pairs as macro-tile << 32 | depth bits and ids,
// rebuilt from the segment offsets (PAIRS: the filled composites, in segment
// order; SORTED: the sorted ids with each id's depth bits).
int seg_debug_pairs(higs_ctx* c, int which, const DeviceCounters& h, size_t np, char* dst,
                    size_t bytes) {
  std::vector<uint32_t> off((size_t)c->n_mt + 1);
  if (hipMemcpy(off.data(), c->mt_off, off.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return HIGS_E_HIP;
  uint32_t gbits = 0;
  for (int64_t v = c->n > 1 ? c->n - 1 : 0; v; v >>= 1) ++gbits;
  std::vector<uint64_t> keys(np);
  std::vector<uint32_t> ids(np);
  if (which == HIGS_DBG_PAIRS) {
    if (!(c->debug_flags & HIGS_DEBUG_KEEP_PAIRS) || !c->dbg_keys) return HIGS_E_STATE;
    std::vector<uint64_t> comp(np);
    if (np && hipMemcpy(comp.data(), c->dbg_keys, np * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return HIGS_E_HIP;
    for (size_t q = 0; q < np; ++q) {
      ids[q] = (uint32_t)(comp[q] & ((1ull << gbits) - 1ull));
      keys[q] = (uint32_t)((comp[q] >> gbits) + h.key_min);
    }
  } else {
    std::vector<uint32_t> fkey((size_t)c->n);
    if (np && hipMemcpy(ids.data(), c->vals[0], np * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return HIGS_E_HIP;
    if (c->n && hipMemcpy(fkey.data(), c->f_key, (size_t)c->n * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return HIGS_E_HIP;
    for (size_t q = 0; q < np; ++q) keys[q] = ids[q] < (uint32_t)c->n ? fkey[ids[q]] : 0u;
  }
  for (int m = 0; m < c->n_mt; ++m)
    for (uint32_t q = off[m]; q < off[m + 1] && q < np; ++q) keys[q] |= (uint64_t)m << 32;
  const size_t kb = bytes < np * 8 ? bytes : np * 8;
  memcpy(dst, keys.data(), kb);
  if (bytes > np * 8) memcpy(dst + np * 8, ids.data(), bytes - np * 8);
  return HIGS_OK;
}
}  // namespace

int higs_debug_copy(higs_ctx* c, int which, void* host_dst, size_t bytes) {
  if (!c || !host_dst) return HIGS_E_INVALID;
  DeviceGuard g(c->device);
  if (hipStreamSynchronize(c->last_stream) != hipSuccess) return HIGS_E_HIP;
  DeviceCounters h;
  if (hipMemcpy(&h, c->dc, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return HIGS_E_HIP;
  const size_t n = (size_t)c->n;
  const size_t np = h.n_pairs, nb = h.n_batches;
  char* dst = static_cast<char*>(host_dst);
  auto cp = [&](const void* src, size_t len) {
    return hipMemcpy(dst, src, len, hipMemcpyDeviceToHost) == hipSuccess ? HIGS_OK : HIGS_E_HIP;
  };
  switch (which) {
    case HIGS_DBG_PROJ: {
      if (c->stage < 1 || bytes > 8 * n * 4) return HIGS_E_INVALID;
      const void* cols[8] = {c->f_mx, c->f_my, c->f_a, c->f_b, c->f_c, c->f_tau, c->f_key, c->f_cnt};
      size_t left = bytes;
      for (int k = 0; k < 8 && left > 0; ++k) {
        const size_t len = left < n * 4 ? left : n * 4;
        if (hipMemcpy(dst + k * n * 4, cols[k], len, hipMemcpyDeviceToHost) != hipSuccess)
          return HIGS_E_HIP;
        left -= len;
      }
      return HIGS_OK;
    }
    case HIGS_DBG_RECORDS:
      if (c->stage < 1 || bytes > n * sizeof(RasterRecord)) return HIGS_E_INVALID;
      return cp(c->rec, bytes);
    case HIGS_DBG_PAIRS:
    case HIGS_DBG_SORTED: {
      if (c->stage < 2 || bytes > np * 12) return HIGS_E_INVALID;
      if (c->segmented()) return seg_debug_pairs(c, which, h, np, dst, bytes);
      const uint64_t* k;
      const uint32_t* v;
      if (which == HIGS_DBG_PAIRS) {
        if (!(c->debug_flags & HIGS_DEBUG_KEEP_PAIRS) || !c->dbg_keys) return HIGS_E_STATE;
        k = c->dbg_keys;
        v = c->dbg_vals;
      } else {
        k = c->keys[h.sort_final & 1u];
        v = c->vals[h.sort_final & 1u];
      }
      std::vector<uint64_t> words(np);
      if (np && hipMemcpy(words.data(), k, np * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return HIGS_E_HIP;
      std::vector<uint32_t> ids(np);
      const uint32_t ish = h.id_shift;
      if (ish) {  // one-word pairs: key << ish | id
        for (size_t q = 0; q < np; ++q) {
          ids[q] = (uint32_t)(words[q] & ((1ull << ish) - 1ull));
          words[q] >>= ish;
        }
      } else if (np && hipMemcpy(ids.data(), v, np * 4, hipMemcpyDeviceToHost) != hipSuccess) {
        return HIGS_E_HIP;
      }
      // keys are stored range-compressed; hand them back as
      // macro-tile << 32 | float32 depth bits
      const uint32_t dbits = depth_bits(h.key_min, h.key_max);
      for (size_t q = 0; q < np; ++q) {
        const uint64_t mt = dbits >= 64 ? 0 : words[q] >> dbits;
        const uint64_t dep = words[q] & ((dbits >= 64 ? 0ull : (1ull << dbits)) - 1ull);
        words[q] = (mt << 32) | (uint64_t)(uint32_t)(dep + h.key_min);
      }
      const size_t kb = bytes < np * 8 ? bytes : np * 8;
      memcpy(dst, words.data(), kb);
      if (bytes > np * 8) memcpy(dst + np * 8, ids.data(), bytes - np * 8);
      return HIGS_OK;
    }
    case HIGS_DBG_MT_OFFSETS:
      if (c->stage < 3 || bytes > ((size_t)c->n_mt_all + 1) * 4) return HIGS_E_INVALID;
      return cp(c->mt_off, bytes);
    case HIGS_DBG_BATCHES:
      if (c->stage < 3 || bytes > nb * 12) return HIGS_E_INVALID;
      return cp(c->batch_tab, bytes);
    case HIGS_DBG_ACTIVE:
      if (c->stage < 4 || bytes > nb * 4) return HIGS_E_INVALID;
      if (c->fused_frame) return HIGS_E_STATE;
      return cp(c->active, bytes);
    case HIGS_DBG_PARTIALS:
      if (c->stage < 4 || bytes > nb * kTilesPerMt * 64 * 16) return HIGS_E_INVALID;
      if (c->fused_frame) return HIGS_E_STATE;
      return cp(c->partials, bytes);
    default:
      return HIGS_E_INVALID;
  }
}

int higs_get_timers(higs_ctx* c, float ms[HIGS_NUM_TIMERS]) {
  if (!c || !ms) return HIGS_E_INVALID;
  if (!c->timing() || c->frames < 1 || c->stage < 4) return HIGS_E_STATE;
  DeviceGuard g(c->device);
  if (hipStreamSynchronize(c->last_stream) != hipSuccess) return HIGS_E_HIP;
  // frames recorded in the ring: the last min(frames, ring), all complete
  const int64_t have = c->frames < c->ring ? c->frames : c->ring;
  for (int k = 0; k < HIGS_NUM_TIMERS; ++k) {
    double sum = 0.0;
    for (int64_t f = 0; f < have; ++f) {
      float t = 0.0f;
      const hipEvent_t* e = c->ev + (f * HIGS_NUM_TIMERS + k) * 2;
      if (hipEventElapsedTime(&t, e[0], e[1]) != hipSuccess) return HIGS_E_HIP;
      sum += t;
    }
    ms[k] = (float)(sum / (double)have);
  }
  return HIGS_OK;
}

}  // extern "C"

// ---- packed SH -----------------------------------------------------------------
extern "C" int64_t higs_sh_packed_bytes(int64_t n) {
  if (n < 0) return HIGS_E_INVALID;
  return (int64_t)kShHeaderBytes + 32 * n;
}

extern "C" int higs_sh_compress(int64_t n, const float* sh, const float* opacities, void* packed,
                                void* stream) {
  if (n < 0 || !packed || (n > 0 && (!sh || !opacities))) return HIGS_E_INVALID;
  if ((reinterpret_cast<uintptr_t>(packed) & 15u) != 0) return HIGS_E_INVALID;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HIGS_E_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return HIGS_E_HIP;
  hipStream_t s = (hipStream_t)stream;
  uint32_t* work = nullptr;
  if (dalloc(&work, (size_t)kShComps * (1 + 1024) + 1) != HIGS_OK) return HIGS_E_NOMEM;
  int rc = hip_err(launch_sh_compress(n, sh, opacities, packed, work, prop.multiProcessorCount, s));
  if (!rc) rc = hip_err(hipStreamSynchronize(s));
  (void)hipFree(work);
  return rc;
}

// ---- allocation-free rendering ------------------------------------------------
// One frame of the whole path with every intermediate in a static device array
// instead of a context's allocations: for callers that cannot allocate device
// memory (code under stream capture, serving loops that must not call
// hipMalloc).  The capacities are fixed; the array lives on every device the
// library runs on until the process ends.
namespace {
constexpr int64_t kNaMaxGaussians = 131072;
constexpr int64_t kNaMaxPairs = 524288;
// every macro-tile holds at most one partly filled batch: pairs / B_r plus one
// per macro-tile bounds the batch count, so pairs that fit never overflow it
constexpr int32_t kNaMaxWidth = 1024, kNaMaxHeight = 1024;
constexpr int64_t kNaMaxBatches = kNaMaxPairs / kMaxBatch +
                                  (int64_t)((kNaMaxWidth + kMtW - 1) / kMtW) *
                                      ((kNaMaxHeight + kMtH - 1) / kMtH) + 16;
constexpr size_t kScratchBytes = (size_t)80 << 20;
constexpr int kNaMaxDevices = 16;

struct NoAllocState {
  bool ready = false;
  unsigned char* base = nullptr;  // device address of this device's scratch array
  higs_ctx ctx;
};
NoAllocState g_noalloc[kNaMaxDevices];
std::mutex g_noalloc_mu;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

extern "C" int higs_render_noalloc(int64_t n, const float* means, const float* scales,
                                   const float* quats, const float* opacities, const float* sh,
                                   const higs_camera* cam, float* image, float* T_out,
                                   void* stream) {
  if (!cam || !image || n < 0) return HIGS_E_INVALID;
  if (n > kNaMaxGaussians || cam->width > kNaMaxWidth || cam->height > kNaMaxHeight)
    return HIGS_E_CAPACITY;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HIGS_E_HIP;
  if (dev < 0 || dev >= kNaMaxDevices) return HIGS_E_UNSUPPORTED;
  NoAllocState& st = g_noalloc[dev];
  hipStream_t s = (hipStream_t)stream;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!st.ready) {
      // once per device, with that device current: the array's device address
      // (the symbol's host-side name is no device address)
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HIGS_E_HIP;
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return HIGS_E_HIP;
      higs_ctx& c = st.ctx;
      c.device = dev;
      c.n_cus = prop.multiProcessorCount;
      higs_default_params(&c.params);
      set_capacities(&c, kNaMaxGaussians, kNaMaxPairs, kNaMaxBatches, kNaMaxWidth, kNaMaxHeight);
      st.base = static_cast<unsigned char*>(ptr);
      if (!carve(&c, st.base, kScratchBytes)) return HIGS_E_UNSUPPORTED;
      // the sort's look-back words start untagged, by a kernel on the
      // caller's stream (the frame's own kernels clear the counters)
      int rc = hip_err(launch_zero_words(c.status, (size_t)c.max_tiles * kRadix, s));
      if (!rc) rc = hip_err(launch_zero_words(reinterpret_cast<uint64_t*>(c.dc),
                                              sizeof(DeviceCounters) / 8, s));
      if (rc) return rc;
      st.ready = true;
    }
  }
  return higs_render(&st.ctx, n, means, scales, quats, opacities, sh, cam, image, T_out, stream);
}

namespace higs {
int ctx_enqueue_counters(higs_ctx* c, void* pinned_dst, hipStream_t s) {
  if (!c || !pinned_dst) return HIGS_E_INVALID;
  return hip_err(hipMemcpyAsync(pinned_dst, c->dc, sizeof(DeviceCounters), hipMemcpyDeviceToHost, s));
}
}  // namespace higs
