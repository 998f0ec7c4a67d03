// Render server: resident scenes, a request queue, continuous batching over
// frame contexts, one HIP stream per context.
//
// Scheduling (all on the caller's host thread, driven by higs_server_poll):
//   retire: a busy context whose end event has completed is done; its frame
//     counters (copied into pinned memory behind the frame on the same stream)
//     report capacity overflow; the frame's device time comes from the two
//     events around it.
//   admit: queued requests in arrival order; a request takes an idle context
//     of its resolution class, else a new one if the contexts held stay within
//     the HBM budget after releasing idle contexts of other classes (least
//     recently used first).  A request that cannot be placed stays queued, and
//     while it does the requests behind it may only reuse idle contexts (no new
//     ones), so the next freed memory goes to it.  At most max_in_flight frames
//     render at once; max_in_flight = 1 is the plain one-frame-at-a-time
//     renderer.
// Frames on different contexts share nothing but the read-only scene arrays,
// so a request's image is the same alone and in the mix (every stage is
// deterministic).
#include <deque>
#include <new>
#include <vector>

#include "higs_internal.h"

using namespace higs;

namespace {

struct Scene {
  int32_t id = -1;
  int64_t n = 0;
  const float *means = nullptr, *scales = nullptr, *quats = nullptr, *opac = nullptr,
              *sh = nullptr;
};

struct Request {
  int64_t id;
  int32_t scene, cls;
  higs_camera cam;
  float* image;
};

struct Slot {
  higs_ctx* ctx = nullptr;
  int32_t cls = 0;
  hipStream_t stream = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  DeviceCounters* counters = nullptr;  // pinned host copy of the frame counters
  int64_t bytes = 0;
  bool busy = false;
  int64_t request = -1;
  uint64_t last_used = 0;
};

}  // namespace

struct higs_server {
  int device = 0;
  higs_params params{};
  higs_server_config cfg{};
  std::vector<Scene> scenes;
  std::vector<Slot*> slots;
  std::deque<Request> queue;
  int64_t bytes = 0, completed = 0, evictions = 0;
  int32_t in_flight = 0;
  uint64_t tick = 0;
};

namespace {

int64_t class_batches(const higs_server* s, int cls) {
  const int64_t n_mt = (int64_t)((s->cfg.width[cls] + kMtW - 1) / kMtW) *
                       ((s->cfg.height[cls] + kMtH - 1) / kMtH);
  return s->cfg.max_pairs[cls] / s->params.batch_cap + n_mt + 16;
}

int64_t class_footprint(const higs_server* s, int cls) {
  return higs_ctx_footprint(&s->params, s->cfg.max_gaussians, s->cfg.max_pairs[cls],
                            class_batches(s, cls), s->cfg.width[cls], s->cfg.height[cls]);
}

void destroy_slot(higs_server* s, Slot* sl) {
  if (sl->ctx) higs_ctx_destroy(sl->ctx);
  if (sl->e0) (void)hipEventDestroy(sl->e0);
  if (sl->e1) (void)hipEventDestroy(sl->e1);
  if (sl->stream) (void)hipStreamDestroy(sl->stream);
  if (sl->counters) (void)hipHostFree(sl->counters);
  s->bytes -= sl->bytes;
  delete sl;
}

Slot* create_slot(higs_server* s, int cls) {
  Slot* sl = new (std::nothrow) Slot();
  if (!sl) return nullptr;
  sl->cls = cls;
  sl->bytes = class_footprint(s, cls);
  s->bytes += sl->bytes;
  bool ok = higs_ctx_create(s->device, &s->params, s->cfg.max_gaussians, s->cfg.max_pairs[cls],
                            class_batches(s, cls), s->cfg.width[cls], s->cfg.height[cls],
                            &sl->ctx) == HIGS_OK;
  ok = ok && hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreate(&sl->e0) == hipSuccess && hipEventCreate(&sl->e1) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&sl->counters), sizeof(DeviceCounters),
                           hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    destroy_slot(s, sl);
    return nullptr;
  }
  s->slots.push_back(sl);
  return sl;
}

// Releases idle contexts of classes other than `cls`, least recently used
// first, until `need` more bytes fit the budget.  True if they fit.
bool make_room(higs_server* s, int cls, int64_t need) {
  while (s->bytes + need > s->cfg.hbm_budget) {
    Slot* victim = nullptr;
    size_t at = 0;
    for (size_t k = 0; k < s->slots.size(); ++k) {
      Slot* c = s->slots[k];
      if (c->busy || c->cls == cls) continue;
      if (!victim || c->last_used < victim->last_used) {
        victim = c;
        at = k;
      }
    }
    if (!victim) return false;
    s->slots.erase(s->slots.begin() + (long)at);
    destroy_slot(s, victim);
    s->evictions += 1;
  }
  return true;
}

const Scene* find_scene(const higs_server* s, int32_t id) {
  for (const Scene& sc : s->scenes)
    if (sc.id == id) return &sc;
  return nullptr;
}

int launch(higs_server* s, Slot* sl, const Request& r) {
  const Scene* sc = find_scene(s, r.scene);
  if (!sc) return HIGS_E_INVALID;
  if (hipEventRecord(sl->e0, sl->stream) != hipSuccess) return HIGS_E_HIP;
  int rc = higs_render(sl->ctx, sc->n, sc->means, sc->scales, sc->quats, sc->opac, sc->sh, &r.cam,
                       r.image, nullptr, sl->stream);
  if (rc) return rc;
  rc = ctx_enqueue_counters(sl->ctx, sl->counters, sl->stream);
  if (rc) return rc;
  if (hipEventRecord(sl->e1, sl->stream) != hipSuccess) return HIGS_E_HIP;
  sl->busy = true;
  sl->request = r.id;
  sl->last_used = ++s->tick;
  s->in_flight += 1;
  return HIGS_OK;
}

}  // namespace

extern "C" {

int higs_server_create(int device, const higs_params* params, const higs_server_config* cfg,
                       higs_server** out) {
  if (!out || !cfg) return HIGS_E_INVALID;
  *out = nullptr;
  if (cfg->n_classes < 1 || cfg->n_classes > HIGS_MAX_CLASSES || cfg->max_gaussians < 1 ||
      cfg->hbm_budget < 1 || cfg->max_in_flight < 1)
    return HIGS_E_INVALID;
  for (int c = 0; c < cfg->n_classes; ++c)
    if (cfg->width[c] < 1 || cfg->height[c] < 1 || cfg->max_pairs[c] < 1) return HIGS_E_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HIGS_E_INVALID;
  higs_server* s = new (std::nothrow) higs_server();
  if (!s) return HIGS_E_NOMEM;
  s->device = device;
  if (params) s->params = *params;
  else higs_default_params(&s->params);
  if (s->params.batch_cap < 1 || s->params.batch_cap > kMaxBatch) {
    delete s;
    return HIGS_E_INVALID;
  }
  s->cfg = *cfg;
  *out = s;
  return HIGS_OK;
}

int higs_server_destroy(higs_server* s) {
  if (!s) return HIGS_E_INVALID;
  for (Slot* sl : s->slots) {
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
    destroy_slot(s, sl);
  }
  delete s;
  return HIGS_OK;
}

int higs_server_add_scene(higs_server* s, int32_t scene_id, int64_t n, const float* means,
                          const float* scales, const float* quats, const float* opacities,
                          const float* sh) {
  if (!s || n < 0 || n > s->cfg.max_gaussians) return HIGS_E_INVALID;
  if (n > 0 && (!means || !scales || !quats || !opacities || !sh)) return HIGS_E_INVALID;
  if (find_scene(s, scene_id)) return HIGS_E_INVALID;
  Scene sc;
  sc.id = scene_id;
  sc.n = n;
  sc.means = means;
  sc.scales = scales;
  sc.quats = quats;
  sc.opac = opacities;
  sc.sh = sh;
  s->scenes.push_back(sc);
  return HIGS_OK;
}

int higs_server_submit(higs_server* s, int64_t request_id, int32_t scene_id, int32_t cls,
                       const higs_camera* cam, float* image) {
  if (!s || !cam || !image || cls < 0 || cls >= s->cfg.n_classes) return HIGS_E_INVALID;
  if (!find_scene(s, scene_id)) return HIGS_E_INVALID;
  if (cam->width < 1 || cam->height < 1 || cam->width > s->cfg.width[cls] ||
      cam->height > s->cfg.height[cls])
    return HIGS_E_CAPACITY;
  s->queue.push_back(Request{request_id, scene_id, cls, *cam, image});
  return HIGS_OK;
}

int higs_server_poll(higs_server* s, higs_completion* done, int32_t max_done) {
  if (!s || (max_done > 0 && !done) || max_done < 0) return HIGS_E_INVALID;
  int32_t n_done = 0;
  // retire finished frames
  for (Slot* sl : s->slots) {
    if (!sl->busy || n_done >= max_done) continue;
    const hipError_t q = hipEventQuery(sl->e1);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return HIGS_E_HIP;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, sl->e0, sl->e1) != hipSuccess) ms = -1.0f;
    done[n_done].request_id = sl->request;
    done[n_done].gpu_ms = ms;
    done[n_done].overflow = sl->counters->overflow;
    done[n_done].cls = sl->cls;
    ++n_done;
    sl->busy = false;
    sl->request = -1;
    s->in_flight -= 1;
    s->completed += 1;
  }
  // admit queued requests
  bool blocked = false;  // an earlier request is waiting for memory
  for (auto it = s->queue.begin(); it != s->queue.end() && s->in_flight < s->cfg.max_in_flight;) {
    Slot* sl = nullptr;
    for (Slot* c : s->slots)
      if (!c->busy && c->cls == it->cls && (!sl || c->last_used > sl->last_used)) sl = c;
    if (!sl && !blocked) {
      const int64_t need = class_footprint(s, it->cls);
      if (need > 0 && make_room(s, it->cls, need)) sl = create_slot(s, it->cls);
    }
    if (!sl) {
      blocked = true;
      ++it;
      continue;
    }
    const int rc = launch(s, sl, *it);
    if (rc) return rc;
    it = s->queue.erase(it);
  }
  return n_done;
}

int higs_server_get_stats(higs_server* s, higs_server_stats* out) {
  if (!s || !out) return HIGS_E_INVALID;
  out->queued = (int32_t)s->queue.size();
  out->in_flight = s->in_flight;
  out->contexts = (int32_t)s->slots.size();
  out->bytes = s->bytes;
  out->completed = s->completed;
  out->evictions = s->evictions;
  return HIGS_OK;
}

}  // extern "C"
