// Render server: resident scenes, a request queue, continuous batching over
// frame contexts, one HIP stream per context, several requests per frame.
//
// Memory: one device arena of hbm_budget bytes, allocated when the server is
// created.  A frame context's buffers are a range of the arena (first fit;
// freed ranges merge with their neighbours), so creating and releasing
// contexts while serving allocates and frees no device memory and never
// synchronises the device.
//
// Scheduling (all on the caller's host thread, driven by higs_server_poll):
//   retire: a busy context whose end event has completed is done; every
//     request of its frame completes (its frame counters, copied into pinned
//     memory behind the frame on the same stream, report capacity overflow;
//     the frame's device time comes from the two events around it).
//   admit: queued requests in arrival order; a request takes an idle context
//     of its resolution class, else a new one if its range fits the arena
//     after releasing idle contexts of other classes (least recently used
//     first).  The frame then also takes the next queued requests of the same
//     class and image size, up to the class's views per frame, so that one
//     launch per kernel renders all of them (higs_render_views).  A request
//     that cannot be placed stays queued, and while it does the requests
//     behind it may only reuse idle contexts (no new ones), so the next freed
//     memory goes to it.  At most max_in_flight frames render at once;
//     max_in_flight = 1 with one view per frame is the plain
//     one-frame-at-a-time renderer.
// Ordering: a frame waits (hipStreamWaitEvent) for the events recorded on the
// caller's streams when its scenes were added and its requests submitted, so
// that the work which wrote the scene arrays or last touched an image comes
// first.  Frames on different contexts share nothing but the read-only scene
// arrays, and every stage is deterministic, so a request's image is the same
// alone and in the mix.
#include <algorithm>
#include <chrono>
#include <deque>
#include <list>
#include <new>
#include <vector>

#include "higs_internal.h"

using namespace higs;

namespace {

struct Guard {
  int prev = -1;
  explicit Guard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~Guard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

struct Scene {
  int32_t id = -1;
  int64_t n = 0;
  const float *means = nullptr, *scales = nullptr, *quats = nullptr, *opac = nullptr,
              *sh = nullptr;
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at add time
};

struct Request {
  int64_t id;
  int32_t scene, cls;
  higs_camera cam;
  float* image;
  hipEvent_t dep;  // recorded on the caller's stream at submit time, or null
};

// Stream, events and pinned counters of a context; kept for reuse when the
// context is released.
struct Shell {
  hipStream_t stream = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  DeviceCounters* counters = nullptr;
};

struct Slot {
  higs_ctx* ctx = nullptr;
  Shell sh;
  int32_t cls = 0, views = 1, batch_cap = 0;
  size_t off = 0, bytes = 0;  // its range of the arena
  bool busy = false;
  std::vector<int64_t> requests;  // of the frame in flight
  uint64_t last_used = 0;
};

// First-fit ranges of the arena (offsets aligned to 2 MiB).
struct Arena {
  unsigned char* base = nullptr;
  size_t size = 0;
  std::vector<std::pair<size_t, size_t>> free;  // (offset, length), by offset
  static constexpr size_t kAlign = (size_t)2 << 20;
  static size_t round(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
  bool take(size_t bytes, size_t* off) {
    const size_t need = round(bytes);
    for (size_t k = 0; k < free.size(); ++k) {
      if (free[k].second < need) continue;
      *off = free[k].first;
      free[k].first += need;
      free[k].second -= need;
      if (free[k].second == 0) free.erase(free.begin() + (long)k);
      return true;
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    const size_t len = round(bytes);
    auto it = std::lower_bound(free.begin(), free.end(), std::make_pair(off, (size_t)0));
    it = free.insert(it, {off, len});
    // merge with the next range, then with the previous one
    auto nx = it + 1;
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = it - 1;
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

struct Done {
  int64_t request;
  float ms;
  uint32_t overflow;
  int32_t cls, views;
};

}  // namespace

struct higs_server {
  int device = 0;
  higs_params params{};
  higs_server_config cfg{};
  int32_t views[HIGS_MAX_CLASSES] = {};      // views per frame of each class
  int32_t batch_cap[HIGS_MAX_CLASSES] = {};  // B_r of each class's contexts
  std::vector<Scene> scenes;
  std::vector<Slot*> slots;
  std::vector<Shell> shells;        // idle shells
  std::vector<hipEvent_t> events;   // idle dependency events
  std::list<Request> queue;         // arrival order (a frame may take requests from its middle)
  std::deque<Done> done;            // retired, not yet returned by poll
  Arena arena;
  int64_t completed = 0, evictions = 0, frames = 0;
  int32_t in_flight = 0;
  int error = 0;                    // an error met after completions were retired
  uint64_t tick = 0;
};

namespace {

int64_t class_pairs(const higs_server* s, int cls, int views) {
  return s->cfg.max_pairs[cls] * (int64_t)views;
}

int64_t class_batches(const higs_server* s, int cls, int views, int cap) {
  const int64_t n_mt = (int64_t)((s->cfg.width[cls] + kMtW - 1) / kMtW) *
                       ((s->cfg.height[cls] + kMtH - 1) / kMtH);
  return class_pairs(s, cls, views) / cap + n_mt * views + 16;
}

higs_params class_params(const higs_server* s, int views, int cap) {
  higs_params p = s->params;
  p.max_views = views;
  p.batch_cap = cap;
  p.use_graphs = s->cfg.use_graphs ? 1 : 0;
  return p;
}

int64_t slot_bytes(const higs_server* s, int cls, int views, int cap) {
  const higs_params p = class_params(s, views, cap);
  return ctx_arena_bytes(&p, s->cfg.max_gaussians, class_pairs(s, cls, views),
                         class_batches(s, cls, views, cap), s->cfg.width[cls], s->cfg.height[cls]);
}

bool get_shell(higs_server* s, Shell* out) {
  if (!s->shells.empty()) {
    *out = s->shells.back();
    s->shells.pop_back();
    return true;
  }
  Shell sh;
  bool ok = hipStreamCreateWithFlags(&sh.stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreate(&sh.e0) == hipSuccess && hipEventCreate(&sh.e1) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&sh.counters), sizeof(DeviceCounters),
                           hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    if (sh.e0) (void)hipEventDestroy(sh.e0);
    if (sh.e1) (void)hipEventDestroy(sh.e1);
    if (sh.stream) (void)hipStreamDestroy(sh.stream);
    if (sh.counters) (void)hipHostFree(sh.counters);
    return false;
  }
  *out = sh;
  return true;
}

void free_shell(Shell& sh) {
  if (sh.stream) (void)hipStreamSynchronize(sh.stream);
  if (sh.e0) (void)hipEventDestroy(sh.e0);
  if (sh.e1) (void)hipEventDestroy(sh.e1);
  if (sh.stream) (void)hipStreamDestroy(sh.stream);
  if (sh.counters) (void)hipHostFree(sh.counters);
  sh = Shell();
}

// Releases an idle slot: its context's host state, its arena range, its shell
// (kept for the next context).  The slot's last frame has completed.
void release_slot(higs_server* s, Slot* sl) {
  if (sl->ctx) (void)ctx_release(sl->ctx);
  s->arena.give(sl->off, sl->bytes);
  s->shells.push_back(sl->sh);
  delete sl;
}

Slot* create_slot(higs_server* s, int cls, int views, int cap, size_t off, size_t bytes) {
  Slot* sl = new (std::nothrow) Slot();
  if (!sl) return nullptr;
  if (!get_shell(s, &sl->sh)) {
    delete sl;
    return nullptr;
  }
  sl->cls = cls;
  sl->views = views;
  sl->batch_cap = cap;
  sl->off = off;
  sl->bytes = bytes;
  const higs_params p = class_params(s, views, cap);
  if (ctx_create_in(s->device, &p, s->cfg.max_gaussians, class_pairs(s, cls, views),
                    class_batches(s, cls, views, cap), s->cfg.width[cls], s->cfg.height[cls],
                    s->arena.base + off, bytes, sl->sh.stream, &sl->ctx) != HIGS_OK) {
    s->shells.push_back(sl->sh);
    delete sl;
    return nullptr;
  }
  s->slots.push_back(sl);
  return sl;
}

// A new context for class cls, in an arena range freed if need be by
// releasing idle contexts of other classes, least recently used first (idle
// contexts of the class itself too when `any_class`, or when made for an
// earlier setting of the class).  Null if none fits.
Slot* make_slot(higs_server* s, int cls, bool any_class) {
  const int views = s->views[cls], cap = s->batch_cap[cls];
  const int64_t b = slot_bytes(s, cls, views, cap);
  if (b <= 0) return nullptr;
  size_t off = 0;
  while (!s->arena.take((size_t)b, &off)) {
    Slot* victim = nullptr;
    size_t at = 0;
    for (size_t k = 0; k < s->slots.size(); ++k) {
      Slot* c = s->slots[k];
      // (an idle context of the class that no longer has the class's
      // setting may go too)
      if (c->busy || (!any_class && c->cls == cls && c->views == s->views[cls] &&
                      c->batch_cap == s->batch_cap[cls]))
        continue;
      if (!victim || c->last_used < victim->last_used) {
        victim = c;
        at = k;
      }
    }
    if (!victim) return nullptr;
    s->slots.erase(s->slots.begin() + (long)at);
    release_slot(s, victim);
    s->evictions += 1;
  }
  Slot* sl = create_slot(s, cls, views, cap, off, (size_t)b);
  if (!sl) s->arena.give(off, (size_t)b);
  return sl;
}

const Scene* find_scene(const higs_server* s, int32_t id) {
  for (const Scene& sc : s->scenes)
    if (sc.id == id) return &sc;
  return nullptr;
}

void give_event(higs_server* s, hipEvent_t e) {
  if (e) s->events.push_back(e);
}

// Renders the requests group[0 .. n) as one frame on the slot.
int launch(higs_server* s, Slot* sl, const Request* const* group, int n) {
  higs_view vs[HIGS_MAX_VIEWS];
  hipStream_t st = sl->sh.stream;
  for (int k = 0; k < n; ++k) {
    const Request& r = *group[k];
    Scene* sc = const_cast<Scene*>(find_scene(s, r.scene));
    if (!sc) return HIGS_E_INVALID;
    if (sc->ready) {
      const hipError_t q = hipEventQuery(sc->ready);
      if (q == hipSuccess) {  // the scene's arrays are written: no more waits
        give_event(s, sc->ready);
        sc->ready = nullptr;
      } else if (q != hipErrorNotReady ||
                 hipStreamWaitEvent(st, sc->ready, 0) != hipSuccess) {
        return HIGS_E_HIP;
      }
    }
    if (r.dep && hipStreamWaitEvent(st, r.dep, 0) != hipSuccess) return HIGS_E_HIP;
    higs_view& v = vs[k];
    v = higs_view{};
    v.n = sc->n;
    v.means = sc->means;
    v.scales = sc->scales;
    v.quats = sc->quats;
    v.opacities = sc->opac;
    v.sh = sc->sh;
    v.camera = r.cam;
    v.image = r.image;
    v.T_out = nullptr;
  }
  if (hipEventRecord(sl->sh.e0, st) != hipSuccess) return HIGS_E_HIP;
  int rc = higs_render_views(sl->ctx, n, vs, st);
  if (rc) return rc;
  rc = ctx_enqueue_counters(sl->ctx, sl->sh.counters, st);
  if (rc) return rc;
  if (hipEventRecord(sl->sh.e1, st) != hipSuccess) return HIGS_E_HIP;
  sl->busy = true;
  sl->requests.clear();
  for (int k = 0; k < n; ++k) sl->requests.push_back(group[k]->id);
  sl->last_used = ++s->tick;
  s->in_flight += 1;
  s->frames += 1;
  return HIGS_OK;
}

// Retires finished frames into s->done.
int retire(higs_server* s) {
  for (Slot* sl : s->slots) {
    if (!sl->busy) continue;
    const hipError_t q = hipEventQuery(sl->sh.e1);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return HIGS_E_HIP;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, sl->sh.e0, sl->sh.e1) != hipSuccess) ms = -1.0f;
    const uint32_t ovf = sl->sh.counters->overflow;
    for (int64_t id : sl->requests)
      s->done.push_back(Done{id, ms, ovf, sl->cls, (int32_t)sl->requests.size()});
    s->completed += (int64_t)sl->requests.size();
    sl->requests.clear();
    sl->busy = false;
    s->in_flight -= 1;
  }
  return HIGS_OK;
}

// Admits queued requests (see the scheduling notes at the top).
int admit(higs_server* s) {
  bool blocked = false;  // an earlier request is waiting for memory
  for (auto it = s->queue.begin(); it != s->queue.end() && s->in_flight < s->cfg.max_in_flight;) {
    Slot* sl = nullptr;
    for (Slot* c : s->slots)
      if (!c->busy && c->cls == it->cls && c->views == s->views[it->cls] &&
          c->batch_cap == s->batch_cap[it->cls] && (!sl || c->last_used > sl->last_used))
        sl = c;
    if (!sl && !blocked) sl = make_slot(s, it->cls, false);
    if (!sl) {
      blocked = true;
      ++it;
      continue;
    }
    // the frame: this request and the next ones of its class and image size
    const Request* group[HIGS_MAX_VIEWS];
    std::list<Request>::iterator taken[HIGS_MAX_VIEWS];
    int n = 0;
    for (auto jt = it; jt != s->queue.end() && n < sl->views; ++jt) {
      if (jt->cls != it->cls || jt->cam.width != it->cam.width || jt->cam.height != it->cam.height)
        continue;
      group[n] = &*jt;
      taken[n++] = jt;
    }
    const int rc = launch(s, sl, group, n);
    if (rc) return rc;
    for (int k = 0; k < n; ++k) give_event(s, group[k]->dep);
    // list erasure leaves the other iterators valid; taken[0] is `it`
    for (int k = n - 1; k >= 1; --k) s->queue.erase(taken[k]);
    it = s->queue.erase(taken[0]);
  }
  return HIGS_OK;
}

// An event recorded now on the caller's stream (null: the legacy default
// stream), for a frame to wait on.
int record_dep(higs_server* s, void* stream, hipEvent_t* out) {
  *out = nullptr;
  hipEvent_t e = nullptr;
  if (!s->events.empty()) {
    e = s->events.back();
    s->events.pop_back();
  } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    return HIGS_E_HIP;
  }
  if (hipEventRecord(e, (hipStream_t)stream) != hipSuccess) {
    s->events.push_back(e);
    return HIGS_E_HIP;
  }
  *out = e;
  return HIGS_OK;
}

// Frames per second of `frames` back-to-back frames of `views` views each on
// `k` contexts (round robin) of class cls with batch cap `cap`, or a negative
// error.  The server holds no context meanwhile.
double trial(higs_server* s, int cls, const Scene& sc, int n_cams, const higs_camera* cams,
             int views, int cap, int frames, int* rc_out) {
  *rc_out = HIGS_OK;
  const int64_t b = slot_bytes(s, cls, views, cap);
  // serving holds contexts of every class: a trial gets the class's share of
  // the arena, and as many contexts (up to max_in_flight) as the share holds
  const size_t share = s->arena.size / (size_t)s->cfg.n_classes;
  if (b <= 0 || Arena::round((size_t)b) > share) return 0.0;
  const int k = std::max(1, std::min({s->cfg.max_in_flight, frames,
                                      (int)(share / Arena::round((size_t)b))}));
  const size_t px = (size_t)s->cfg.width[cls] * s->cfg.height[cls] * 3;
  float* images = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&images), px * 4 * (size_t)views * k) != hipSuccess) {
    *rc_out = HIGS_E_NOMEM;
    return 0.0;
  }
  const int saved_views = s->views[cls], saved_cap = s->batch_cap[cls];
  s->views[cls] = views;
  s->batch_cap[cls] = cap;
  // up to k contexts, as many as the (otherwise empty) arena holds
  std::vector<Slot*> mine;
  int rc = HIGS_OK;
  for (int i = 0; i < k && !rc; ++i) {
    size_t off = 0;
    if (!s->arena.take((size_t)b, &off)) break;
    Slot* sl = create_slot(s, cls, views, cap, off, (size_t)b);
    if (!sl) {
      s->arena.give(off, (size_t)b);
      rc = HIGS_E_NOMEM;
    } else {
      mine.push_back(sl);
    }
  }
  if (!rc && mine.empty()) rc = HIGS_E_NOMEM;
  double fps = 0.0;
  if (!rc) {
    std::vector<Request> reqs((size_t)views * k);
    auto run = [&](int count, int first_cam) -> int {
      for (int f = 0; f < count; ++f) {
        Slot* sl = mine[(size_t)f % mine.size()];
        if (sl->busy && hipStreamSynchronize(sl->sh.stream) != hipSuccess) return HIGS_E_HIP;
        sl->busy = false;
        const Request* group[HIGS_MAX_VIEWS];
        for (int v = 0; v < views; ++v) {
          Request& r = reqs[((size_t)f % mine.size()) * views + v];
          r = Request{-1, sc.id, cls, cams[(first_cam + f * views + v) % n_cams],
                      images + px * (((size_t)f % mine.size()) * views + v), nullptr};
          group[v] = &r;
        }
        const int e = launch(s, sl, group, views);
        if (e) return e;
        s->in_flight -= 1;  // not a served frame
        s->frames -= 1;
      }
      for (Slot* sl : mine) {
        if (hipStreamSynchronize(sl->sh.stream) != hipSuccess) return HIGS_E_HIP;
        sl->busy = false;
      }
      return HIGS_OK;
    };
    rc = run((int)mine.size() * 2, 0);  // warm-up (records the graphs)
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (!rc && (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess))
      rc = HIGS_E_HIP;
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = HIGS_E_HIP;
    const auto h0 = std::chrono::steady_clock::now();
    if (!rc) rc = run(frames, 7);
    const auto h1 = std::chrono::steady_clock::now();
    if (!rc) {
      const double sec = std::chrono::duration<double>(h1 - h0).count();
      fps = sec > 0.0 ? (double)frames * views / sec : 0.0;
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  }
  for (Slot* sl : mine) {
    sl->busy = false;
    s->slots.erase(std::find(s->slots.begin(), s->slots.end(), sl));
    release_slot(s, sl);
  }
  (void)hipFree(images);
  s->views[cls] = saved_views;
  s->batch_cap[cls] = saved_cap;
  *rc_out = rc;
  return fps;
}

}  // namespace

extern "C" {

int higs_server_create(int device, const higs_params* params, const higs_server_config* cfg,
                       higs_server** out) {
  if (!out || !cfg) return HIGS_E_INVALID;
  *out = nullptr;
  if (cfg->n_classes < 1 || cfg->n_classes > HIGS_MAX_CLASSES || cfg->max_gaussians < 1 ||
      cfg->hbm_budget < 1 || cfg->max_in_flight < 1 || (cfg->use_graphs != 0 && cfg->use_graphs != 1))
    return HIGS_E_INVALID;
  for (int c = 0; c < cfg->n_classes; ++c) {
    if (cfg->width[c] < 1 || cfg->height[c] < 1 || cfg->max_pairs[c] < 1) return HIGS_E_INVALID;
    if (cfg->views_per_frame[c] < 0 || cfg->views_per_frame[c] > HIGS_MAX_VIEWS)
      return HIGS_E_INVALID;
  }
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
  for (int c = 0; c < cfg->n_classes; ++c) {
    s->views[c] = cfg->views_per_frame[c] > 0 ? cfg->views_per_frame[c] : 1;
    s->batch_cap[c] = s->params.batch_cap;
    if (slot_bytes(s, c, s->views[c], s->batch_cap[c]) < 0) {
      delete s;
      return HIGS_E_INVALID;
    }
  }
  Guard g(device);
  s->arena.size = (size_t)cfg->hbm_budget / Arena::kAlign * Arena::kAlign;
  if (s->arena.size == 0 ||
      hipMalloc(reinterpret_cast<void**>(&s->arena.base), s->arena.size) != hipSuccess) {
    delete s;
    return HIGS_E_NOMEM;
  }
  s->arena.free.push_back({0, s->arena.size});
  *out = s;
  return HIGS_OK;
}

int higs_server_destroy(higs_server* s) {
  if (!s) return HIGS_E_INVALID;
  Guard g(s->device);
  for (Slot* sl : s->slots) {
    if (sl->sh.stream) (void)hipStreamSynchronize(sl->sh.stream);
    if (sl->ctx) (void)ctx_release(sl->ctx);
    free_shell(sl->sh);
    delete sl;
  }
  for (Shell& sh : s->shells) free_shell(sh);
  for (Request& r : s->queue)
    if (r.dep) s->events.push_back(r.dep);
  for (Scene& sc : s->scenes)
    if (sc.ready) s->events.push_back(sc.ready);
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  if (s->arena.base) (void)hipFree(s->arena.base);
  delete s;
  return HIGS_OK;
}

int higs_server_add_scene(higs_server* s, int32_t scene_id, int64_t n, const float* means,
                          const float* scales, const float* quats, const float* opacities,
                          const float* sh, void* stream) {
  if (!s || n < 0 || n > s->cfg.max_gaussians) return HIGS_E_INVALID;
  if (n > 0 && (!means || !scales || !quats || !opacities || !sh)) return HIGS_E_INVALID;
  if (find_scene(s, scene_id)) return HIGS_E_INVALID;
  Guard g(s->device);
  Scene sc;
  sc.id = scene_id;
  sc.n = n;
  sc.means = means;
  sc.scales = scales;
  sc.quats = quats;
  sc.opac = opacities;
  sc.sh = sh;
  const int rc = record_dep(s, stream, &sc.ready);
  if (rc) return rc;
  s->scenes.push_back(sc);
  return HIGS_OK;
}

int higs_server_submit(higs_server* s, int64_t request_id, int32_t scene_id, int32_t cls,
                       const higs_camera* cam, float* image, void* stream) {
  if (!s || !cam || !image || cls < 0 || cls >= s->cfg.n_classes) return HIGS_E_INVALID;
  if (!find_scene(s, scene_id)) return HIGS_E_INVALID;
  if (cam->width < 1 || cam->height < 1 || cam->width > s->cfg.width[cls] ||
      cam->height > s->cfg.height[cls])
    return HIGS_E_CAPACITY;
  if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f)) return HIGS_E_INVALID;
  Guard g(s->device);
  hipEvent_t dep = nullptr;
  const int rc = record_dep(s, stream, &dep);
  if (rc) return rc;
  s->queue.push_back(Request{request_id, scene_id, cls, *cam, image, dep});
  return HIGS_OK;
}

int higs_server_poll(higs_server* s, higs_completion* done, int32_t max_done) {
  if (!s || (max_done > 0 && !done) || max_done < 0) return HIGS_E_INVALID;
  Guard g(s->device);
  int rc = retire(s);
  if (!rc) rc = admit(s);
  if (rc && !s->error) s->error = rc;
  // completions first; an error is returned once nothing retired is left
  int32_t n = 0;
  while (n < max_done && !s->done.empty()) {
    const Done& d = s->done.front();
    done[n].request_id = d.request;
    done[n].gpu_ms = d.ms;
    done[n].overflow = d.overflow;
    done[n].cls = d.cls;
    done[n].views = d.views;
    ++n;
    s->done.pop_front();
  }
  if (n > 0) return n;
  if (s->error) {
    const int e = s->error;
    s->error = 0;
    return e;
  }
  return 0;
}

int higs_server_get_stats(higs_server* s, higs_server_stats* out) {
  if (!s || !out) return HIGS_E_INVALID;
  out->queued = (int32_t)s->queue.size();
  out->in_flight = s->in_flight;
  out->contexts = (int32_t)s->slots.size();
  int64_t bytes = 0;
  for (const Slot* sl : s->slots) bytes += (int64_t)Arena::round(sl->bytes);
  out->bytes = bytes;
  out->completed = s->completed;
  out->evictions = s->evictions;
  out->frames = s->frames;
  for (int c = 0; c < HIGS_MAX_CLASSES; ++c) {
    out->views_per_frame[c] = c < s->cfg.n_classes ? s->views[c] : 0;
    out->batch_cap[c] = c < s->cfg.n_classes ? s->batch_cap[c] : 0;
  }
  return HIGS_OK;
}

int higs_server_tune(higs_server* s, int32_t cls, int32_t scene_id, int32_t n_cams,
                     const higs_camera* cams, int32_t frames, int32_t allow_batch_cap,
                     higs_tune_report* out) {
  if (!s || !cams || !out || n_cams < 1 || frames < 1 || cls < 0 || cls >= s->cfg.n_classes)
    return HIGS_E_INVALID;
  const Scene* sc = find_scene(s, scene_id);
  if (!sc) return HIGS_E_INVALID;
  for (int k = 0; k < n_cams; ++k)
    if (cams[k].width != s->cfg.width[cls] || cams[k].height != s->cfg.height[cls])
      return HIGS_E_INVALID;
  if (s->in_flight != 0 || !s->queue.empty()) return HIGS_E_STATE;
  Guard g(s->device);
  // the trials take the whole arena: every idle context goes
  for (Slot* sl : s->slots) release_slot(s, sl);
  s->slots.clear();
  *out = higs_tune_report{};
  static const int kViews[] = {1, 2, 4, 8, 16};
  static const int kCaps[] = {1024, 512, 256};
  double fps_of[HIGS_TUNE_MAX_TRIALS];
  for (int ci = 0; ci < (allow_batch_cap ? 3 : 1); ++ci) {
    const int cap = allow_batch_cap ? kCaps[ci] : s->params.batch_cap;
    for (int v : kViews) {
      if (out->n_trials >= HIGS_TUNE_MAX_TRIALS) break;
      int rc = HIGS_OK;
      const double fps = trial(s, cls, *sc, n_cams, cams, v, cap, frames, &rc);
      if (rc) return rc;
      if (fps <= 0.0) continue;  // the context does not fit the arena
      const int t = out->n_trials++;
      out->trial_views[t] = v;
      out->trial_batch_cap[t] = cap;
      out->trial_fps[t] = (float)fps;
      fps_of[t] = fps;
    }
  }
  if (out->n_trials == 0) return HIGS_E_CAPACITY;  // no candidate fits the arena
  // the fewest views per frame (then the largest B_r) within 3% of the
  // fastest trial: grouping adds latency, and closer figures are noise
  double top = 0.0;
  for (int t = 0; t < out->n_trials; ++t) top = std::max(top, fps_of[t]);
  int best_v = 0, best_c = 0;
  for (int t = 0; t < out->n_trials; ++t) {
    if (fps_of[t] < 0.97 * top) continue;
    const int v = out->trial_views[t], c = out->trial_batch_cap[t];
    if (!best_v || v < best_v || (v == best_v && c > best_c)) {
      best_v = v;
      best_c = c;
    }
  }
  s->views[cls] = best_v;
  s->batch_cap[cls] = best_c;
  out->views_per_frame = best_v;
  out->batch_cap = best_c;
  return HIGS_OK;
}

int higs_server_set_class(higs_server* s, int32_t cls, int32_t views_per_frame, int32_t batch_cap) {
  if (!s || cls < 0 || cls >= s->cfg.n_classes || views_per_frame < 1 ||
      views_per_frame > HIGS_MAX_VIEWS || batch_cap < 1 || batch_cap > kMaxBatch)
    return HIGS_E_INVALID;
  if (slot_bytes(s, cls, views_per_frame, batch_cap) < 0) return HIGS_E_INVALID;
  s->views[cls] = views_per_frame;
  s->batch_cap[cls] = batch_cap;
  return HIGS_OK;
}

}  // extern "C"
