// CPU stand-in for the parts of the HIP runtime and device language that
// libhigs uses, for a host-only test build of the library's own sources
// (bounds checking under AddressSanitizer, termination of every kernel, and
// the kernels' results on small frames).  Test infrastructure only: the
// product library is built for gfx950 by hipcc and never sees this header.
//
// Execution model: a kernel launch runs its workgroups one after another on
// the calling thread's behalf; the threads of a workgroup are OS threads
// (one per work-item) that meet at a workgroup barrier, and the 64 lanes of a
// wave meet at a wave barrier inside every cross-lane operation (ballot,
// shuffles, readfirstlane).  A work-item that returns drops out of both
// barriers, as an exited wave does on the GPU.  __shared__ variables are
// function statics, so one copy serves the workgroup that is running.
// Device memory is host memory from aligned_alloc (AddressSanitizer watches
// every access).  Streams and events are synchronous.
#pragma once

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <sys/mman.h>
#include <sys/wait.h>
#include <unistd.h>

#include <atomic>
#include <map>
#include <barrier>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __shared__ static
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
#define amdgpu_waves_per_eu(...) unused
#define HIP_DYNAMIC_SHARED(type, name) type* name = reinterpret_cast<type*>(cpuhip::g_dyn_lds);
#define __align__(n) __attribute__((aligned(n)))
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __HIP_MEMORY_SCOPE_WORKGROUP 0
#define __HIP_MEMORY_SCOPE_SYSTEM 0

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint3_ {
  unsigned x, y, z;
};
struct float2 {
  float x, y;
};
struct float3 {
  float x, y, z;
};
inline float3 make_float3(float a, float b, float c) { return float3{a, b, c}; }
struct __attribute__((aligned(16))) float4 {
  float x, y, z, w;
};
struct __attribute__((aligned(8))) uint2 {
  unsigned x, y;
};
struct __attribute__((aligned(16))) uint4 {
  unsigned x, y, z, w;
};
inline float2 make_float2(float a, float b) { return float2{a, b}; }
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return uint4{a, b, c, d}; }
inline float4 make_float4(float a, float b, float c, float d) { return float4{a, b, c, d}; }

namespace cpuhip {

constexpr int kWave = 64;

struct Wave {
  std::barrier<>* bar = nullptr;
  uint64_t slot[kWave];
  std::atomic<int> present[kWave];
};

struct Block {
  std::barrier<>* bar = nullptr;
  std::vector<Wave*> waves;
  std::atomic<uint32_t> or_acc[2];
};

inline thread_local uint3_ tl_thread{0, 0, 0};
inline thread_local uint3_ tl_block{0, 0, 0};
inline thread_local Block* tl_blk = nullptr;
inline thread_local int tl_phase = 0;
inline dim3 g_block_dim, g_grid_dim;
inline unsigned char* g_dyn_lds = nullptr;

inline int lane_id() {
  const int t = (int)(tl_thread.x + g_block_dim.x * (tl_thread.y + g_block_dim.y * tl_thread.z));
  return t % kWave;
}
inline int wave_id() {
  const int t = (int)(tl_thread.x + g_block_dim.x * (tl_thread.y + g_block_dim.y * tl_thread.z));
  return t / kWave;
}

// All present lanes' 64-bit values; `mask` gets the present lanes.
inline void reset_spin();
inline void wave_exchange(uint64_t v, uint64_t out[kWave], uint64_t* mask) {
  reset_spin();
  Wave& w = *tl_blk->waves[wave_id()];
  const int l = lane_id();
  w.slot[l] = v;
  w.present[l].store(1);
  w.bar->arrive_and_wait();
  uint64_t m = 0;
  for (int k = 0; k < kWave; ++k)
    if (w.present[k].load()) {
      m |= 1ull << k;
      out[k] = w.slot[k];
    } else {
      out[k] = 0;
    }
  w.bar->arrive_and_wait();
  w.present[l].store(0);
  *mask = m;
}

template <class T>
inline uint64_t to_bits(T v) {
  uint64_t b = 0;
  static_assert(sizeof(T) <= 8, "wave exchange of at most 8 bytes");
  memcpy(&b, &v, sizeof(T));
  return b;
}
template <class T>
inline T from_bits(uint64_t b) {
  T v;
  memcpy(&v, &b, sizeof(T));
  return v;
}

// A pool of work-item threads, reused by every workgroup of every launch
// (thread creation under AddressSanitizer dominates otherwise).
class Pool {
 public:
  void run(unsigned nt, const std::function<void(unsigned)>& job) {
    std::unique_lock<std::mutex> lk(mu_);
    while (workers_.size() < nt) {
      const unsigned idx = (unsigned)workers_.size();
      workers_.emplace_back([this, idx]() { loop(idx); });
    }
    job_ = &job;
    nt_ = nt;
    left_ = nt;
    ++gen_;
    cv_.notify_all();
    done_.wait(lk, [this]() { return left_ == 0; });
    job_ = nullptr;
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }

 private:
  void loop(unsigned idx) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(unsigned)>* job;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&]() { return gen_ != seen; });
        seen = gen_;
        if (stop_) return;
        if (idx >= nt_) continue;
        job = job_;
      }
      (*job)(idx);
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (--left_ == 0) done_.notify_one();
      }
    }
  }
  std::mutex mu_;
  std::condition_variable cv_, done_;
  std::vector<std::thread> workers_;
  const std::function<void(unsigned)>* job_ = nullptr;
  unsigned nt_ = 0, left_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};
inline Pool*& pool_ptr() {
  static Pool* p = new Pool();
  return p;
}
inline Pool& pool() { return *pool_ptr(); }

// CPUHIP_PROCS = k > 1: the workgroups of a launch run in k forked processes
// at once (workgroup w in process w mod k), so that workgroups of a
// persistent kernel really interleave; device memory is then a shared mapping
// (no AddressSanitizer redzones), and every process has its own LDS.
inline int procs() {
  static int k = getenv("CPUHIP_PROCS") ? atoi(getenv("CPUHIP_PROCS")) : 1;
  return k;
}

template <class... A, class... P>
void launch(void (*k)(P...), dim3 grid, dim3 block, size_t shmem, A... args) {
  const unsigned nt = block.x * block.y * block.z;
  std::vector<unsigned char> dyn(shmem + 16);
  g_dyn_lds = dyn.data();
  g_block_dim = block;
  g_grid_dim = grid;
  const unsigned nw = (nt + kWave - 1) / kWave;
  const unsigned n_blocks = grid.x * grid.y * grid.z;
  const int np = procs() > 1 && n_blocks > 1 ? procs() : 1;
  std::vector<pid_t> kids;
  int me = 0;
  if (np > 1) {
    fflush(stdout);
    fflush(stderr);
    for (int c = 1; c < np; ++c) {
      const pid_t pid = fork();
      if (pid == 0) {
        me = c;
        pool_ptr() = new Pool();  // the parent's worker threads do not exist here
        kids.clear();
        break;
      }
      kids.push_back(pid);
    }
  }
  unsigned flat = 0;
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx, ++flat) {
        if ((int)(flat % (unsigned)np) != me) continue;
        Block B;
        std::barrier<> bbar((ptrdiff_t)nt);
        B.bar = &bbar;
        B.or_acc[0] = 0;
        B.or_acc[1] = 0;
        std::vector<std::barrier<>*> wbars;
        for (unsigned w = 0; w < nw; ++w) {
          const unsigned cnt = (w + 1) * kWave <= nt ? kWave : nt - w * kWave;
          wbars.push_back(new std::barrier<>((ptrdiff_t)cnt));
          Wave* wv = new Wave();
          wv->bar = wbars.back();
          for (int l = 0; l < kWave; ++l) wv->present[l] = 0;
          B.waves.push_back(wv);
        }
        const std::function<void(unsigned)> job = [&](unsigned t) {
          tl_thread = uint3_{t % block.x, (t / block.x) % block.y, t / (block.x * block.y)};
          tl_block = uint3_{bx, by, bz};
          tl_blk = &B;
          tl_phase = 0;
          k(args...);
          B.waves[t / kWave]->bar->arrive_and_drop();
          B.bar->arrive_and_drop();
        };
        pool().run(nt, job);
        for (Wave* w : B.waves) delete w;
        for (auto* b : wbars) delete b;
      }
  if (np > 1) {
    if (me != 0) _exit(0);
    for (pid_t pid : kids) {
      int st = 0;
      waitpid(pid, &st, 0);
      if (!WIFEXITED(st) || WEXITSTATUS(st) != 0) {
        fprintf(stderr, "cpuhip: a workgroup process failed\n");
        abort();
      }
    }
  }
}

}  // namespace cpuhip

#define threadIdx (cpuhip::tl_thread)
#define blockIdx (cpuhip::tl_block)
#define blockDim (cpuhip::g_block_dim)
#define gridDim (cpuhip::g_grid_dim)

inline void __syncthreads() {
  cpuhip::reset_spin();
  cpuhip::tl_blk->bar->arrive_and_wait();
}
inline int __syncthreads_or(int p) {
  cpuhip::Block& b = *cpuhip::tl_blk;
  const int ph = cpuhip::tl_phase;
  if (p) b.or_acc[ph].fetch_or(1u);
  b.bar->arrive_and_wait();
  const int r = b.or_acc[ph].load() != 0;
  if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) b.or_acc[ph ^ 1].store(0);
  b.bar->arrive_and_wait();
  cpuhip::tl_phase ^= 1;
  return r;
}
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __threadfence_block() { std::atomic_thread_fence(std::memory_order_seq_cst); }

inline uint64_t __ballot(int p) {
  uint64_t v[64], m;
  cpuhip::wave_exchange(p ? 1ull : 0ull, v, &m);
  uint64_t r = 0;
  for (int k = 0; k < 64; ++k)
    if (((m >> k) & 1ull) && v[k]) r |= 1ull << k;
  return r;
}
inline int __any(int p) { return __ballot(p) != 0; }
inline int __all(int p) {
  uint64_t v[64], m;
  cpuhip::wave_exchange(p ? 1ull : 0ull, v, &m);
  for (int k = 0; k < 64; ++k)
    if (((m >> k) & 1ull) && !v[k]) return 0;
  return 1;
}
template <class T>
inline T __shfl(T x, int src, int width = 64) {
  uint64_t v[64], m;
  cpuhip::wave_exchange(cpuhip::to_bits(x), v, &m);
  const int l = cpuhip::lane_id();
  const int s = (l / width) * width + (((src % width) + width) % width);
  return ((m >> s) & 1ull) ? cpuhip::from_bits<T>(v[s]) : x;
}
template <class T>
inline T __shfl_up(T x, unsigned d, int width = 64) {
  uint64_t v[64], m;
  cpuhip::wave_exchange(cpuhip::to_bits(x), v, &m);
  const int l = cpuhip::lane_id();
  const int s = l - (int)d;
  if (s < (l / width) * width) return x;
  return ((m >> s) & 1ull) ? cpuhip::from_bits<T>(v[s]) : x;
}
template <class T>
inline T __shfl_down(T x, unsigned d, int width = 64) {
  uint64_t v[64], m;
  cpuhip::wave_exchange(cpuhip::to_bits(x), v, &m);
  const int l = cpuhip::lane_id();
  const int s = l + (int)d;
  if (s >= (l / width + 1) * width) return x;
  return ((m >> s) & 1ull) ? cpuhip::from_bits<T>(v[s]) : x;
}
template <class T>
inline T __shfl_xor(T x, int mask, int width = 64) {
  uint64_t v[64], m;
  cpuhip::wave_exchange(cpuhip::to_bits(x), v, &m);
  const int l = cpuhip::lane_id();
  const int s = l ^ mask;
  if (s / width != l / width) return x;
  return ((m >> s) & 1ull) ? cpuhip::from_bits<T>(v[s]) : x;
}
template <class T>
inline T __builtin_amdgcn_readfirstlane(T x) {
  uint64_t v[64], m;
  cpuhip::wave_exchange(cpuhip::to_bits(x), v, &m);
  return cpuhip::from_bits<T>(v[__builtin_ctzll(m)]);
}

template <class T>
inline T min(T a, T b) {
  return b < a ? b : a;
}
template <class T>
inline T max(T a, T b) {
  return a < b ? b : a;
}
inline unsigned __float_as_uint(float f) {
  unsigned u;
  memcpy(&u, &f, 4);
  return u;
}
inline float __uint_as_float(unsigned u) {
  float f;
  memcpy(&f, &u, 4);
  return f;
}
inline int __float_as_int(float f) { return (int)__float_as_uint(f); }
inline float __int_as_float(int i) { return __uint_as_float((unsigned)i); }
// The lanes of a wave execute in lockstep on the GPU; here the wave's threads
// meet at the wave barrier instead.
inline void __builtin_amdgcn_wave_barrier() {
  cpuhip::tl_blk->waves[cpuhip::wave_id()]->bar->arrive_and_wait();
}
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __popc(unsigned v) { return __builtin_popcount(v); }
inline int __ffsll(unsigned long long v) { return __builtin_ffsll((long long)v); }
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
inline int __clz(int v) { return v ? __builtin_clz((unsigned)v) : 32; }
inline int __clzll(long long v) { return v ? __builtin_clzll((unsigned long long)v) : 64; }

inline float __builtin_amdgcn_sqrtf(float x) { return sqrtf(x); }
inline float __builtin_amdgcn_rcpf(float x) { return 1.0f / x; }
inline float __builtin_amdgcn_rsqf(float x) { return 1.0f / sqrtf(x); }
inline float __builtin_amdgcn_logf(float x) { return log2f(x); }
inline float __builtin_amdgcn_exp2f(float x) { return exp2f(x); }
inline unsigned __builtin_amdgcn_alignbit(unsigned hi, unsigned lo, unsigned s) {
  s &= 31u;
  const uint64_t v = ((uint64_t)hi << 32) | lo;
  return (unsigned)(v >> s);
}

// atomics (device scope = process scope here)
template <class T>
inline T atomicAdd(T* p, T v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline unsigned atomicAdd(unsigned* p, int v) { return __atomic_fetch_add(p, (unsigned)v, __ATOMIC_SEQ_CST); }
inline float atomicAdd(float* p, float v) {
  uint32_t* q = reinterpret_cast<uint32_t*>(p);
  uint32_t old = __atomic_load_n(q, __ATOMIC_SEQ_CST);
  for (;;) {
    float f;
    memcpy(&f, &old, 4);
    f += v;
    uint32_t nw;
    memcpy(&nw, &f, 4);
    if (__atomic_compare_exchange_n(q, &old, nw, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
      memcpy(&f, &old, 4);
      return f;
    }
  }
}
template <class T>
inline T atomicOr(T* p, T v) {
  return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST);
}
template <class T>
inline T atomicAnd(T* p, T v) {
  return __atomic_fetch_and(p, v, __ATOMIC_SEQ_CST);
}
template <class T>
inline T atomicMax(T* p, T v) {
  T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (old < v && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return old;
}
template <class T>
inline T atomicMin(T* p, T v) {
  T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (old > v && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return old;
}
template <class T>
inline T atomicExch(T* p, T v) {
  return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST);
}
template <class T>
inline T atomicCAS(T* p, T cmp, T v) {
  __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return cmp;
}
namespace cpuhip {
// A work-item that keeps loading the same word is waiting for another
// workgroup: after a while it sleeps between loads, so that the GPU code's
// spin bounds (sized for GPU speed) stay long enough at emulation speed.
// (atomic loads since the work-item last met its wave or workgroup)
inline thread_local unsigned tl_spin_count = 0;
template <class T>
inline T spin_load(const T* p) {
  if (++tl_spin_count > 4096) usleep(20);
  return __atomic_load_n(p, __ATOMIC_SEQ_CST);
}
}  // namespace cpuhip
namespace cpuhip {
inline void reset_spin() { tl_spin_count = 0; }
}  // namespace cpuhip
#define __hip_atomic_load(p, order, scope) cpuhip::spin_load(p)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), __ATOMIC_SEQ_CST)
#define __hip_atomic_fetch_add(p, v, order, scope) __atomic_fetch_add((p), (v), __ATOMIC_SEQ_CST)
#define __hip_atomic_fetch_or(p, v, order, scope) __atomic_fetch_or((p), (v), __ATOMIC_SEQ_CST)

// ---- runtime ---------------------------------------------------------------
typedef int hipError_t;
enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotReady = 600,
};
typedef struct cpuhip_stream* hipStream_t;
typedef struct cpuhip_event {
  double t;
}* hipEvent_t;
enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
};
#define hipStreamNonBlocking 1
#define hipStreamDefault 0
#define hipHostMallocDefault 0
#define hipEventDisableTiming 2
struct hipDeviceProp_t {
  char name[256];
  int multiProcessorCount;
  size_t totalGlobalMem;
};
#define HIP_SYMBOL(x) (&(x))

namespace cpuhip {
// compute units the CPU "device" reports (persistent kernels launch a grid
// sized by it): CPUHIP_CUS, default 2
inline int g_cus = getenv("CPUHIP_CUS") ? atoi(getenv("CPUHIP_CUS")) : 2;
inline double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace cpuhip

namespace cpuhip {
inline std::map<void*, size_t>& shared_maps() {
  static std::map<void*, size_t> m;
  return m;
}
}  // namespace cpuhip
inline hipError_t hipMalloc(void** p, size_t n) {
  const size_t bytes = (n + 255) / 256 * 256;
  if (cpuhip::procs() > 1) {  // visible to the workgroup processes
    void* q = mmap(nullptr, bytes ? bytes : 256, PROT_READ | PROT_WRITE, MAP_SHARED | MAP_ANONYMOUS,
                   -1, 0);
    if (q == MAP_FAILED) return hipErrorOutOfMemory;
    cpuhip::shared_maps()[q] = bytes ? bytes : 256;
    *p = q;
    return hipSuccess;
  }
  *p = aligned_alloc(256, bytes);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void* p) {
  auto it = cpuhip::shared_maps().find(p);
  if (it != cpuhip::shared_maps().end()) {
    munmap(p, it->second);
    cpuhip::shared_maps().erase(it);
    return hipSuccess;
  }
  free(p);
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
inline hipError_t hipHostFree(void* p) { return hipFree(p); }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  if (n) memcpy(d, s, n);
  return hipSuccess;
}
// Graph capture: work enqueued on a capturing stream is recorded (arguments
// by value, copies read their source at replay) and runs at hipGraphLaunch.
struct cpuhip_graph {
  std::vector<std::function<void()>> ops;
};
typedef cpuhip_graph* hipGraph_t;
typedef struct cpuhip_graph_exec {
  std::vector<std::function<void()>> ops;
}* hipGraphExec_t;
typedef void* hipGraphNode_t;
enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
};
namespace cpuhip {
inline std::map<const void*, cpuhip_graph*>& captures() {
  static std::map<const void*, cpuhip_graph*> m;
  return m;
}
inline cpuhip_graph* capturing(const void* s) {
  auto it = captures().find(s);
  return it == captures().end() ? nullptr : it->second;
}
}  // namespace cpuhip
inline hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s || cpuhip::capturing(s)) return hipErrorInvalidValue;
  cpuhip::captures()[s] = new cpuhip_graph();
  return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  cpuhip_graph* c = cpuhip::capturing(s);
  if (!c) return hipErrorInvalidValue;
  cpuhip::captures().erase(s);
  *g = c;
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *e = new cpuhip_graph_exec{g->ops};
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto& op : e->ops) op();
  return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st = nullptr) {
  if (cpuhip_graph* g = cpuhip::capturing(st)) {
    g->ops.push_back([=] { hipMemcpy(d, s, n, k); });
    return hipSuccess;
  }
  return hipMemcpy(d, s, n, k);
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st = nullptr) {
  if (cpuhip::capturing(st)) {  // a memset node in a graph: never recorded by the library
    fprintf(stderr, "cpuhip: hipMemsetAsync on a capturing stream\n");
    abort();
  }
  if (n) memset(d, v, n);
  return hipSuccess;
}
inline hipError_t hipMemset(void* d, int v, size_t n) { return hipMemsetAsync(d, v, n); }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = reinterpret_cast<hipStream_t>(new char[1]);
  return hipSuccess;
}
inline hipError_t hipStreamCreate(hipStream_t* s) { return hipStreamCreateWithFlags(s, 0); }
inline hipError_t hipStreamDestroy(hipStream_t s) {
  delete[] reinterpret_cast<char*>(s);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new cpuhip_event{0.0};
  return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t st = nullptr) {
  if (cpuhip::capturing(st)) {  // the library records no events inside a graph
    fprintf(stderr, "cpuhip: hipEventRecord on a capturing stream\n");
    abort();
  }
  e->t = cpuhip::now_ms();
  return hipSuccess;
}
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)(b->t - a->t);
  return hipSuccess;
}
inline hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  memset(p, 0, sizeof(*p));
  strcpy(p->name, "cpu");
  p->multiProcessorCount = cpuhip::g_cus;
  p->totalGlobalMem = (size_t)1 << 34;
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipPeekAtLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "cpu emulation error"; }
template <class K>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, K, int, size_t) {
  *n = 1;
  return hipSuccess;
}
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}

namespace cpuhip {
template <class... A, class... P>
void launch_on(const void* stream, void (*k)(P...), dim3 grid, dim3 block, size_t shmem, A... args) {
  if (cpuhip_graph* g = capturing(stream)) {
    g->ops.push_back([=] { launch(k, grid, block, shmem, args...); });
    return;
  }
  launch(k, grid, block, shmem, args...);
}
}  // namespace cpuhip
#define hipLaunchKernelGGL(k, grid, block, shmem, stream, ...) \
  cpuhip::launch_on((const void*)(stream), (k), dim3(grid), dim3(block), (size_t)(shmem), ##__VA_ARGS__)
