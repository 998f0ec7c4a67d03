// Test driver for the CPU build of libhigs (see hip/hip_runtime.h): renders
// the frames described in <in>/job.txt through the library's C-ABI and writes
// what the tests compare (counts, image, transmittance, sorted pairs, batch
// table) into <out>.
//
// job.txt: one frame per line after a header line "n max_pairs max_batches
// sort_mode batch_cap n_cus entry precision sh_format chain fuse" (entry 0 = the stages one
// by one on a context, 1 = the allocation-free entry point, 2 = every frame as
// a view of one higs_render_views frame, 3 = higs_render with graph replay,
// 4 = as 2 with graph replay, the frame recorded by a first call with the
// cameras rotated and replayed for the outputs, 5 = every frame a request to
// a render server whose frames hold all of them, with graph replay, served
// twice: the second round's images must equal the first's); a frame line is "n_use W H fx fy cx cy
// R00 .. t2 (12 floats) bg0 bg1 bg2".  Scene arrays are raw float32 files
// means, scales, quats, opac, sh in <in>.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <sys/mman.h>

#include <string>
#include <vector>

#include "../../include/higs.h"

static std::vector<float> load(const std::string& path, size_t count) {
  std::vector<float> v(count);
  FILE* f = fopen(path.c_str(), "rb");
  if (!f || fread(v.data(), 4, count, f) != count) {
    fprintf(stderr, "cannot read %s\n", path.c_str());
    exit(2);
  }
  fclose(f);
  return v;
}

static void save(const std::string& path, const void* p, size_t bytes) {
  FILE* f = fopen(path.c_str(), "wb");
  if (!f || (bytes && fwrite(p, 1, bytes, f) != bytes)) {
    fprintf(stderr, "cannot write %s\n", path.c_str());
    exit(2);
  }
  fclose(f);
}

extern "C" int higs_render_noalloc(int64_t n, const float* means, const float* scales,
                                   const float* quats, const float* opacities, const float* sh,
                                   const higs_camera* cam, float* image, float* T_out,
                                   void* stream) __attribute__((weak));

// Entry 5: the frames as requests to a render server (one class of the
// largest camera size, all requests in one frame, graph replay), in two
// rounds; writes the first round's images and T = -1 (the server writes no T).
static int serve_job(const higs_params& p, long long n, long long max_pairs, int max_w, int max_h,
                     const std::vector<higs_camera>& cams, const std::vector<long long>& uses,
                     const std::vector<float>& means, const std::vector<float>& scales,
                     const std::vector<float>& quats, const std::vector<float>& opac,
                     const float* sh_in, const std::string& out) {
  const int V = (int)cams.size();
  higs_server_config cfg{};
  cfg.n_classes = 1;
  cfg.width[0] = max_w;
  cfg.height[0] = max_h;
  cfg.max_pairs[0] = max_pairs;
  cfg.max_gaussians = n;
  cfg.max_in_flight = 2;
  cfg.views_per_frame[0] = V;
  cfg.use_graphs = 1;
  higs_params q = p;
  q.max_views = V;
  const int64_t n_mt = (int64_t)((max_w + 63) / 64) * ((max_h + 31) / 32);
  const int64_t fp = higs_ctx_footprint(&q, n, max_pairs * V, max_pairs * V / p.batch_cap + n_mt * V + 16,
                                        max_w, max_h);
  if (fp <= 0) return 3;
  cfg.hbm_budget = 2 * (fp + ((int64_t)8 << 20));
  higs_server* srv = nullptr;
  int rc = higs_server_create(0, &p, &cfg, &srv);
  if (rc) {
    fprintf(stderr, "higs_server_create: %d\n", rc);
    return 3;
  }
  for (int f = 0; f < V; ++f) {
    rc = higs_server_add_scene(srv, f, uses[f], means.data(), scales.data(), quats.data(),
                               opac.data(), sh_in, nullptr);
    if (rc) return 3;
  }
  std::vector<std::vector<float>> img[2];
  for (int round = 0; round < 2; ++round) {
    img[round].resize(V);
    for (int f = 0; f < V; ++f) {
      img[round][f].assign((size_t)cams[f].width * cams[f].height * 3, -7.0f);
      rc = higs_server_submit(srv, round * V + f, f, 0, &cams[f], img[round][f].data(), nullptr);
      if (rc) return 3;
    }
    int got = 0;
    higs_completion done[8];
    for (int it = 0; it < 1000 && got < V; ++it) {
      const int k = higs_server_poll(srv, done, 8);
      if (k < 0) return 5;
      for (int j = 0; j < k; ++j)
        if (done[j].overflow || done[j].views != V) return 5;
      got += k;
    }
    if (got != V) return 5;
  }
  higs_server_stats st{};
  if (higs_server_get_stats(srv, &st) || st.frames != 2 || st.completed != 2 * V) return 6;
  for (int f = 0; f < V; ++f)
    if (memcmp(img[0][f].data(), img[1][f].data(), img[0][f].size() * 4)) return 6;
  FILE* summary = fopen((out + "/counts.txt").c_str(), "w");
  for (int f = 0; f < V; ++f) {
    const size_t npx = (size_t)cams[f].width * cams[f].height;
    const std::string pre = out + "/f" + std::to_string(f) + "_";
    save(pre + "image", img[0][f].data(), npx * 12);
    std::vector<float> T(npx, -1.0f);
    save(pre + "T", T.data(), npx * 4);
    fprintf(summary, "0 0 0 0 -1 0 0\n");
  }
  fclose(summary);
  return higs_server_destroy(srv) ? 7 : 0;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: frame_driver <in> <out>\n");
    return 2;
  }
  const std::string in = argv[1], out = argv[2];
  FILE* jf = fopen((in + "/job.txt").c_str(), "r");
  if (!jf) return 2;
  long long n, max_pairs, max_batches;
  int sort_mode, batch_cap, n_cus, entry;
  int precision = 0, sh_format = 0;
  int chain = 64, fuse = 1;
  if (fscanf(jf, "%lld %lld %lld %d %d %d %d %d %d %d %d", &n, &max_pairs, &max_batches, &sort_mode,
             &batch_cap, &n_cus, &entry, &precision, &sh_format, &chain, &fuse) != 11)
    return 2;
  std::vector<float> means = load(in + "/means", (size_t)n * 3);
  std::vector<float> scales = load(in + "/scales", (size_t)n * 3);
  std::vector<float> quats = load(in + "/quats", (size_t)n * 4);
  std::vector<float> opac = load(in + "/opac", (size_t)n);
  std::vector<float> sh = load(in + "/sh", (size_t)n * 48);
  higs_params p;
  higs_default_params(&p);
  p.sort_mode = sort_mode;
  p.batch_cap = batch_cap;
  p.raster_precision = precision;
  p.sh_format = sh_format;
  p.raster_chain = chain;
  p.fuse_merge = fuse;
  // packed SH: compressed once by the library, written out for the tests
  std::vector<unsigned char> packed;
  if (sh_format == HIGS_SH_PACKED32) {
    packed.resize((size_t)higs_sh_packed_bytes(n));
    if (higs_sh_compress(n, sh.data(), opac.data(), packed.data(), nullptr)) return 3;
    save(out + "/packed", packed.data(), packed.size());
  }
  const float* sh_in = sh_format == HIGS_SH_PACKED32
                           ? reinterpret_cast<const float*>(packed.data())
                           : sh.data();
  higs_ctx* ctx = nullptr;
  int max_w = 1, max_h = 1;
  std::vector<higs_camera> cams;
  std::vector<long long> uses;
  for (;;) {
    higs_camera c;
    long long use;
    if (fscanf(jf, "%lld %d %d %f %f %f %f", &use, &c.width, &c.height, &c.fx, &c.fy, &c.cx,
               &c.cy) != 7)
      break;
    for (int k = 0; k < 12; ++k)
      if (fscanf(jf, "%f", &c.world_to_cam[k]) != 1) return 2;
    for (int k = 0; k < 3; ++k)
      if (fscanf(jf, "%f", &c.background[k]) != 1) return 2;
    cams.push_back(c);
    uses.push_back(use);
    if (c.width > max_w) max_w = c.width;
    if (c.height > max_h) max_h = c.height;
  }
  fclose(jf);
  const int debug_flags = getenv("HIGS_CPU_DEBUG") ? atoi(getenv("HIGS_CPU_DEBUG")) : 0;
  if (entry == 5) return serve_job(p, n, max_pairs, max_w, max_h, cams, uses, means, scales, quats,
                                   opac, sh_in, out);
  if (entry == 2 || entry == 4) p.max_views = (int)cams.size();
  if (entry == 3 || entry == 4) p.use_graphs = 1;
  // graph replay needs a stream other than the legacy default one (the CPU
  // runtime never dereferences a stream handle)
  static int stream_tag = 0;
  void* stream = (entry == 3 || entry == 4) ? static_cast<void*>(&stream_tag) : nullptr;
  if (entry != 1) {
    const int rc = higs_ctx_create(0, &p, n, max_pairs, max_batches, max_w, max_h, &ctx);
    if (rc) {
      fprintf(stderr, "higs_ctx_create: %d\n", rc);
      return 3;
    }
    if (debug_flags && higs_set_debug(ctx, debug_flags)) return 3;
  }
  FILE* summary = fopen((out + "/counts.txt").c_str(), "w");
  if (entry == 2 || entry == 4) {  // every frame of the job as one view of a single frame
    std::vector<higs_view> vs(cams.size());
    std::vector<float*> bufs;
    for (size_t f = 0; f < cams.size(); ++f) {
      const size_t npx = (size_t)cams[f].width * cams[f].height;
      float* b = static_cast<float*>(mmap(nullptr, npx * 16, PROT_READ | PROT_WRITE,
                                         MAP_SHARED | MAP_ANONYMOUS, -1, 0));
      if (b == MAP_FAILED) return 2;
      for (size_t q = 0; q < npx * 4; ++q) b[q] = -7.0f;
      bufs.push_back(b);
      higs_view& v = vs[f];
      v.n = uses[f];
      v.means = means.data();
      v.scales = scales.data();
      v.quats = quats.data();
      v.opacities = opac.data();
      v.sh = sh_in;
      v.camera = cams[f];
      v.image = b;
      v.T_out = b + npx * 3;
    }
    int rc = 0;
    if (entry == 4 && vs.size() > 1) {
      // first frame: the same shape with the cameras rotated, into other
      // buffers (recorded and replayed); the second replays the graph
      std::vector<higs_view> rot(vs);
      std::vector<std::vector<float>> junk(vs.size());
      for (size_t f = 0; f < vs.size(); ++f) {
        rot[f].camera = vs[(f + 1) % vs.size()].camera;
        junk[f].resize((size_t)rot[f].camera.width * rot[f].camera.height * 4);
        rot[f].image = junk[f].data();
        rot[f].T_out = junk[f].data() + (size_t)rot[f].camera.width * rot[f].camera.height * 3;
      }
      bool same_size = true;
      for (size_t f = 0; f < vs.size(); ++f)
        same_size = same_size && rot[f].camera.width == rot[0].camera.width &&
                    rot[f].camera.height == rot[0].camera.height;
      if (same_size) rc = higs_render_views(ctx, (int32_t)rot.size(), rot.data(), stream);
    }
    if (!rc) rc = higs_render_views(ctx, (int32_t)vs.size(), vs.data(), stream);
    higs_counts cn{};
    if (!rc && higs_get_counts(ctx, &cn)) return 4;
    for (size_t f = 0; f < cams.size(); ++f) {
      const size_t npx = (size_t)cams[f].width * cams[f].height;
      const std::string pre = out + "/f" + std::to_string(f) + "_";
      save(pre + "image", bufs[f], npx * 12);
      save(pre + "T", bufs[f] + npx * 3, npx * 4);
      fprintf(summary, "%d %lld %lld %lld %lld %u %d\n", rc, (long long)cn.n_visible,
              (long long)cn.n_pairs, (long long)cn.n_batches, (long long)cn.n_evaluations,
              cn.overflow, cn.graphs);
    }
    fclose(summary);
    higs_ctx_destroy(ctx);
    return 0;
  }
  for (size_t f = 0; f < cams.size(); ++f) {
    const higs_camera& c = cams[f];
    const size_t npx = (size_t)c.width * c.height;
    // outputs in a shared mapping: with CPUHIP_PROCS > 1 the workgroups that
    // write them run in other processes
    float* image_p = static_cast<float*>(mmap(nullptr, npx * 16, PROT_READ | PROT_WRITE,
                                              MAP_SHARED | MAP_ANONYMOUS, -1, 0));
    if (image_p == MAP_FAILED) return 2;
    float* T_p = image_p + npx * 3;
    for (size_t q = 0; q < npx * 4; ++q) image_p[q] = -7.0f;
    struct View {
      float* p;
      size_t n;
      float* data() { return p; }
      size_t size() const { return n; }
    } image{image_p, npx * 3}, T{T_p, npx};
    int rc = 0;
    higs_counts cn{};
    const std::string pre = out + "/f" + std::to_string(f) + "_";
    if (entry == 3) {
      rc = higs_render(ctx, uses[f], means.data(), scales.data(), quats.data(), opac.data(), sh_in,
                       &c, image.data(), T.data(), stream);
      if (!rc && higs_get_counts(ctx, &cn)) return 4;
    } else if (entry == 0) {
      // stage by stage, reading back each stage's output as soon as it exists,
      // so that a failure names its stage
      rc = higs_project(ctx, uses[f], means.data(), scales.data(), quats.data(), opac.data(),
                        sh_in, &c, nullptr);
      if (!rc) rc = higs_bin_sort(ctx, nullptr);
      if (!rc && higs_get_counts(ctx, &cn)) return 4;
      if (!rc && !cn.overflow && (debug_flags & HIGS_DEBUG_KEEP_PAIRS)) {
        const size_t np = (size_t)cn.n_pairs;
        std::vector<unsigned char> pairs(np * 12);
        if (np && higs_debug_copy(ctx, HIGS_DBG_PAIRS, pairs.data(), pairs.size())) return 4;
        save(pre + "pairs", pairs.data(), pairs.size());
      }
      if (!rc && !cn.overflow) {
        const size_t np = (size_t)cn.n_pairs;
        std::vector<unsigned char> pairs(np * 12);
        if (np && higs_debug_copy(ctx, HIGS_DBG_SORTED, pairs.data(), pairs.size())) return 4;
        save(pre + "sorted", pairs.data(), pairs.size());
      }
      if (!rc) rc = higs_batch(ctx, nullptr);
      if (!rc && higs_get_counts(ctx, &cn)) return 4;
      if (!rc && !cn.overflow) {
        const size_t nb = (size_t)cn.n_batches;
        std::vector<uint32_t> tab(nb * 3);
        if (nb && higs_debug_copy(ctx, HIGS_DBG_BATCHES, tab.data(), tab.size() * 4)) return 4;
        save(pre + "batches", tab.data(), tab.size() * 4);
      }
      if (!rc) rc = higs_raster(ctx, image.data(), T.data(), nullptr);
      if (!rc && higs_get_counts(ctx, &cn)) return 4;
    } else {
      rc = higs_render_noalloc ? higs_render_noalloc(uses[f], means.data(), scales.data(),
                                                     quats.data(), opac.data(), sh.data(), &c,
                                                     image.data(), T.data(), nullptr)
                               : -100;
    }
    save(pre + "image", image.data(), image.size() * 4);
    save(pre + "T", T.data(), T.size() * 4);
    munmap(image_p, npx * 16);
    fprintf(summary, "%d %lld %lld %lld %lld %u %d\n", rc, (long long)cn.n_visible,
            (long long)cn.n_pairs, (long long)cn.n_batches, (long long)cn.n_evaluations,
            cn.overflow, cn.graphs);
    fflush(summary);
  }
  fclose(summary);
  if (ctx) higs_ctx_destroy(ctx);
  return 0;
}
