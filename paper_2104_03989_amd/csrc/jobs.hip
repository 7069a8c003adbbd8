// Job server of the C ABI: whole simplification jobs (the paper's statement
// of the problem, Sec. 3: reference model, view/light distribution and an
// initial latent model in; optimised mesh and maps out), admitted by HBM
// budget, kept resident on the device and stepped by one server thread.
//
// Continuous batching: the server keeps kSlots execution slots (a stream and
// a context whose scratch serves the steps queued on it, in stream order).
// Each slot keeps kDepth steps queued: whenever one completes (polled with
// hipEventQuery) the slot enqueues the next step of an active job that has
// none in flight (round robin, so steps of different jobs interleave and
// overlap on the device, and a job never waits for a round of other jobs),
// or else the next step of a job already on it (so a job stepping alone
// has its next step queued while the current one runs).  Queued jobs are admitted between any two
// dispatches as soon as their footprint, plus the slots' scratch for their
// shapes, fits the budget; their uploads run on an admission stream of
// their own.  Per-step latency is device time from an event recorded when
// the step is enqueued to the step's completion event; p50/p99 are reported
// per job.
//
// Cameras and lights of every step are drawn at admission from a
// counter-based generator (SplitMix64, Steele, Lea and Flood 2014: value i
// of a stream is the SplitMix64 output function of seed + (i+1) * golden
// gamma) and kept in HBM, so a step needs no host work.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "jobs.h"

namespace adr {

namespace {

constexpr int kSlots = 4;
// Steps queued per slot and per job: the host enqueues the next step while
// the device runs the current one, so a job stepping alone is not bound by
// the launch latency of its ~30 calls.
constexpr int kDepth = 2;
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t seed, uint64_t i) {
  return (double)(splitmix_out(seed + (i + 1) * kGamma) >> 11) * (1.0 / 9007199254740992.0);
}

// Three normal deviates from four uniforms (Box-Muller), normalised.
void unit_vector(uint64_t seed, uint64_t base, double out[3]) {
  double g[4];
  for (int k = 0; k < 2; ++k) {
    double u1 = 1.0 - uniform01(seed, base + 2 * k), u2 = uniform01(seed, base + 2 * k + 1);
    double r = sqrt(-2.0 * log(u1));
    g[2 * k] = r * cos(2.0 * M_PI * u2);
    g[2 * k + 1] = r * sin(2.0 * M_PI * u2);
  }
  double n = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  if (!(n > 0.0)) n = 1.0, g[0] = 0.0, g[1] = 0.0, g[2] = 1.0;
  for (int k = 0; k < 3; ++k) out[k] = g[k] / n;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int chain_texels(int size, int levels) {
  int n = 0;
  for (int l = 0; l < levels; ++l) n += (size >> l) * (size >> l);
  return n;
}

int full_levels(int size) {
  int l = 1;
  while ((1 << (l - 1)) < size) ++l;
  return l;
}

using Clock = std::chrono::steady_clock;

}  // namespace

extern "C" adr_status adr_job_views(uint64_t seed, int32_t step, int32_t n_views, int32_t light_per_view,
                                    float* dirs, float* lights) {
  if (n_views < 1 || step < 0 || !dirs || !lights) return ADR_E_INVALID;
  for (int b = 0; b < n_views; ++b) {
    double d[3], l[3];
    uint64_t base = ((uint64_t)step * (uint64_t)n_views + (uint64_t)b) * 8ull;
    unit_vector(seed, base, d);
    uint64_t lb = light_per_view ? base + 4 : (uint64_t)step * (uint64_t)n_views * 8ull + 4;
    unit_vector(seed, lb, l);
    for (int k = 0; k < 3; ++k) {
      dirs[3 * b + k] = (float)d[k];
      lights[3 * b + k] = (float)l[k];
    }
  }
  return ADR_OK;
}

struct JobTex {
  void* data = nullptr;
  int size = 0, levels = 0, channels = 0, fmt = 0;
  adr_texture tex() const { return adr_texture{data, size, levels, channels, fmt}; }
};

struct Job {
  uint64_t id = 0;
  int state = ADR_JOB_QUEUED;
  int step = 0;
  float last_loss = 0.f;
  size_t footprint = 0;
  char why[200] = "";
  adr_job_desc d{};
  // host copies
  std::vector<float> ref_pos, ref_uv, lat_pos, lat_uv, ref_normal, ref_orm, lat_normal, lat_orm;
  std::vector<int32_t> ref_tri, ref_uv_tri, lat_tri, lat_uv_tri, ref_adj, lat_adj;
  std::vector<uint8_t> ref_kd, lat_kd;
  // device
  void* block = nullptr;
  adr_mesh ref_mesh{}, lat_mesh{};
  JobTex rkd, rnm, rorm, kd, nm, orm;
  float *g_pos = nullptr, *g_kd = nullptr, *g_nm = nullptr, *g_orm = nullptr;
  float *m[4] = {nullptr, nullptr, nullptr, nullptr}, *v[4] = {nullptr, nullptr, nullptr, nullptr};
  float *mvp = nullptr, *eye = nullptr, *light = nullptr, *rgb = nullptr;
  uint64_t *ref_vis = nullptr, *vis = nullptr;
  float *ref_color = nullptr, *ref_image = nullptr, *color = nullptr, *dimage = nullptr, *loss = nullptr;
  // up to kDepth steps of a job in flight, stream-ordered on one slot;
  // step t uses ring entry t % kDepth
  float* loss_host = nullptr;  // pinned, kDepth floats
  hipEvent_t start_ev[kDepth] = {}, done_ev[kDepth] = {};
  int inflight = 0;            // steps enqueued and not yet completed (all on one slot)
  bool stopping = false;       // failed: enqueue nothing more, release once the queued steps are done
  std::vector<float> lat_ms;
  // results
  std::vector<float> out_pos, out_normal, out_orm;
  std::vector<uint8_t> out_kd;
};

// An execution slot: a stream, a context whose scratch serves the steps on
// it (stream-ordered), the latent forward's received antialiasing (read by
// the backward that follows it), and the steps queued on it.
struct Slot {
  adr_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  float* aa = nullptr;
  size_t aa_cap = 0;
  // the steps queued on the stream, oldest first: (job, step)
  std::deque<std::pair<Job*, int>> q;
};

struct JobServer {
  adr_ctx* owner = nullptr;
  int device = 0;
  uint64_t budget = 0;
  uint64_t used = 0;            // resident jobs' footprints
  uint64_t scratch_hw = 0;      // per-slot scratch the admitted shapes need (grows, never shrinks)
  uint64_t next_id = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::vector<uint64_t> active;
  size_t rr = 0;                // round-robin cursor over active
  std::thread th;
  bool stop = false;
  bool started = false;
  Slot slot[kSlots];
  adr_ctx* adm_ctx = nullptr;   // admission: uploads, reference frame, mip chains
  hipStream_t adm_stream = nullptr;
};

namespace {

size_t tex_bytes(int size, int fmt, int channels) {
  int L = full_levels(size);
  return (size_t)chain_texels(size, L) * (fmt == ADR_TEX_RGBA8 ? 4 : 4 * (size_t)channels);
}

// Device bytes of a job (everything in its one allocation).
size_t job_bytes(const adr_job_desc& d) {
  size_t B = d.n_views, HW = (size_t)d.width * d.height;
  size_t s = 0;
  auto add = [&](size_t x) { s += align256(x); };
  add(d.ref_n_pos * 12);
  add(d.ref_n_tri * 12);
  add(d.ref_n_uv * 8);
  add(d.ref_n_tri * 12);
  add(d.ref_n_tri * 12);
  add(d.ref_n_pos * 24);  // reference vertex frame, computed once
  add(d.lat_n_pos * 12);
  add(d.lat_n_tri * 12);
  add(d.lat_n_uv * 8);
  add(d.lat_n_tri * 12);
  add(d.lat_n_tri * 12);
  add(tex_bytes(d.ref_kd_size, d.ref_kd_format, 3));
  add(tex_bytes(d.ref_normal_size, ADR_TEX_F32, 3));
  if (d.model == ADR_SHADE_GGX) add(tex_bytes(d.ref_orm_size, ADR_TEX_F32, 3));
  add(tex_bytes(d.lat_kd_size, d.lat_kd_format, 3));
  add(tex_bytes(d.lat_normal_size, ADR_TEX_F32, 3));
  if (d.model == ADR_SHADE_GGX) add(tex_bytes(d.lat_orm_size, ADR_TEX_F32, 3));
  // gradients (chain layout) and Adam state (level 0)
  add(d.lat_n_pos * 12 * 3);
  if (d.opt_mask & 2) {
    add(tex_bytes(d.lat_kd_size, ADR_TEX_F32, 3));
    add((size_t)d.lat_kd_size * d.lat_kd_size * 12 * 2);
  }
  if (d.opt_mask & 4) {
    add(tex_bytes(d.lat_normal_size, ADR_TEX_F32, 3));
    add((size_t)d.lat_normal_size * d.lat_normal_size * 12 * 2);
  }
  if ((d.opt_mask & 8) && d.model == ADR_SHADE_GGX) {
    add(tex_bytes(d.lat_orm_size, ADR_TEX_F32, 3));
    add((size_t)d.lat_orm_size * d.lat_orm_size * 12 * 2);
  }
  add((size_t)d.n_steps * B * 16 * 4);
  add((size_t)d.n_steps * B * 3 * 4 * 3);
  add(B * HW * 8 * 2);          // visibility of reference and latent
  add(B * HW * 12 * 4);         // reference colour and image, latent colour and dL/dimage
  add(256);                     // loss
  return s;
}

// Scratch a slot needs to step a job of this shape: the slot context's
// buffers as the render calls size them (for the larger of the two meshes,
// with the growth margin of a quarter the context allocates), and the
// slot's received-antialiasing buffer.
size_t slot_scratch_bytes(const adr_job_desc& d) {
  const size_t B = d.n_views, HW = (size_t)d.width * d.height;
  const size_t V = std::max(d.ref_n_pos, d.lat_n_pos), T = std::max(d.ref_n_tri, d.lat_n_tri);
  const size_t tiles = (size_t)((d.width + 15) / 16) * ((d.height + 15) / 16) * B;
  const size_t maps = 1 + ((d.opt_mask & 2) ? 1 : 0) + ((d.opt_mask & 4) ? 1 : 0) +
                      (((d.opt_mask & 8) && d.model == ADR_SHADE_GGX) ? 1 : 0);
  const size_t parts[] = {B * V * 16, B * T, V * 24, V * 24, V * 12, V * 12, B * T * 4, (B + 1) * 4, B * T * 4,
                          tiles * 4, B * HW * 12, B * V * 16, V * 36, maps * B * HW * 16, V * 72, B * V * 32,
                          V * 24};
  size_t s = 0;
  for (size_t x : parts) s += align256(x + x / 4);
  return s + align256(B * HW * 32);
}

adr_status copy_desc(Job& j, const adr_job_desc& d, char* msg, size_t n) {
  auto bad = [&](const char* what) {
    snprintf(msg, n, "job description: %s", what);
    return ADR_E_INVALID;
  };
  if (d.ref_n_pos < 1 || d.ref_n_tri < 1 || d.ref_n_uv < 1 || d.lat_n_pos < 1 || d.lat_n_tri < 1 || d.lat_n_uv < 1)
    return bad("empty mesh");
  if (!d.ref_pos || !d.ref_tri || !d.ref_uv || !d.ref_uv_tri || !d.lat_pos || !d.lat_tri || !d.lat_uv || !d.lat_uv_tri)
    return bad("mesh arrays are required");
  if (d.model != ADR_SHADE_BLINN_PHONG && d.model != ADR_SHADE_GGX) return bad("model");
  auto pow2 = [](int x) { return x > 0 && x <= 16384 && (x & (x - 1)) == 0; };
  if (!pow2(d.ref_kd_size) || !pow2(d.ref_normal_size) || !pow2(d.lat_kd_size) || !pow2(d.lat_normal_size))
    return bad("map sizes must be powers of two");
  if (!d.ref_kd || !d.ref_normal || !d.lat_kd || !d.lat_normal) return bad("maps are required");
  if (d.model == ADR_SHADE_GGX && (!pow2(d.ref_orm_size) || !pow2(d.lat_orm_size) || !d.ref_orm || !d.lat_orm))
    return bad("GGX needs ORM maps");
  if ((d.ref_kd_format != ADR_TEX_F32 && d.ref_kd_format != ADR_TEX_RGBA8) ||
      (d.lat_kd_format != ADR_TEX_F32 && d.lat_kd_format != ADR_TEX_RGBA8))
    return bad("kd format");
  if ((d.opt_mask & 2) && d.lat_kd_format != ADR_TEX_F32) return bad("optimised kd must be F32");
  if (d.n_views < 1 || d.n_views > 64 || d.width < 1 || d.width > 4096 || d.height < 1 || d.height > 4096)
    return bad("views");
  if (d.n_steps < 1 || d.n_steps > 1000000) return bad("n_steps");
  if (d.loss_kind < ADR_LOSS_L1 || d.loss_kind > ADR_LOSS_L2_TONEMAP) return bad("loss kind");
  if (!(d.dist > 0.f) || !(d.fov_deg > 0.f && d.fov_deg < 180.f) || !(d.lr0 > 0.f)) return bad("camera or lr");
  j.d = d;
  auto cp = [](auto& dst, const auto* src, size_t count) { dst.assign(src, src + count); };
  cp(j.ref_pos, d.ref_pos, 3 * (size_t)d.ref_n_pos);
  cp(j.ref_tri, d.ref_tri, 3 * (size_t)d.ref_n_tri);
  cp(j.ref_uv, d.ref_uv, 2 * (size_t)d.ref_n_uv);
  cp(j.ref_uv_tri, d.ref_uv_tri, 3 * (size_t)d.ref_n_tri);
  cp(j.lat_pos, d.lat_pos, 3 * (size_t)d.lat_n_pos);
  cp(j.lat_tri, d.lat_tri, 3 * (size_t)d.lat_n_tri);
  cp(j.lat_uv, d.lat_uv, 2 * (size_t)d.lat_n_uv);
  cp(j.lat_uv_tri, d.lat_uv_tri, 3 * (size_t)d.lat_n_tri);
  for (int k = 0; k < 3 * d.ref_n_tri; ++k)
    if (j.ref_tri[k] < 0 || j.ref_tri[k] >= d.ref_n_pos || j.ref_uv_tri[k] < 0 || j.ref_uv_tri[k] >= d.ref_n_uv)
      return bad("reference index out of range");
  for (int k = 0; k < 3 * d.lat_n_tri; ++k)
    if (j.lat_tri[k] < 0 || j.lat_tri[k] >= d.lat_n_pos || j.lat_uv_tri[k] < 0 || j.lat_uv_tri[k] >= d.lat_n_uv)
      return bad("latent index out of range");
  size_t rk = (size_t)d.ref_kd_size * d.ref_kd_size * (d.ref_kd_format == ADR_TEX_RGBA8 ? 4 : 12);
  size_t lk = (size_t)d.lat_kd_size * d.lat_kd_size * (d.lat_kd_format == ADR_TEX_RGBA8 ? 4 : 12);
  cp(j.ref_kd, (const uint8_t*)d.ref_kd, rk);
  cp(j.lat_kd, (const uint8_t*)d.lat_kd, lk);
  cp(j.ref_normal, d.ref_normal, 3 * (size_t)d.ref_normal_size * d.ref_normal_size);
  cp(j.lat_normal, d.lat_normal, 3 * (size_t)d.lat_normal_size * d.lat_normal_size);
  if (d.model == ADR_SHADE_GGX) {
    cp(j.ref_orm, d.ref_orm, 3 * (size_t)d.ref_orm_size * d.ref_orm_size);
    cp(j.lat_orm, d.lat_orm, 3 * (size_t)d.lat_orm_size * d.lat_orm_size);
  }
  j.ref_adj.resize(3 * (size_t)d.ref_n_tri);
  j.lat_adj.resize(3 * (size_t)d.lat_n_tri);
  adr_mesh_adjacency(j.ref_tri.data(), d.ref_n_tri, j.ref_adj.data());
  adr_mesh_adjacency(j.lat_tri.data(), d.lat_n_tri, j.lat_adj.data());
  // point the stored description at the copies
  j.d.ref_pos = j.ref_pos.data(); j.d.ref_tri = j.ref_tri.data(); j.d.ref_uv = j.ref_uv.data();
  j.d.ref_uv_tri = j.ref_uv_tri.data(); j.d.lat_pos = j.lat_pos.data(); j.d.lat_tri = j.lat_tri.data();
  j.d.lat_uv = j.lat_uv.data(); j.d.lat_uv_tri = j.lat_uv_tri.data();
  j.d.ref_kd = j.ref_kd.data(); j.d.lat_kd = j.lat_kd.data();
  j.d.ref_normal = j.ref_normal.data(); j.d.lat_normal = j.lat_normal.data();
  j.d.ref_orm = j.ref_orm.empty() ? nullptr : j.ref_orm.data();
  j.d.lat_orm = j.lat_orm.empty() ? nullptr : j.lat_orm.data();
  return ADR_OK;
}

// Carves the job's single allocation and uploads everything (on stream st).
adr_status admit(JobServer* s, Job& j, hipStream_t st, adr_ctx* ctx) {
  const adr_job_desc& d = j.d;
  if (hipMalloc(&j.block, j.footprint) != hipSuccess) return ADR_E_NOMEM;
  if (hipHostMalloc((void**)&j.loss_host, kDepth * sizeof(float)) != hipSuccess) return ADR_E_NOMEM;
  for (int k = 0; k < kDepth; ++k)
    if (hipEventCreate(&j.start_ev[k]) != hipSuccess || hipEventCreate(&j.done_ev[k]) != hipSuccess) return ADR_E_HIP;
  char* p = (char*)j.block;
  auto take = [&](size_t bytes) {
    void* r = p;
    p += align256(bytes);
    return r;
  };
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
  };
  bool ok = true;
  auto mesh = [&](adr_mesh& m, const std::vector<float>& pos, const std::vector<int32_t>& tri,
                  const std::vector<float>& uv, const std::vector<int32_t>& uvt,
                  const std::vector<int32_t>& adj, int np, int nt, int nu) {
    m.pos = (float*)take(np * 12);
    m.tri = (int32_t*)take(nt * 12);
    m.uv = (float*)take(nu * 8);
    m.uv_tri = (int32_t*)take(nt * 12);
    m.adj = (int32_t*)take(nt * 12);
    m.n_pos = np;
    m.n_tri = nt;
    m.n_uv = nu;
    ok &= up((void*)m.pos, pos.data(), np * 12) && up((void*)m.tri, tri.data(), nt * 12) &&
          up((void*)m.uv, uv.data(), nu * 8) && up((void*)m.uv_tri, uvt.data(), nt * 12) &&
          up((void*)m.adj, adj.data(), nt * 12);
  };
  mesh(j.ref_mesh, j.ref_pos, j.ref_tri, j.ref_uv, j.ref_uv_tri, j.ref_adj, d.ref_n_pos, d.ref_n_tri, d.ref_n_uv);
  {
    // the reference never moves: its vertex frame is computed once here
    float* frame = (float*)take((size_t)d.ref_n_pos * 24);
    ok &= adr_mesh_frame(ctx, &j.ref_mesh, frame, frame + 3 * (size_t)d.ref_n_pos, (adr_stream)st) == ADR_OK;
    j.ref_mesh.nrm = frame;
    j.ref_mesh.tan = frame + 3 * (size_t)d.ref_n_pos;
  }
  mesh(j.lat_mesh, j.lat_pos, j.lat_tri, j.lat_uv, j.lat_uv_tri, j.lat_adj, d.lat_n_pos, d.lat_n_tri, d.lat_n_uv);
  auto tex = [&](JobTex& t, const void* src, int size, int fmt) {
    t.size = size;
    t.levels = full_levels(size);
    t.fmt = fmt;
    t.channels = fmt == ADR_TEX_RGBA8 ? 4 : 3;
    t.data = take(tex_bytes(size, fmt, 3));
    ok &= up(t.data, src, (size_t)size * size * (fmt == ADR_TEX_RGBA8 ? 4 : 12));
    adr_texture at = t.tex();
    ok &= adr_mip_build(ctx, &at, (adr_stream)st) == ADR_OK;
  };
  tex(j.rkd, j.ref_kd.data(), d.ref_kd_size, d.ref_kd_format);
  tex(j.rnm, j.ref_normal.data(), d.ref_normal_size, ADR_TEX_F32);
  if (d.model == ADR_SHADE_GGX) tex(j.rorm, j.ref_orm.data(), d.ref_orm_size, ADR_TEX_F32);
  tex(j.kd, j.lat_kd.data(), d.lat_kd_size, d.lat_kd_format);
  tex(j.nm, j.lat_normal.data(), d.lat_normal_size, ADR_TEX_F32);
  if (d.model == ADR_SHADE_GGX) tex(j.orm, j.lat_orm.data(), d.lat_orm_size, ADR_TEX_F32);
  // gradients and Adam state, zeroed
  std::vector<std::pair<void*, size_t>> zero;
  j.g_pos = (float*)take(d.lat_n_pos * 12 * 3);
  j.m[0] = j.g_pos + 3 * d.lat_n_pos;
  j.v[0] = j.g_pos + 6 * d.lat_n_pos;
  zero.push_back({j.g_pos, (size_t)d.lat_n_pos * 36});
  auto gmap = [&](float*& g, float*& m, float*& v, const JobTex& t) {
    size_t chain = tex_bytes(t.size, ADR_TEX_F32, 3), lvl0 = (size_t)t.size * t.size * 12;
    g = (float*)take(chain);
    m = (float*)take(lvl0 * 2);
    v = m + lvl0 / 4;
    zero.push_back({g, chain});
    zero.push_back({m, lvl0 * 2});
  };
  if (d.opt_mask & 2) gmap(j.g_kd, j.m[1], j.v[1], j.kd);
  if (d.opt_mask & 4) gmap(j.g_nm, j.m[2], j.v[2], j.nm);
  if ((d.opt_mask & 8) && d.model == ADR_SHADE_GGX) gmap(j.g_orm, j.m[3], j.v[3], j.orm);
  // cameras and lights of every step
  size_t B = d.n_views, N = (size_t)d.n_steps * B;
  j.mvp = (float*)take(N * 64);
  float* e3 = (float*)take(N * 36);
  j.eye = e3;
  j.light = e3 + 3 * N;
  j.rgb = e3 + 6 * N;
  {
    std::vector<float> mvp(N * 16), eye(N * 3), lit(N * 3), rgb(N * 3, 1.0f), dirs(B * 3);
    for (int t = 0; t < d.n_steps; ++t) {
      adr_job_views(d.seed, t, (int)B, d.light_per_view, dirs.data(), lit.data() + 3 * B * t);
      adr_views_build(dirs.data(), (int)B, d.dist, d.fov_deg, d.width, d.height, mvp.data() + 16 * B * t,
                      eye.data() + 3 * B * t);
    }
    ok &= up(j.mvp, mvp.data(), N * 64) && up(j.eye, eye.data(), N * 12) && up(j.light, lit.data(), N * 12) &&
          up(j.rgb, rgb.data(), N * 12);
    ok &= hipStreamSynchronize(st) == hipSuccess;  // host vectors go out of scope
  }
  size_t HW = (size_t)d.width * d.height;
  j.ref_vis = (uint64_t*)take(B * HW * 8);
  j.vis = (uint64_t*)take(B * HW * 8);
  j.ref_color = (float*)take(B * HW * 12);
  j.ref_image = (float*)take(B * HW * 12);
  j.color = (float*)take(B * HW * 12);
  j.dimage = (float*)take(B * HW * 12);
  j.loss = (float*)take(256);
  for (auto& z : zero) ok &= launch_fill_f32((float*)z.first, (int64_t)(z.second / 4), 0.f, st) == hipSuccess;
  ok &= (size_t)(p - (char*)j.block) <= j.footprint;
  return ok ? ADR_OK : ADR_E_HIP;
}

void release_dev(Job& j) {
  if (j.block) (void)hipFree(j.block);
  if (j.loss_host) (void)hipHostFree(j.loss_host);
  for (int k = 0; k < kDepth; ++k) {
    if (j.start_ev[k]) (void)hipEventDestroy(j.start_ev[k]);
    if (j.done_ev[k]) (void)hipEventDestroy(j.done_ev[k]);
    j.start_ev[k] = j.done_ev[k] = nullptr;
  }
  j.block = nullptr;
  j.loss_host = nullptr;
}

// Optimisation step t of job j on slot sl, bracketed by the start and
// completion events of its ring entry.
adr_status enqueue_step(Slot& sl, Job& j, int t) {
  const adr_job_desc& d = j.d;
  adr_ctx* ctx = sl.ctx;
  hipStream_t st = sl.st;
  const int q = t % kDepth;
  if (hipEventRecord(j.start_ev[q], st) != hipSuccess) return ADR_E_HIP;
  size_t B = d.n_views;
  adr_views v{j.mvp + 16 * B * t, j.eye + 3 * B * t, j.light + 3 * B * t, j.rgb + 3 * B * t, (int)B, d.width,
              d.height};
  adr_material rm{d.model, j.rkd.tex(), j.rnm.tex(), d.model == ADR_SHADE_GGX ? j.rorm.tex() : j.rkd.tex()};
  adr_material lm{d.model, j.kd.tex(), j.nm.tex(), d.model == ADR_SHADE_GGX ? j.orm.tex() : j.kd.tex()};
  adr_fwd_out ro{j.ref_vis, j.ref_color, j.ref_image, nullptr, nullptr, nullptr, nullptr};
  adr_status r = adr_render_fwd(ctx, &j.ref_mesh, &rm, &v, nullptr, 0, &ro, 0, st);
  if (r != ADR_OK) return r;
  const size_t aa_bytes = B * (size_t)d.width * d.height * 32;
  if (sl.aa_cap < aa_bytes) {
    if (sl.aa && hipFree(sl.aa) != hipSuccess) return ADR_E_HIP;
    sl.aa = nullptr;
    sl.aa_cap = 0;
    if (hipMalloc(&sl.aa, aa_bytes) != hipSuccess) return ADR_E_NOMEM;
    sl.aa_cap = aa_bytes;
  }
  adr_fwd_out lo{j.vis, j.color, nullptr, j.dimage, j.loss, nullptr, nullptr, sl.aa};
  // the map Adam rebuilds the latent chains after every step; the first
  // forward builds them
  r = adr_render_fwd(ctx, &j.lat_mesh, &lm, &v, j.ref_image, d.loss_kind, &lo, t == 0 ? ADR_FWD_BUILD_MIPS : 0, st);
  if (r != ADR_OK) return r;
  adr_grads g{(d.opt_mask & 1) ? j.g_pos : nullptr, nullptr, j.g_kd, j.g_nm, j.g_orm};
  r = adr_render_bwd(ctx, &j.lat_mesh, &lm, &v, &lo, nullptr, &g, ADR_BWD_DEFER_MIP_ADJOINT, st);
  if (r != ADR_OK) return r;
  float lr = d.lr0 * powf(10.0f, -d.lr_decay_k * (float)t);
  if (d.opt_mask & 1) {
    adr_param prm{(float*)j.lat_mesh.pos, j.g_pos, j.m[0], j.v[0], 3 * (int64_t)d.lat_n_pos};
    r = adr_adam_step(ctx, &prm, 1, t + 1, lr, 0.9f, 0.999f, 1e-8f, st);
    if (r != ADR_OK) return r;
  }
  adr_map_param mp[3];
  int nm = 0;
  if (j.g_kd) mp[nm++] = adr_map_param{j.kd.tex(), j.g_kd, j.m[1], j.v[1]};
  if (j.g_nm) mp[nm++] = adr_map_param{j.nm.tex(), j.g_nm, j.m[2], j.v[2]};
  if (j.g_orm) mp[nm++] = adr_map_param{j.orm.tex(), j.g_orm, j.m[3], j.v[3]};
  r = adr_adam_step_maps(ctx, mp, nm, t + 1, lr, 0.9f, 0.999f, 1e-8f, st);
  if (r != ADR_OK) return r;
  if (hipMemcpyAsync(j.loss_host + q, j.loss, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess)
    return ADR_E_HIP;
  if (hipEventRecord(j.done_ev[q], st) != hipSuccess) return ADR_E_HIP;
  return ADR_OK;
}

// Copies the optimised model to host memory and releases the job's device
// memory (on a stream the job's steps are complete on).
void finish(hipStream_t st, Job& j) {
  const adr_job_desc& d = j.d;
  j.out_pos.resize(3 * (size_t)d.lat_n_pos);
  (void)hipMemcpyAsync(j.out_pos.data(), j.lat_mesh.pos, j.out_pos.size() * 4, hipMemcpyDeviceToHost, st);
  size_t kdb = (size_t)j.kd.size * j.kd.size * (j.kd.fmt == ADR_TEX_RGBA8 ? 4 : 12);
  j.out_kd.resize(kdb);
  (void)hipMemcpyAsync(j.out_kd.data(), j.kd.data, kdb, hipMemcpyDeviceToHost, st);
  j.out_normal.resize(3 * (size_t)j.nm.size * j.nm.size);
  (void)hipMemcpyAsync(j.out_normal.data(), j.nm.data, j.out_normal.size() * 4, hipMemcpyDeviceToHost, st);
  if (d.model == ADR_SHADE_GGX) {
    j.out_orm.resize(3 * (size_t)j.orm.size * j.orm.size);
    (void)hipMemcpyAsync(j.out_orm.data(), j.orm.data, j.out_orm.size() * 4, hipMemcpyDeviceToHost, st);
  }
  (void)hipStreamSynchronize(st);
  release_dev(j);
}

// Admits queued jobs in arrival order while their footprint and the slots'
// scratch for their shapes fit the budget.  Called with the lock held; drops
// it while a job uploads.
void admit_queued(JobServer* s, std::unique_lock<std::mutex>& lk) {
  while (!s->queue.empty()) {
    Job& j = *s->jobs.at(s->queue.front());
    const uint64_t hw = std::max<uint64_t>(s->scratch_hw, slot_scratch_bytes(j.d));
    if (s->used + j.footprint + (uint64_t)kSlots * hw > s->budget) break;
    s->queue.pop_front();
    s->used += j.footprint;
    s->scratch_hw = hw;
    lk.unlock();
    adr_status r = admit(s, j, s->adm_stream, s->adm_ctx);
    lk.lock();
    if (r != ADR_OK) {
      snprintf(j.why, sizeof(j.why), "admission failed (%d): %s", r, adr_last_error());
      release_dev(j);
      s->used -= j.footprint;
      j.state = ADR_JOB_FAILED;
    } else {
      j.state = ADR_JOB_RUNNING;
      s->active.push_back(j.id);
    }
  }
}

// Releases a job that ended (done: its results copied out first) once no
// step of it is in flight.  Called with the lock held.
void retire(JobServer* s, Job& j) {
  if (j.state == ADR_JOB_RUNNING && j.step >= j.d.n_steps) {
    finish(s->adm_stream, j);
    j.state = ADR_JOB_DONE;
  } else {
    release_dev(j);
  }
  s->used -= j.footprint;
  s->active.erase(std::find(s->active.begin(), s->active.end(), j.id));
}

// The oldest step queued on slot sl has completed: its loss and device
// latency.  Called with the lock held.
void complete_head(JobServer* s, Slot& sl) {
  Job& j = *sl.q.front().first;
  const int t = sl.q.front().second;
  sl.q.pop_front();
  j.inflight -= 1;
  const int q = t % kDepth;
  float ms = 0.f;
  hipError_t e = hipEventElapsedTime(&ms, j.start_ev[q], j.done_ev[q]);
  const float loss = j.loss_host[q];
  if (!j.stopping) {
    if (e != hipSuccess) {
      snprintf(j.why, sizeof(j.why), "step %d: %s", t + 1, hipGetErrorString(e));
      j.stopping = true;
    } else if (!std::isfinite(loss)) {
      snprintf(j.why, sizeof(j.why), "non-finite loss %g at step %d", loss, t + 1);
      j.stopping = true;
    } else {
      j.lat_ms.push_back(ms);
      j.last_loss = loss;
      j.step = t + 1;
    }
  }
  if (j.stopping && j.inflight == 0) {
    j.state = ADR_JOB_FAILED;
    retire(s, j);
  } else if (j.step >= j.d.n_steps && j.inflight == 0) {
    retire(s, j);
  }
}

// The job slot k enqueues next: an active job with no step in flight (round
// robin: steps of different jobs interleave), else the next step of a job
// already queued on this slot (its steps must stay on one stream).
Job* next_for_slot(JobServer* s, int k) {
  const size_t n = s->active.size();
  for (size_t i = 0; i < n; ++i) {
    const size_t c = (s->rr + i) % n;
    Job* j = s->jobs.at(s->active[c]).get();
    if (j->inflight == 0 && !j->stopping && j->step < j->d.n_steps) {
      s->rr = (c + 1) % n;
      return j;
    }
  }
  for (auto& e : s->slot[k].q) {
    Job* j = e.first;
    if (j->inflight < kDepth && !j->stopping && j->step + j->inflight < j->d.n_steps) return j;
  }
  return nullptr;
}

void server_loop(JobServer* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    admit_queued(s, lk);
    int busy = 0;
    for (int k = 0; k < kSlots; ++k) {
      Slot& sl = s->slot[k];
      // completed steps, oldest first
      while (!sl.q.empty()) {
        Job& j = *sl.q.front().first;
        const hipError_t q = hipEventQuery(j.done_ev[sl.q.front().second % kDepth]);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess && !j.stopping) {
          snprintf(j.why, sizeof(j.why), "step %d: %s", sl.q.front().second + 1, hipGetErrorString(q));
          j.stopping = true;
          (void)hipStreamSynchronize(sl.st);
        }
        complete_head(s, sl);
      }
      // keep kDepth steps queued on the slot
      while ((int)sl.q.size() < kDepth) {
        Job* j = next_for_slot(s, k);
        if (!j) break;
        const int t = j->step + j->inflight;
        adr_status r = enqueue_step(sl, *j, t);
        if (r != ADR_OK) {
          snprintf(j->why, sizeof(j->why), "step %d could not be launched (%d): %s", t + 1, r, adr_last_error());
          j->stopping = true;
          (void)hipStreamSynchronize(sl.st);
          // the steps of the job already queued have completed; retire it
          // when the loop drains them (at once if none)
          if (j->inflight == 0) {
            j->state = ADR_JOB_FAILED;
            retire(s, *j);
          }
          continue;
        }
        j->inflight += 1;
        sl.q.emplace_back(j, t);
      }
      busy += (int)sl.q.size();
    }
    if (busy == 0 && s->queue.empty()) {
      s->cv.wait_for(lk, std::chrono::milliseconds(50));
    } else {
      // steps take about a millisecond: poll their events every 20 us
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

float percentile(std::vector<float> v, double q) {
  if (v.empty()) return 0.f;
  std::sort(v.begin(), v.end());
  size_t k = (size_t)std::min<double>(v.size() - 1, std::floor(q * (v.size() - 1) + 0.5));
  return v[k];
}

}  // namespace

JobServer* jobs_create(adr_ctx* owner, int device, uint64_t budget) {
  auto* s = new (std::nothrow) JobServer();
  if (!s) return nullptr;
  s->owner = owner;
  s->device = device;
  s->budget = budget;
  for (int k = 0; k < kSlots; ++k) {
    if (adr_ctx_create(device, budget, &s->slot[k].ctx) != ADR_OK ||
        hipStreamCreateWithFlags(&s->slot[k].st, hipStreamNonBlocking) != hipSuccess) {
      jobs_destroy(s);
      return nullptr;
    }
  }
  if (adr_ctx_create(device, budget, &s->adm_ctx) != ADR_OK ||
      hipStreamCreateWithFlags(&s->adm_stream, hipStreamNonBlocking) != hipSuccess) {
    jobs_destroy(s);
    return nullptr;
  }
  return s;
}

void jobs_destroy(JobServer* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  (void)hipDeviceSynchronize();  // steps still in flight
  for (auto& kv : s->jobs) release_dev(*kv.second);
  for (Slot& sl : s->slot) {
    if (sl.aa) (void)hipFree(sl.aa);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.ctx) adr_ctx_destroy(sl.ctx);
  }
  if (s->adm_stream) (void)hipStreamDestroy(s->adm_stream);
  if (s->adm_ctx) adr_ctx_destroy(s->adm_ctx);
  delete s;
}

adr_status jobs_submit(JobServer* s, const adr_job_desc* d, uint64_t* id, char* msg, size_t n) {
  auto j = std::make_unique<Job>();
  adr_status r = copy_desc(*j, *d, msg, n);
  if (r != ADR_OK) return r;
  j->footprint = job_bytes(j->d);
  const uint64_t need = j->footprint + (uint64_t)kSlots * slot_scratch_bytes(j->d);
  if (need > s->budget) {
    snprintf(msg, n, "job needs %llu bytes (with the slots' scratch for its shape), budget is %llu",
             (unsigned long long)need, (unsigned long long)s->budget);
    return ADR_E_OVER_BUDGET;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  j->id = s->next_id++;
  *id = j->id;
  s->queue.push_back(j->id);
  s->jobs[j->id] = std::move(j);
  if (!s->started) {
    s->started = true;
    s->th = std::thread(server_loop, s);
  }
  s->cv.notify_all();
  return ADR_OK;
}

adr_status jobs_poll(JobServer* s, uint64_t id, adr_job_status* st, adr_job_result* out, char* msg, size_t n) {
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) {
    snprintf(msg, n, "unknown job %llu", (unsigned long long)id);
    return ADR_E_NOTFOUND;
  }
  Job& j = *it->second;
  st->state = j.state;
  st->step = j.step;
  st->last_loss = j.last_loss;
  st->p50_ms = percentile(j.lat_ms, 0.50);
  st->p99_ms = percentile(j.lat_ms, 0.99);
  st->device_bytes = (j.state == ADR_JOB_RUNNING) ? j.footprint : 0;
  if (j.state == ADR_JOB_FAILED) {
    snprintf(msg, n, "job %llu failed: %s", (unsigned long long)id, j.why);
    bool nonfinite = strncmp(j.why, "non-finite", 10) == 0;
    s->jobs.erase(it);
    return nonfinite ? ADR_E_NONFINITE : ADR_E_HIP;
  }
  if (j.state != ADR_JOB_DONE) return ADR_PENDING;
  if (out) {
    if (out->pos) memcpy(out->pos, j.out_pos.data(), j.out_pos.size() * 4);
    if (out->kd) memcpy(out->kd, j.out_kd.data(), j.out_kd.size());
    if (out->normal) memcpy(out->normal, j.out_normal.data(), j.out_normal.size() * 4);
    if (out->orm && !j.out_orm.empty()) memcpy(out->orm, j.out_orm.data(), j.out_orm.size() * 4);
    s->jobs.erase(it);
  }
  return ADR_OK;
}

}  // namespace adr
