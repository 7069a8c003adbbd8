// C ABI of the render loop: argument validation, context scratch and the
// stream-ordered launch sequences of one forward and one backward pass.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <unordered_map>
#include <vector>

#include <cmath>

#include "internal.h"
#include "jobs.h"

using namespace adr;

namespace {

thread_local char g_err[512] = "";

adr_status fail(adr_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

}  // namespace

adr_status adr::report(adr_status code, const char* msg) { return fail(code, "%s", msg); }

namespace {

adr_status hip_fail(hipError_t e, const char* where) {
  return fail(ADR_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int x) {
  int l = 0;
  while ((1 << (l + 1)) <= x) ++l;
  return l;
}

}  // namespace

// ----------------------------------------------------------------- context

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Span {
  hipEvent_t a, b;
  int stage;
};

// What the geometry a forward leaves in the scratch (vertex frame and its
// accumulators, snapped vertices, triangle orientations) was computed for.
struct GeomKey {
  const void *pos, *tri, *mvp, *vis;
  int n_pos, n_tri, B, W, H, ms;
  bool det;
  hipStream_t st;
  bool same(const GeomKey& o) const {
    return pos == o.pos && tri == o.tri && mvp == o.mvp && vis == o.vis && n_pos == o.n_pos && n_tri == o.n_tri &&
           B == o.B && W == o.W && H == o.H && ms == o.ms && det == o.det && st == o.st;
  }
};

struct adr_ctx {
  int device = 0;
  uint64_t budget = 0;
  Buf oit_g, oit_a;  // depth-peeling adjoint: dL/d(composite behind) and dL/d alpha per pixel
  Buf snap, orient, nacc, tacc, nrm, tan, big, big_cnt, med, partial, gcolor, dclip, dattr, texrec, image_s, mvpd;
  Buf fix_n, fix_t, fix_attr, fix_clip, fix_pos, det_k0, det_v0, det_k1, det_v1, det_hist, det_tmp, det_vals,
      det_part, lap_r, lap_part;
  adr::JobServer* jobs = nullptr;
  uint32_t prof = 0;  // stages bracketed with events (bit per stage)
  int tiny_bbox = kTinyBBox, med_bbox = kMedBBox;  // raster work split
  // set by a forward that computed the geometry in the scratch; cleared by
  // every other call on the context
  bool geom_ok = false;
  GeomKey geom{};
  std::vector<Span> spans;
  std::vector<hipEvent_t> pool;
  unsigned char* noalloc = nullptr;  // this device's copy of the no-allocation scratch array
};

namespace {

GeomKey geom_key(const MeshD& m, const ViewsD& v, const float* mvp, const void* vis, bool det, hipStream_t st) {
  return GeomKey{m.pos, m.tri, mvp, vis, m.n_pos, m.n_tri, v.B, v.W, v.H, v.ms, det, st};
}

hipEvent_t take_event(adr_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  // timing events without the system-scope release: a plain event record
  // writes back the L2 and stalls the stream for ~10 us at every stage
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel stage with events on its stream while profiling is on.
struct StageTimer {
  adr_ctx* c;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageTimer(adr_ctx* c_, int stage_, hipStream_t st_) : c(c_), stage(stage_), st(st_) {
    if (((c->prof >> stage) & 1u) && (a = take_event(c)) != nullptr) (void)hipEventRecord(a, st);
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) {
      c->pool.push_back(a);
      return;
    }
    (void)hipEventRecord(b, st);
    c->spans.push_back({a, b, stage});
  }
};


adr_status ensure(Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return ADR_OK;
  if (b.p) {
    hipError_t e = hipFree(b.p);  // synchronises the device: no work still uses it
    if (e != hipSuccess) return hip_fail(e, "hipFree");
    b.p = nullptr;
    b.cap = 0;
  }
  size_t cap = bytes + bytes / 4;
  hipError_t e = hipMalloc(&b.p, cap);
  if (e != hipSuccess) return fail(ADR_E_NOMEM, "hipMalloc(%zu): %s", cap, hipGetErrorString(e));
  b.cap = cap;
  return ADR_OK;
}

void release(Buf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

// Validates a texture; requires_f32 forbids RGBA8; ch3 requires 3 channels.
adr_status check_tex(const adr_texture& t, const char* name, bool allow_rgba8, Tex& out) {
  if (!t.data) return fail(ADR_E_INVALID, "%s: data is NULL", name);
  if (!pow2(t.size) || t.size > 16384) return fail(ADR_E_INVALID, "%s: size %d is not a power of two in [1,16384]", name, t.size);
  int maxl = ilog2(t.size) + 1;
  if (t.levels < 1 || t.levels > maxl) return fail(ADR_E_INVALID, "%s: levels %d outside [1,%d]", name, t.levels, maxl);
  if (t.format == ADR_TEX_RGBA8) {
    if (!allow_rgba8) return fail(ADR_E_INVALID, "%s: RGBA8 not allowed here", name);
    if (t.channels != 4) return fail(ADR_E_INVALID, "%s: RGBA8 needs channels = 4", name);
  } else if (t.format == ADR_TEX_F32) {
    if (t.channels != 3 && t.channels != 1) return fail(ADR_E_INVALID, "%s: F32 channels must be 1 or 3", name);
  } else {
    return fail(ADR_E_INVALID, "%s: unknown format %d", name, t.format);
  }
  out.data = t.data;
  out.size = t.size;
  out.levels = t.levels;
  out.channels = t.channels;
  out.fmt = t.format;
  int off = 0;
  for (int l = 0; l <= kMaxLevels; ++l) {
    out.off[l] = off;
    if (l < t.levels) off += (t.size >> l) * (t.size >> l);
  }
  return ADR_OK;
}

adr_status check_common(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                        const adr_views* views, MeshD& m, ViewsD& v, Tex& kd, Tex& nm, Tex& orm) {
  if (!ctx) return fail(ADR_E_INVALID, "ctx is NULL");
  if (!mesh || !mat || !views) return fail(ADR_E_INVALID, "mesh, material and views are required");
  if (mesh->n_pos < 0 || mesh->n_tri < 0 || mesh->n_uv < 0) return fail(ADR_E_INVALID, "negative mesh size");
  if (mesh->n_tri > 0 && (!mesh->pos || !mesh->tri || !mesh->uv || !mesh->uv_tri || !mesh->adj))
    return fail(ADR_E_INVALID, "mesh arrays pos, tri, uv, uv_tri and adj are required");
  if (mesh->n_tri > 0 && (mesh->n_pos < 1 || mesh->n_uv < 1)) return fail(ADR_E_INVALID, "triangles without vertices");
  if ((int64_t)views->n_views * mesh->n_tri > 0x7fffffffLL || (int64_t)views->n_views * mesh->n_pos > 0x7fffffffLL)
    return fail(ADR_E_INVALID, "views x mesh size exceeds 2^31");
  if (views->n_views < 1 || views->n_views > 4096) return fail(ADR_E_INVALID, "n_views %d outside [1,4096]", views->n_views);
  if (views->width < 1 || views->width > 4096 || views->height < 1 || views->height > 4096)
    return fail(ADR_E_INVALID, "image size %dx%d outside [1,4096]", views->width, views->height);
  if (!views->mvp || !views->eye || !views->light_dir || !views->light_rgb) return fail(ADR_E_INVALID, "views arrays are required");
  if (mat->model != ADR_SHADE_BLINN_PHONG && mat->model != ADR_SHADE_GGX) return fail(ADR_E_INVALID, "unknown shading model %d", mat->model);
  adr_status s;
  if ((s = check_tex(mat->kd, "kd", true, kd)) != ADR_OK) return s;
  if (kd.fmt == ADR_TEX_F32 && kd.channels != 3) return fail(ADR_E_INVALID, "kd: F32 needs 3 channels");
  if ((s = check_tex(mat->normal, "normal", false, nm)) != ADR_OK) return s;
  if (nm.channels != 3) return fail(ADR_E_INVALID, "normal: needs 3 channels");
  if (mat->model == ADR_SHADE_GGX) {
    if ((s = check_tex(mat->orm, "orm", false, orm)) != ADR_OK) return s;
    if (orm.channels != 3) return fail(ADR_E_INVALID, "orm: needs 3 channels");
  } else {
    orm = kd;
  }
  m.pos = mesh->pos;
  m.tri = mesh->tri;
  m.uv = mesh->uv;
  m.uv_tri = mesh->uv_tri;
  m.adj = mesh->adj;
  m.n_pos = mesh->n_pos;
  m.n_tri = mesh->n_tri;
  m.n_uv = mesh->n_uv;
  v.mvp = views->mvp;
  v.eye = views->eye;
  v.light_dir = views->light_dir;
  v.light_rgb = views->light_rgb;
  v.B = views->n_views;
  v.W = views->width;
  v.H = views->height;
  v.ms = 1;
  views_derive(v);
  return ADR_OK;
}

adr_status prepare_scratch(adr_ctx* ctx, const MeshD& m, const ViewsD& v, bool bwd, Scratch& s,
                           int tex_slots = 0, bool det = false) {
  ctx->geom_ok = false;
  size_t B = v.B, V = m.n_pos > 0 ? m.n_pos : 1, T = m.n_tri > 0 ? m.n_tri : 1;
  size_t tiles = (size_t)((v.W + 15) / 16) * ((v.H + 15) / 16) * B;
  adr_status r;
  if ((r = ensure(ctx->snap, B * V * 16)) ||
      (r = ensure(ctx->orient, B * T)) || (r = ensure(ctx->nacc, V * 24)) ||
      (r = ensure(ctx->tacc, V * 24)) || (r = ensure(ctx->nrm, V * 12)) ||
      (r = ensure(ctx->tan, V * 12)) || (r = ensure(ctx->big, B * T * 4)) ||
      (r = ensure(ctx->big_cnt, (B + 1) * 4)) || (r = ensure(ctx->med, B * T * 4)) ||
      (r = ensure(ctx->partial, tiles * 4)) || (r = ensure(ctx->mvpd, B * 128)))
    return r;
  if (bwd) {
    if ((r = ensure(ctx->gcolor, B * v.W * v.H * 12)) || (r = ensure(ctx->dclip, B * V * 16)) ||
        (r = ensure(ctx->dattr, V * 36)))
      return r;
    if (tex_slots > 0 && (r = ensure(ctx->texrec, (size_t)(1 + tex_slots) * B * v.W * v.H * 16))) return r;
  }
  s.image_s = nullptr;
  if (v.ms > 1) {
    if ((r = ensure(ctx->image_s, B * v.W * v.H * 12))) return r;
    s.image_s = (float*)ctx->image_s.p;
  }
  s.det = det;
  if (bwd) {
    if ((r = ensure(ctx->fix_attr, V * 72)) || (r = ensure(ctx->fix_clip, B * V * 32)) ||
        (r = ensure(ctx->fix_pos, V * 24)))
      return r;
    s.fix_attr = (unsigned long long*)ctx->fix_attr.p;
    s.fix_clip = (unsigned long long*)ctx->fix_clip.p;
    s.fix_pos = (unsigned long long*)ctx->fix_pos.p;
  }
  if (det) {
    if ((r = ensure(ctx->fix_n, V * 24)) || (r = ensure(ctx->fix_t, V * 24))) return r;
    s.fix_n = (unsigned long long*)ctx->fix_n.p;
    s.fix_t = (unsigned long long*)ctx->fix_t.p;
    if (bwd) {
      if (tex_slots > 0) {
        const int64_t E = det_entries(v, tex_slots);
        if (E >= (int64_t)0xFFFFFFFF) return fail(ADR_E_INVALID, "deterministic mode: view batch too large (%lld texel terms)", (long long)E);
        const int64_t hw = radix_hist_words(E);
        if ((r = ensure(ctx->det_k0, E * 4)) || (r = ensure(ctx->det_v0, E * 4)) || (r = ensure(ctx->det_k1, E * 4)) ||
            (r = ensure(ctx->det_v1, E * 4)) || (r = ensure(ctx->det_vals, det_vals_bytes(E))) ||
            (r = ensure(ctx->det_hist, hw * 4)) || (r = ensure(ctx->det_tmp, scan_tmp_words(hw) * 4 + 4)) ||
            (r = ensure(ctx->det_part, det_part_bytes(E))))
          return r;
        s.det_k0 = (uint32_t*)ctx->det_k0.p;
        s.det_v0 = (uint32_t*)ctx->det_v0.p;
        s.det_k1 = (uint32_t*)ctx->det_k1.p;
        s.det_v1 = (uint32_t*)ctx->det_v1.p;
        det_carve(ctx->det_vals.p, E, s);
        s.det_hist = (uint32_t*)ctx->det_hist.p;
        s.det_tmp = (uint32_t*)ctx->det_tmp.p;
        s.det_part = (float4*)ctx->det_part.p;
      }
    }
  }
  s.snap = (int*)ctx->snap.p;
  s.mvpd = (double*)ctx->mvpd.p;
  s.orient = (int8_t*)ctx->orient.p;
  s.nacc = (double*)ctx->nacc.p;
  s.tacc = (double*)ctx->tacc.p;
  s.nrm = (float*)ctx->nrm.p;
  s.tan = (float*)ctx->tan.p;
  s.big = (uint32_t*)ctx->big.p;
  s.big_cnt = (uint32_t*)ctx->big_cnt.p;
  s.med = (uint32_t*)ctx->med.p;
  s.partial = (float*)ctx->partial.p;
  s.tiny_bbox = ctx->tiny_bbox;
  s.med_bbox = ctx->med_bbox;
  s.gcolor = (float*)ctx->gcolor.p;
  s.dclip = (float*)ctx->dclip.p;
  s.dattr = (float*)ctx->dattr.p;
  s.texrec = (float4*)ctx->texrec.p;
  s.n_partial = (int)tiles;
  return ADR_OK;
}

}  // namespace

#define HIPCHK(x, where)                         \
  do {                                           \
    hipError_t e_ = (x);                         \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

#define TIMED(stage, x, where)                   \
  do {                                           \
    StageTimer t_(ctx, stage, st);               \
    HIPCHK(x, where);                            \
  } while (0)

// Multisampling factor from the flags (1, 2 or 4 samples per pixel axis);
// switches the views to the sample grid.  0 on a bad combination.
static int apply_msaa(int32_t flags, ViewsD& v) {
  const bool m2 = flags & ADR_MSAA_2X2, m4 = flags & ADR_MSAA_4X4;
  if (m2 && m4) return 0;
  const int ms = m4 ? 4 : (m2 ? 2 : 1);
  v.ms = ms;
  v.W *= ms;
  v.H *= ms;
  views_derive(v);
  return ms;
}

// Validation shared by the forward entry points (no device work).
static adr_status check_fwd(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat, const adr_views* views,
                            const float* ref_image, int32_t loss_kind, const adr_fwd_out* out, int32_t flags,
                            MeshD& m, ViewsD& v, Tex& kd, Tex& nm, Tex& orm) {
  adr_status r = check_common(ctx, mesh, mat, views, m, v, kd, nm, orm);
  if (r != ADR_OK) return r;
  if (!out || !out->vis || !out->color) return fail(ADR_E_INVALID, "out->vis and out->color are required");
  if (ref_image) {
    if (loss_kind < ADR_LOSS_L1 || loss_kind > ADR_LOSS_L2_TONEMAP) return fail(ADR_E_INVALID, "unknown loss kind %d", loss_kind);
    if (!out->dimage || !out->loss) return fail(ADR_E_INVALID, "out->dimage and out->loss are required with a reference image");
  }
  if (flags & ~(ADR_FWD_BUILD_MIPS | ADR_FWD_NO_AA | ADR_DETERMINISTIC | ADR_INDEPENDENT_MIPS | ADR_MSAA_2X2 |
                ADR_MSAA_4X4 | ADR_BWD_DEFER_MIP_ADJOINT))
    return fail(ADR_E_INVALID, "unknown flags 0x%x", flags);
  if ((flags & ADR_FWD_BUILD_MIPS) && (flags & ADR_INDEPENDENT_MIPS))
    return fail(ADR_E_INVALID, "independent mip levels are not rebuilt from level 0");
  if (!apply_msaa(flags, v) || v.W > 16384 || v.H > 16384)
    return fail(ADR_E_INVALID, "multisampling: one factor, at most 16384 samples per axis");
  return ADR_OK;
}

#define STAGE(stage, x, where)      \
  do {                              \
    if (timed) {                    \
      TIMED(stage, x, where);       \
    } else {                        \
      HIPCHK(x, where);             \
    }                               \
  } while (0)

// The forward's launch sequence on the scratch s; `timed` brackets the
// stages with events when the context profiles them.
static adr_status fwd_launches(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat, const MeshD& m,
                               const ViewsD& v, const Tex& kd, const Tex& nm, const Tex& orm, const float* ref_image,
                               int32_t loss_kind, const adr_fwd_out* out, int32_t flags, hipStream_t st, Scratch& s,
                               bool timed) {
  if (flags & ADR_FWD_BUILD_MIPS) {
    const Tex* maps[3] = {&kd, &nm, &orm};
    int nmaps = mat->model == ADR_SHADE_GGX ? 3 : 2;
    MipSet ms{};
    for (int k = 0; k < nmaps; ++k)
      if (maps[k]->fmt == ADR_TEX_F32 && maps[k]->levels > 1) ms.t[ms.n++] = *maps[k];
    STAGE(10, launch_mip_build_set(ms, st), "mip build");
  }
  int64_t npx = (int64_t)v.B * v.W * v.H;
  const bool own_frame = !(mesh->nrm && mesh->tan);
  if (!own_frame) {
    s.nrm = const_cast<float*>(mesh->nrm);  // read only on this path
    s.tan = const_cast<float*>(mesh->tan);
  } else {
    STAGE(0, launch_vertex_frame(m, s, st), "vertex frame");
  }
  STAGE(1, launch_xform(m, v, s, st), "transform");
  STAGE(12, launch_clear_vis(out->vis, out->coverage, npx, s.big_cnt, v.B, st), "clear");
  STAGE(2, launch_raster(m, v, s, out->vis, out->coverage, st), "raster");
  STAGE(3, launch_shade_fwd(m, v, mat->model, kd, nm, orm, s, out->vis, out->color, out->tri_id, st), "shade");
  STAGE(4, launch_aa_loss_fwd(m, v, s, out->vis, out->color, ref_image, loss_kind,
                            (flags & ADR_FWD_NO_AA) ? 1 : 0, out->image, out->dimage, out->loss, st, out->aa),
        "antialias/loss");
  if (ref_image) STAGE(18, launch_loss_reduce(v, ref_image, s, out->loss, st), "loss reduction");
  return ADR_OK;
}

// ---- the no-allocation forward's scratch ----
//
// One static device array: every GPU the library runs on holds its own copy
// (a module global) until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host it is a stand-in, not a
// device address): adr_ctx_create looks up each device's address once, with
// that device current, and the entry point carves its buffers from it.
static __device__ __align__(256) unsigned char scratch[ADR_NOALLOC_SCRATCH_BYTES];
static std::mutex g_noalloc_mu;
static std::unordered_map<int, unsigned char*> g_noalloc_addr;

// Address of the current device's copy (device `device` must be current).
static adr_status noalloc_address(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc_addr.find(device);
  if (it == g_noalloc_addr.end()) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(no-allocation scratch)");
    it = g_noalloc_addr.emplace(device, static_cast<unsigned char*>(p)).first;
  }
  *out = it->second;
  return ADR_OK;
}

// The forward's scratch carved from the context's device copy of the array
// (256-byte aligned pieces, the same sizes prepare_scratch allocates);
// returns the bytes used, and fills s when it is given.  Nothing here starts
// at zero: the kernels clear what they accumulate into (the frame
// accumulators, the triangle counters).
static size_t noalloc_carve(adr_ctx* ctx, const MeshD& m, const ViewsD& v, bool det, Scratch* s) {
  const size_t B = v.B, V = m.n_pos > 0 ? m.n_pos : 1, T = m.n_tri > 0 ? m.n_tri : 1;
  const size_t tiles = (size_t)((v.W + 15) / 16) * ((v.H + 15) / 16) * B;
  size_t off = 0;
  auto take = [&](size_t bytes) -> unsigned char* {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return s ? ctx->noalloc + o : nullptr;
  };
  unsigned char* snap = take(B * V * 16);
  unsigned char* orient = take(B * T);
  unsigned char* nacc = take(V * 24);
  unsigned char* tacc = take(V * 24);
  unsigned char* nrm = take(V * 12);
  unsigned char* tan = take(V * 12);
  unsigned char* big = take(B * T * 4);
  unsigned char* big_cnt = take((B + 1) * 4);
  unsigned char* med = take(B * T * 4);
  unsigned char* partial = take(tiles * 4);
  unsigned char* mvpd = take(B * 128);
  unsigned char* image_s = v.ms > 1 ? take(B * v.W * v.H * 12) : nullptr;
  unsigned char* fix_n = det ? take(V * 24) : nullptr;
  unsigned char* fix_t = det ? take(V * 24) : nullptr;
  if (s) {
    *s = Scratch{};
    s->snap = (int*)snap;
    s->orient = (int8_t*)orient;
    s->nacc = (double*)nacc;
    s->tacc = (double*)tacc;
    s->nrm = (float*)nrm;
    s->tan = (float*)tan;
    s->big = (uint32_t*)big;
    s->big_cnt = (uint32_t*)big_cnt;
    s->med = (uint32_t*)med;
    s->partial = (float*)partial;
    s->mvpd = (double*)mvpd;
    s->n_partial = (int)tiles;
    s->image_s = (float*)image_s;
    s->det = det;
    s->fix_n = (unsigned long long*)fix_n;
    s->fix_t = (unsigned long long*)fix_t;
    s->tiny_bbox = ctx->tiny_bbox;
    s->med_bbox = ctx->med_bbox;
  }
  return off;
}

extern "C" {

const char* adr_last_error(void) { return g_err; }

adr_status adr_ctx_create(int32_t device, uint64_t hbm_budget_bytes, adr_ctx** out) {
  if (!out) return fail(ADR_E_INVALID, "out is NULL");
  *out = nullptr;
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n), "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(ADR_E_INVALID, "device %d outside [0,%d)", device, n);
  HIPCHK(hipSetDevice(device), "hipSetDevice");
  adr_ctx* c = new (std::nothrow) adr_ctx();
  if (!c) return fail(ADR_E_NOMEM, "context allocation");
  c->device = device;
  if (hbm_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
    const uint64_t reserve = 4ull << 30;
    hbm_budget_bytes = fr > reserve ? fr - reserve : fr / 2;
  }
  c->budget = hbm_budget_bytes;
  // this device's copy of the no-allocation scratch array (device current)
  adr_status rs = noalloc_address(device, &c->noalloc);
  if (rs != ADR_OK) {
    delete c;
    return rs;
  }
  *out = c;
  return ADR_OK;
}

adr_status adr_ctx_destroy(adr_ctx* ctx) {
  if (!ctx) return fail(ADR_E_INVALID, "ctx is NULL");
  (void)hipSetDevice(ctx->device);
  adr::jobs_destroy(ctx->jobs);
  ctx->jobs = nullptr;
  (void)hipDeviceSynchronize();
  Buf* bufs[] = {&ctx->fix_n, &ctx->fix_t, &ctx->fix_attr, &ctx->fix_clip, &ctx->fix_pos, &ctx->det_k0,
                 &ctx->det_v0, &ctx->det_k1, &ctx->det_v1, &ctx->det_hist, &ctx->det_tmp, &ctx->det_vals,
                 &ctx->det_part, &ctx->lap_r, &ctx->lap_part, &ctx->texrec, &ctx->image_s, &ctx->snap, &ctx->orient, &ctx->nacc, &ctx->tacc, &ctx->nrm, &ctx->tan,
                 &ctx->big, &ctx->big_cnt, &ctx->med, &ctx->oit_g, &ctx->oit_a, &ctx->partial, &ctx->gcolor, &ctx->dclip, &ctx->dattr,
                 &ctx->mvpd};
  for (Buf* b : bufs) release(*b);
  for (const Span& sp : ctx->spans) {
    (void)hipEventDestroy(sp.a);
    (void)hipEventDestroy(sp.b);
  }
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  delete ctx;
  return ADR_OK;
}

adr_status adr_render_fwd(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                          const adr_views* views, const float* ref_image, int32_t loss_kind,
                          const adr_fwd_out* out, int32_t flags, adr_stream stream) {
  MeshD m;
  ViewsD v;
  Tex kd, nm, orm;
  adr_status r = check_fwd(ctx, mesh, mat, views, ref_image, loss_kind, out, flags, m, v, kd, nm, orm);
  if (r != ADR_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  Scratch s;
  if ((r = prepare_scratch(ctx, m, v, false, s, 0, (flags & ADR_DETERMINISTIC) != 0)) != ADR_OK) return r;
  v.mvpd = s.mvpd;
  const bool own_frame = !(mesh->nrm && mesh->tan);
  if ((r = fwd_launches(ctx, mesh, mat, m, v, kd, nm, orm, ref_image, loss_kind, out, flags, st, s, true)) != ADR_OK)
    return r;
  // the frame, snapped vertices and orientations now in the scratch (the
  // raster writes every triangle's orientation) serve a backward that follows
  if (own_frame) {
    ctx->geom = geom_key(m, v, views->mvp, out->vis, (flags & ADR_DETERMINISTIC) != 0, st);
    ctx->geom_ok = true;
  }
  return ADR_OK;
}

adr_status adr_render_fwd_noalloc(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                                  const adr_views* views, const float* ref_image, int32_t loss_kind,
                                  const adr_fwd_out* out, int32_t flags, adr_stream stream) {
  MeshD m;
  ViewsD v;
  Tex kd, nm, orm;
  adr_status r = check_fwd(ctx, mesh, mat, views, ref_image, loss_kind, out, flags, m, v, kd, nm, orm);
  if (r != ADR_OK) return r;
  if (!ctx->noalloc) return fail(ADR_E_HIP, "no-allocation scratch of device %d was not set up", ctx->device);
  Scratch s;
  const size_t need = noalloc_carve(ctx, m, v, (flags & ADR_DETERMINISTIC) != 0, nullptr);
  if (need > (size_t)ADR_NOALLOC_SCRATCH_BYTES)
    return fail(ADR_E_INVALID,
                "adr_render_fwd_noalloc: %d views x %d triangles / %d vertices at %dx%d samples need %zu bytes of "
                "scratch; the no-allocation forward holds at most %llu",
                v.B, m.n_tri, m.n_pos, v.W, v.H, need, (unsigned long long)ADR_NOALLOC_SCRATCH_BYTES);
  noalloc_carve(ctx, m, v, (flags & ADR_DETERMINISTIC) != 0, &s);
  v.mvpd = s.mvpd;
  // the context's own scratch no longer holds this forward's geometry
  ctx->geom_ok = false;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  return fwd_launches(ctx, mesh, mat, m, v, kd, nm, orm, ref_image, loss_kind, out, flags, st, s, false);
}

adr_status adr_render_bwd(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                          const adr_views* views, const adr_fwd_out* saved, const float* dloss,
                          const adr_grads* grads, int32_t flags, adr_stream stream) {
  MeshD m;
  ViewsD v;
  Tex kd, nm, orm;
  adr_status r = check_common(ctx, mesh, mat, views, m, v, kd, nm, orm);
  if (r != ADR_OK) return r;
  if (!saved || !saved->vis || !saved->color || !saved->dimage)
    return fail(ADR_E_INVALID, "saved->vis, color and dimage are required");
  if (!grads) return fail(ADR_E_INVALID, "grads is NULL");
  if (grads->kd && kd.fmt != ADR_TEX_F32) return fail(ADR_E_INVALID, "kd gradient needs an F32 kd map");
  if (grads->orm && mat->model != ADR_SHADE_GGX) return fail(ADR_E_INVALID, "orm gradient needs GGX");
  if (flags & ~(ADR_FWD_BUILD_MIPS | ADR_FWD_NO_AA | ADR_DETERMINISTIC | ADR_INDEPENDENT_MIPS | ADR_MSAA_2X2 |
                ADR_MSAA_4X4 | ADR_BWD_DEFER_MIP_ADJOINT))
    return fail(ADR_E_INVALID, "unknown flags 0x%x", flags);
  if (!apply_msaa(flags, v) || v.W > 16384 || v.H > 16384)
    return fail(ADR_E_INVALID, "multisampling: one factor, at most 16384 samples per axis");
  const bool det = (flags & ADR_DETERMINISTIC) != 0;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  const bool reuse = ctx->geom_ok && ctx->geom.same(geom_key(m, v, views->mvp, saved->vis, det, st));
  Scratch s;
  if ((r = prepare_scratch(ctx, m, v, true, s, tex_slots(mat->model, grads->kd, grads->normal, grads->orm), det)) !=
      ADR_OK)
    return r;
  v.mvpd = s.mvpd;
  const int64_t n_clip = 4 * (int64_t)v.B * (m.n_pos > 0 ? m.n_pos : 1), n_attr = 9 * (int64_t)(m.n_pos > 0 ? m.n_pos : 1);
  if (!reuse) {
    TIMED(0, launch_vertex_frame(m, s, st), "vertex frame");
    TIMED(1, launch_xform(m, v, s, st), "transform");
    TIMED(1, launch_orient(m, v, s, st), "orientation");
  }
  {
    FillSet f{};
    f.add(s.fix_clip, n_clip);
    f.add(s.fix_attr, n_attr);
    f.add(s.fix_pos, 3 * (int64_t)(m.n_pos > 0 ? m.n_pos : 1));
    TIMED(12, launch_fill_multi(f, st), "clear");
  }
  TIMED(5, launch_aa_bwd(m, v, s, saved->vis, saved->color, saved->dimage, dloss,
                       (flags & ADR_FWD_NO_AA) ? 1 : 0, st, saved->aa),
         "antialias adjoint");
  TIMED(6, launch_shade_bwd(m, v, mat->model, kd, nm, orm, grads->kd, grads->normal, grads->orm, s,
                            saved->vis, st),
        "shading adjoint");
  TIMED(12, launch_fix_to_f32(s.fix_clip, s.dclip, n_clip, det, st, s.fix_attr, s.dattr, n_attr),
        "accumulator conversion");
  TIMED(11, launch_tex_bwd(v, mat->model, kd, nm, orm, grads->kd, grads->normal, grads->orm, s, st),
        "texel adjoint");
  {
    MipSet ms{};
    const Tex* maps[3] = {&kd, &nm, &orm};
    float* gs[3] = {grads->kd, grads->normal, grads->orm};
    for (int k = 0; k < 3; ++k)
      if (gs[k] && maps[k]->levels > 1) {
        ms.t[ms.n] = *maps[k];
        ms.g[ms.n++] = gs[k];
      }
    if (!(flags & (ADR_INDEPENDENT_MIPS | ADR_BWD_DEFER_MIP_ADJOINT)))
      TIMED(7, launch_mip_adjoint_set(ms, st), "mip adjoint");
  }
  if (m.n_pos > 0 && (grads->pos || grads->vnormal))
    TIMED(8, launch_mesh_bwd(m, v, s, grads->pos, grads->vnormal, st, true), "mesh adjoint");
  return ADR_OK;
}

// ---- depth peeling (order-independent transparency) ----

static adr_status check_alpha(const adr_material* mat, Tex& al, bool& has) {
  has = mat->alpha.data != nullptr;
  al = Tex{};
  if (!has) return ADR_OK;
  adr_status r = check_tex(mat->alpha, "alpha", false, al);
  if (r != ADR_OK) return r;
  if (al.channels != 1) return fail(ADR_E_INVALID, "alpha: needs 1 channel");
  return ADR_OK;
}

static adr_status check_oit(const adr_oit_out* o, int32_t flags, bool fwd) {
  if (!o) return fail(ADR_E_INVALID, "out is NULL");
  if (o->n_layers < 1 || o->n_layers > 16) return fail(ADR_E_INVALID, "n_layers %d outside [1,16]", o->n_layers);
  if (!o->vis || !o->color || !o->alpha || !o->blend || !o->comp)
    return fail(ADR_E_INVALID, "out->vis, color, alpha, blend and comp are required");
  if (flags & (ADR_MSAA_2X2 | ADR_MSAA_4X4 | ADR_DETERMINISTIC))
    return fail(ADR_E_UNIMPL, "depth peeling with multisampling or the deterministic mode is not implemented");
  if (flags & ~(ADR_FWD_BUILD_MIPS | ADR_FWD_NO_AA | ADR_INDEPENDENT_MIPS | ADR_BWD_DEFER_MIP_ADJOINT))
    return fail(ADR_E_INVALID, "unknown flags 0x%x", flags);
  if (fwd && (flags & ADR_FWD_BUILD_MIPS) && (flags & ADR_INDEPENDENT_MIPS))
    return fail(ADR_E_INVALID, "independent mip levels are not rebuilt from level 0");
  return ADR_OK;
}

adr_status adr_render_oit_fwd(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                              const adr_views* views, const float* ref_image, int32_t loss_kind,
                              const adr_oit_out* out, int32_t flags, adr_stream stream) {
  MeshD m;
  ViewsD v;
  Tex kd, nm, orm, al;
  bool has_al;
  adr_status r = check_common(ctx, mesh, mat, views, m, v, kd, nm, orm);
  if (r != ADR_OK) return r;
  if ((r = check_alpha(mat, al, has_al)) != ADR_OK || (r = check_oit(out, flags, true)) != ADR_OK) return r;
  if (ref_image) {
    if (loss_kind < ADR_LOSS_L1 || loss_kind > ADR_LOSS_L2_TONEMAP) return fail(ADR_E_INVALID, "unknown loss kind %d", loss_kind);
    if (!out->dimage || !out->loss) return fail(ADR_E_INVALID, "out->dimage and out->loss are required with a reference image");
  }
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  Scratch s;
  if ((r = prepare_scratch(ctx, m, v, false, s)) != ADR_OK) return r;
  v.mvpd = s.mvpd;
  if (flags & ADR_FWD_BUILD_MIPS) {
    const Tex* maps[4] = {&kd, &nm, &orm, &al};
    MipSet ms{};
    for (int k = 0; k < 4; ++k) {
      if (k == 2 && mat->model != ADR_SHADE_GGX) continue;
      if (k == 3 && !has_al) continue;
      if (maps[k]->fmt == ADR_TEX_F32 && maps[k]->levels > 1) ms.t[ms.n++] = *maps[k];
    }
    TIMED(10, launch_mip_build_set(ms, st), "mip build");
  }
  const bool own_frame = !(mesh->nrm && mesh->tan);
  if (!own_frame) {
    s.nrm = const_cast<float*>(mesh->nrm);  // read only on this path
    s.tan = const_cast<float*>(mesh->tan);
  } else {
    TIMED(0, launch_vertex_frame(m, s, st), "vertex frame");
  }
  TIMED(1, launch_xform(m, v, s, st), "transform");
  if (own_frame) {  // orientations: every peeling pass's raster writes them
    ctx->geom = geom_key(m, v, views->mvp, out->vis, false, st);
    ctx->geom_ok = true;
  }
  const int64_t npx = (int64_t)v.B * v.W * v.H;
  const int L = out->n_layers;
  const int no_aa = (flags & ADR_FWD_NO_AA) ? 1 : 0;
  // front to back: peel, then shade each layer
  for (int k = 0; k < L; ++k) {
    uint64_t* vk = out->vis + k * npx;
    TIMED(12, launch_clear_vis(vk, nullptr, npx, s.big_cnt, v.B, st), "clear");
    TIMED(2, launch_raster(m, v, s, vk, nullptr, st, k > 0 ? out->vis + (k - 1) * npx : nullptr), "raster");
    TIMED(3, launch_shade_fwd(m, v, mat->model, kd, nm, orm, s, vk, out->color + 3 * k * npx, nullptr, st,
                              has_al ? &al : nullptr, out->alpha + k * npx),
          "shade");
  }
  // back to front: blend over what lies behind, antialias the layer
  for (int k = L - 1; k >= 0; --k) {
    const uint64_t* vk = out->vis + k * npx;
    const float* behind = k + 1 < L ? out->comp + 3 * (k + 1) * npx : nullptr;
    float* bk = out->blend + 3 * k * npx;
    TIMED(15, launch_oit_blend(npx, vk, out->color + 3 * k * npx, out->alpha + k * npx, behind, bk, st), "blend");
    TIMED(4, launch_aa_loss_fwd(m, v, s, vk, bk, k == 0 ? ref_image : nullptr, loss_kind, no_aa,
                                out->comp + 3 * k * npx, k == 0 ? out->dimage : nullptr, k == 0 ? out->loss : nullptr,
                                st, out->aa ? out->aa + 8 * k * npx : nullptr),
          "antialias/loss");
    if (k == 0 && ref_image) TIMED(18, launch_loss_reduce(v, ref_image, s, out->loss, st), "loss reduction");
  }
  return ADR_OK;
}

adr_status adr_render_oit_bwd(adr_ctx* ctx, const adr_mesh* mesh, const adr_material* mat,
                              const adr_views* views, const adr_oit_out* saved, const float* dloss,
                              const adr_grads* grads, int32_t flags, adr_stream stream) {
  MeshD m;
  ViewsD v;
  Tex kd, nm, orm, al;
  bool has_al;
  adr_status r = check_common(ctx, mesh, mat, views, m, v, kd, nm, orm);
  if (r != ADR_OK) return r;
  if ((r = check_alpha(mat, al, has_al)) != ADR_OK || (r = check_oit(saved, flags, false)) != ADR_OK) return r;
  if (!saved->dimage) return fail(ADR_E_INVALID, "saved->dimage is required");
  if (!grads) return fail(ADR_E_INVALID, "grads is NULL");
  if (grads->kd && kd.fmt != ADR_TEX_F32) return fail(ADR_E_INVALID, "kd gradient needs an F32 kd map");
  if (grads->orm && mat->model != ADR_SHADE_GGX) return fail(ADR_E_INVALID, "orm gradient needs GGX");
  if (grads->alpha && !has_al) return fail(ADR_E_INVALID, "alpha gradient needs an alpha map");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  float* gal = has_al ? grads->alpha : nullptr;
  const bool reuse = ctx->geom_ok && ctx->geom.same(geom_key(m, v, views->mvp, saved->vis, false, st));
  Scratch s;
  if ((r = prepare_scratch(ctx, m, v, true, s, tex_slots(mat->model, grads->kd, grads->normal, grads->orm, gal))) !=
      ADR_OK)
    return r;
  v.mvpd = s.mvpd;
  const int64_t npx = (int64_t)v.B * v.W * v.H;
  if ((r = ensure(ctx->oit_g, npx * 12)) || (r = ensure(ctx->oit_a, npx * 4))) return r;
  float* gbehind = (float*)ctx->oit_g.p;
  float* galpha = (float*)ctx->oit_a.p;
  const int64_t n_clip = 4 * (int64_t)v.B * (m.n_pos > 0 ? m.n_pos : 1), n_attr = 9 * (int64_t)(m.n_pos > 0 ? m.n_pos : 1);
  if (!reuse) {
    TIMED(0, launch_vertex_frame(m, s, st), "vertex frame");
    TIMED(1, launch_xform(m, v, s, st), "transform");
    TIMED(1, launch_orient(m, v, s, st), "orientation");
  }
  {
    FillSet f{};
    f.add(s.fix_clip, n_clip);
    f.add(s.fix_attr, n_attr);
    f.add(s.fix_pos, 3 * (int64_t)(m.n_pos > 0 ? m.n_pos : 1));
    TIMED(12, launch_fill_multi(f, st), "clear");
  }
  const int L = saved->n_layers;
  const int no_aa = (flags & ADR_FWD_NO_AA) ? 1 : 0;
  // front to back: dL/dC_k -> dL/dB_k (antialiasing adjoint) -> dL/dc_k,
  // dL/da_k and dL/dC_{k+1} (blend adjoint) -> shading and texel adjoints
  for (int k = 0; k < L; ++k) {
    const uint64_t* vk = saved->vis + k * npx;
    const float* ck = saved->color + 3 * k * npx;
    const float* ak = saved->alpha + k * npx;
    const float* behind = k + 1 < L ? saved->comp + 3 * (k + 1) * npx : nullptr;
    TIMED(5, launch_aa_bwd(m, v, s, vk, saved->blend + 3 * k * npx, k == 0 ? saved->dimage : gbehind,
                           k == 0 ? dloss : nullptr, no_aa, st, saved->aa ? saved->aa + 8 * k * npx : nullptr),
          "antialias adjoint");
    TIMED(15, launch_oit_blend_bwd(npx, vk, ck, ak, behind, s.gcolor, galpha, k + 1 < L ? gbehind : nullptr, st),
          "blend adjoint");
    TIMED(6, launch_shade_bwd(m, v, mat->model, kd, nm, orm, grads->kd, grads->normal, grads->orm, s, vk, st,
                              has_al ? &al : nullptr, gal, has_al ? galpha : nullptr),
          "shading adjoint");
    TIMED(11, launch_tex_bwd(v, mat->model, kd, nm, orm, grads->kd, grads->normal, grads->orm, s, st,
                             has_al ? &al : nullptr, gal),
          "texel adjoint");
  }
  TIMED(12, launch_fix_to_f32(s.fix_clip, s.dclip, n_clip, false, st, s.fix_attr, s.dattr, n_attr),
        "accumulator conversion");
  {
    MipSet ms{};
    const Tex* maps[4] = {&kd, &nm, &orm, &al};
    float* gs[4] = {grads->kd, grads->normal, grads->orm, gal};
    for (int k = 0; k < 4; ++k)
      if (gs[k] && maps[k]->levels > 1) {
        ms.t[ms.n] = *maps[k];
        ms.g[ms.n++] = gs[k];
      }
    if (!(flags & (ADR_INDEPENDENT_MIPS | ADR_BWD_DEFER_MIP_ADJOINT)))
      TIMED(7, launch_mip_adjoint_set(ms, st), "mip adjoint");
  }
  if (m.n_pos > 0 && (grads->pos || grads->vnormal))
    TIMED(8, launch_mesh_bwd(m, v, s, grads->pos, grads->vnormal, st, true), "mesh adjoint");
  return ADR_OK;
}

static adr_status check_tess(adr_ctx* ctx, const adr_mesh* base, const adr_tess* tess,
                             const adr_texture* disp, MeshD& m, TessD& ts, Tex& d) {
  if (!ctx || !base || !tess || !disp) return fail(ADR_E_INVALID, "ctx, base, tess and disp are required");
  if (base->n_pos < 1 || base->n_tri < 1 || !base->pos || !base->tri)
    return fail(ADR_E_INVALID, "base mesh needs positions and triangles");
  if (tess->n_vert < 0 || (tess->n_vert > 0 && (!tess->vidx || !tess->w || !tess->duv)))
    return fail(ADR_E_INVALID, "tessellation table arrays are required");
  adr_status r = check_tex(*disp, "disp", false, d);
  if (r != ADR_OK) return r;
  if (d.channels != 1) return fail(ADR_E_INVALID, "disp: needs 1 channel");
  m.pos = base->pos;
  m.tri = base->tri;
  m.uv = base->uv;
  m.uv_tri = base->uv_tri;
  m.adj = base->adj;
  m.n_pos = base->n_pos;
  m.n_tri = base->n_tri;
  m.n_uv = base->n_uv;
  // the frame stage only needs uv for tangents; the base mesh is given them
  if (!m.uv || !m.uv_tri) return fail(ADR_E_INVALID, "base mesh needs uv and uv_tri");
  ts.vidx = tess->vidx;
  ts.w = tess->w;
  ts.duv = tess->duv;
  ts.n = tess->n_vert;
  return ADR_OK;
}

adr_status adr_tess_fwd(adr_ctx* ctx, const adr_mesh* base, const adr_tess* tess,
                        const adr_texture* disp, float* pos_out, adr_stream stream) {
  if (ctx) ctx->geom_ok = false;
  MeshD m;
  TessD ts;
  Tex d;
  adr_status r = check_tess(ctx, base, tess, disp, m, ts, d);
  if (r != ADR_OK) return r;
  if (ts.n > 0 && !pos_out) return fail(ADR_E_INVALID, "pos_out is required");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  ViewsD v{};
  v.B = 1;
  v.W = v.H = 1;
  Scratch s;
  if ((r = prepare_scratch(ctx, m, v, false, s)) != ADR_OK) return r;
  TIMED(0, launch_vertex_frame(m, s, st), "vertex frame");
  TIMED(0, launch_tess_fwd(m, ts, s.nacc, d, pos_out, st), "tessellation");
  return ADR_OK;
}

adr_status adr_tess_bwd(adr_ctx* ctx, const adr_mesh* base, const adr_tess* tess,
                        const adr_texture* disp, float* g_pos_out, float* g_base_pos,
                        float* g_disp, adr_stream stream) {
  if (ctx) ctx->geom_ok = false;
  MeshD m;
  TessD ts;
  Tex d;
  adr_status r = check_tess(ctx, base, tess, disp, m, ts, d);
  if (r != ADR_OK) return r;
  if ((ts.n > 0 && !g_pos_out) || !g_base_pos) return fail(ADR_E_INVALID, "g_pos_out and g_base_pos are required");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  ViewsD v{};
  v.B = 1;
  v.W = v.H = 1;
  Scratch s;
  if ((r = prepare_scratch(ctx, m, v, true, s)) != ADR_OK) return r;
  TIMED(8, launch_vertex_frame(m, s, st), "vertex frame");
  TIMED(8, launch_fill_f32(s.dattr, 9 * (int64_t)m.n_pos, 0.f, st), "clear");
  TIMED(8, launch_tess_bwd(m, ts, s.nacc, d, g_pos_out, g_base_pos, s.dattr, g_disp, st), "tessellation adjoint");
  v.B = 0;  // no clip-space gradients: only the normal adjoint is folded into positions
  TIMED(8, launch_mesh_bwd(m, v, s, g_base_pos, nullptr, st), "mesh adjoint");
  return ADR_OK;
}

adr_status adr_mesh_frame(adr_ctx* ctx, const adr_mesh* mesh, float* nrm_out, float* tan_out,
                          adr_stream stream) {
  if (ctx) ctx->geom_ok = false;
  if (!ctx || !mesh) return fail(ADR_E_INVALID, "ctx and mesh are required");
  if (mesh->n_pos < 0 || mesh->n_tri < 0 || mesh->n_uv < 0) return fail(ADR_E_INVALID, "negative mesh size");
  if (mesh->n_pos > 0 && (!nrm_out || !tan_out)) return fail(ADR_E_INVALID, "nrm_out and tan_out are required");
  if (mesh->n_tri > 0 && (!mesh->pos || !mesh->tri || !mesh->uv || !mesh->uv_tri))
    return fail(ADR_E_INVALID, "mesh needs pos, tri, uv and uv_tri");
  MeshD m{mesh->pos, mesh->tri, mesh->uv, mesh->uv_tri, mesh->adj, mesh->n_pos, mesh->n_tri, mesh->n_uv};
  if (m.n_pos == 0) return ADR_OK;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  ViewsD v{};
  v.B = 1;
  v.W = v.H = 1;
  Scratch s;
  adr_status r;
  if ((r = prepare_scratch(ctx, m, v, false, s)) != ADR_OK) return r;
  s.nrm = nrm_out;
  s.tan = tan_out;
  TIMED(0, launch_vertex_frame(m, s, st), "vertex frame");
  return ADR_OK;
}

adr_status adr_laplacian(adr_ctx* ctx, const adr_one_ring* ring, const float* pos, const float* delta_ref,
                         float lambda, float* delta_out, float* loss, float* g_pos, adr_stream stream) {
  if (ctx) ctx->geom_ok = false;
  if (!ctx || !ring) return fail(ADR_E_INVALID, "ctx and ring are required");
  const int n = ring->n_pos;
  if (n < 0) return fail(ADR_E_INVALID, "negative vertex count");
  if (n > 0 && (!ring->offs || !ring->nbr || !pos)) return fail(ADR_E_INVALID, "ring offs/nbr and pos are required");
  if (!std::isfinite(lambda)) return fail(ADR_E_INVALID, "lambda is not finite");
  if (n == 0) return ADR_OK;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  adr_status r;
  if ((r = ensure(ctx->lap_r, (size_t)n * 12)) || (r = ensure(ctx->lap_part, (size_t)((n + 255) / 256) * 8)))
    return r;
  TIMED(8, launch_laplacian(n, pos, ring->offs, ring->nbr, delta_ref, lambda, (float*)ctx->lap_r.p,
                            (double*)ctx->lap_part.p, delta_out, loss, g_pos, st),
        "laplacian");
  return ADR_OK;
}

adr_status adr_image_downsample(adr_ctx* ctx, const float* in, int32_t n_views, int32_t height, int32_t width,
                                int32_t k, float* out, adr_stream stream) {
  if (ctx) ctx->geom_ok = false;
  if (!ctx || !in || !out) return fail(ADR_E_INVALID, "ctx, in and out are required");
  if (n_views < 1 || height < 1 || width < 1 || k < 1 || k > 64 || (int64_t)height * k > 65536 ||
      (int64_t)width * k > 65536)
    return fail(ADR_E_INVALID, "downsample: bad sizes");
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  TIMED(12, launch_downsample(in, n_views, height, width, k, out, st), "downsample");
  return ADR_OK;
}

static adr_status check_skin(adr_ctx* ctx, int32_t n_pos, int32_t n_bones) {
  if (!ctx) return fail(ADR_E_INVALID, "ctx is NULL");
  if (n_pos < 0) return fail(ADR_E_INVALID, "skin: negative vertex count");
  if (n_bones < 1 || n_bones > 4096) return fail(ADR_E_INVALID, "skin: n_bones must be in 1..4096");
  return ADR_OK;
}

adr_status adr_skin_fwd(adr_ctx* ctx, const float* pos, const float* weights, const float* bones, int32_t n_pos,
                        int32_t n_bones, float* pos_out, float* blend_out, adr_stream stream) {
  if (ctx) ctx->geom_ok = false;
  adr_status r = check_skin(ctx, n_pos, n_bones);
  if (r != ADR_OK) return r;
  if (n_pos == 0) return ADR_OK;
  if (!pos || !weights || !bones || !pos_out) return fail(ADR_E_INVALID, "skin: pos, weights, bones and pos_out are required");
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  TIMED(13, launch_skin_fwd(n_pos, n_bones, pos, weights, bones, pos_out, blend_out, st), "skinning");
  return ADR_OK;
}

adr_status adr_skin_bwd(adr_ctx* ctx, const float* pos, const float* bones, const float* blend, int32_t n_pos,
                        int32_t n_bones, float* g_pos_out, float* g_pos, float* g_weights, adr_stream stream) {
  if (ctx) ctx->geom_ok = false;
  adr_status r = check_skin(ctx, n_pos, n_bones);
  if (r != ADR_OK) return r;
  if (n_pos == 0) return ADR_OK;
  if (!pos || !bones || !blend || !g_pos_out) return fail(ADR_E_INVALID, "skin: pos, bones, blend and g_pos_out are required");
  if (g_pos == g_pos_out) return fail(ADR_E_INVALID, "skin: g_pos must not alias g_pos_out");
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  TIMED(14, launch_skin_bwd(n_pos, n_bones, pos, bones, blend, g_pos_out, g_pos, g_weights, st), "skinning adjoint");
  return ADR_OK;
}

adr_status adr_ctx_set_raster(adr_ctx* ctx, int32_t tiny_bbox, int32_t med_bbox) {
  if (!ctx) return fail(ADR_E_INVALID, "ctx is NULL");
  if (tiny_bbox < 1 || tiny_bbox > 1024 || med_bbox < tiny_bbox || med_bbox > 65536)
    return fail(ADR_E_INVALID, "raster split: need 1 <= tiny <= 1024 and tiny <= med <= 65536");
  ctx->tiny_bbox = tiny_bbox;
  ctx->med_bbox = med_bbox;
  return ADR_OK;
}

adr_status adr_ctx_profile(adr_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(ADR_E_INVALID, "ctx is NULL");
  ctx->prof = enable != 0 ? (1u << ADR_N_STAGES) - 1u : 0u;
  return ADR_OK;
}

adr_status adr_ctx_profile_stages(adr_ctx* ctx, uint32_t stage_mask) {
  if (!ctx) return fail(ADR_E_INVALID, "ctx is NULL");
  if (stage_mask >> ADR_N_STAGES) return fail(ADR_E_INVALID, "stage mask 0x%x names no stage", stage_mask);
  ctx->prof = stage_mask;
  return ADR_OK;
}

adr_status adr_ctx_profile_read(adr_ctx* ctx, double* ms, int64_t* count) {
  if (!ctx || !ms || !count) return fail(ADR_E_INVALID, "ctx, ms and count are required");
  for (int k = 0; k < ADR_N_STAGES; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
  }
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  for (const Span& sp : ctx->spans) {
    HIPCHK(hipEventSynchronize(sp.b), "hipEventSynchronize");
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, sp.a, sp.b), "hipEventElapsedTime");
    ms[sp.stage] += t;
    count[sp.stage] += 1;
    ctx->pool.push_back(sp.a);
    ctx->pool.push_back(sp.b);
  }
  ctx->spans.clear();
  return ADR_OK;
}

adr_status adr_adam_step(adr_ctx* ctx, const adr_param* params, int32_t n_params, int32_t t,
                         float lr, float beta1, float beta2, float eps, adr_stream stream) {
  if (ctx) ctx->geom_ok = false;
  if (!ctx) return fail(ADR_E_INVALID, "ctx is NULL");
  if (n_params < 0 || (n_params > 0 && !params)) return fail(ADR_E_INVALID, "bad params");
  if (t < 1) return fail(ADR_E_INVALID, "t must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return fail(ADR_E_INVALID, "bad Adam hyper-parameters");
  for (int k = 0; k < n_params; ++k) {
    if (params[k].n < 0) return fail(ADR_E_INVALID, "param %d: negative size", k);
    if (params[k].n > 0 && (!params[k].param || !params[k].grad || !params[k].m || !params[k].v))
      return fail(ADR_E_INVALID, "param %d: NULL pointer", k);
  }
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  TIMED(9, launch_adam(params, n_params, t, lr, beta1, beta2, eps, st), "adam");
  return ADR_OK;
}

adr_status adr_adam_step_maps(adr_ctx* ctx, const adr_map_param* maps, int32_t n_maps, int32_t t, float lr,
                              float beta1, float beta2, float eps, adr_stream stream) {
  if (ctx) ctx->geom_ok = false;
  if (!ctx) return fail(ADR_E_INVALID, "ctx is NULL");
  if (n_maps < 0 || (n_maps > 0 && !maps)) return fail(ADR_E_INVALID, "bad maps");
  if (t < 1) return fail(ADR_E_INVALID, "t must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return fail(ADR_E_INVALID, "bad Adam hyper-parameters");
  std::vector<Tex> ts((size_t)n_maps);
  for (int k = 0; k < n_maps; ++k) {
    adr_status r = check_tex(maps[k].tex, "map", false, ts[k]);
    if (r != ADR_OK) return r;
    if (!maps[k].grad || !maps[k].m || !maps[k].v) return fail(ADR_E_INVALID, "map %d: NULL grad, m or v", k);
  }
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  for (int k0 = 0; k0 < n_maps; k0 += 4) {
    AdamMapSet a{};
    for (int k = k0; k < n_maps && k < k0 + 4; ++k) {
      a.ms.t[a.ms.n] = ts[k];
      a.ms.g[a.ms.n] = maps[k].grad;
      a.m[a.ms.n] = maps[k].m;
      a.v[a.ms.n++] = maps[k].v;
    }
    TIMED(16, launch_adam_maps_tiles(a, t, lr, beta1, beta2, eps, st), "map adam");
    TIMED(17, launch_adam_maps_top(a, st), "map adam (upper levels)");
  }
  return ADR_OK;
}

adr_status adr_mip_build(adr_ctx* ctx, const adr_texture* tex, adr_stream stream) {
  if (ctx) ctx->geom_ok = false;
  if (!ctx || !tex) return fail(ADR_E_INVALID, "ctx and tex are required");
  Tex t;
  adr_status r = check_tex(*tex, "tex", true, t);
  if (r != ADR_OK) return r;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  TIMED(10, launch_mip_build(t, st), "mip build");
  return ADR_OK;
}

adr_status adr_mesh_adjacency(const int32_t* tri, int32_t n_tri, int32_t* adj) {
  if (n_tri < 0 || (n_tri > 0 && (!tri || !adj))) return fail(ADR_E_INVALID, "bad arguments");
  std::unordered_map<uint64_t, std::pair<int64_t, int32_t>> first;  // edge -> (t*3+k, count)
  first.reserve((size_t)n_tri * 2);
  for (int64_t i = 0; i < 3 * (int64_t)n_tri; ++i) adj[i] = -1;
  std::vector<int64_t> partner(3 * (size_t)n_tri, -1);
  for (int32_t t = 0; t < n_tri; ++t) {
    for (int k = 0; k < 3; ++k) {
      uint32_t a = (uint32_t)tri[3 * t + (k + 1) % 3], b = (uint32_t)tri[3 * t + (k + 2) % 3];
      uint64_t key = a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a;
      auto it = first.find(key);
      if (it == first.end()) {
        first.emplace(key, std::make_pair((int64_t)3 * t + k, 1));
      } else {
        if (it->second.second == 1) partner[3 * (size_t)t + k] = it->second.first;
        it->second.second += 1;
      }
    }
  }
  // an edge shared by exactly two triangles links them; otherwise -1
  for (int32_t t = 0; t < n_tri; ++t) {
    for (int k = 0; k < 3; ++k) {
      int64_t p = partner[3 * (size_t)t + k];
      if (p < 0) continue;
      uint32_t a = (uint32_t)tri[3 * t + (k + 1) % 3], b = (uint32_t)tri[3 * t + (k + 2) % 3];
      uint64_t key = a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a;
      if (first[key].second != 2) continue;
      adj[3 * (int64_t)t + k] = (int32_t)(p / 3);
      adj[p] = t;
    }
  }
  return ADR_OK;
}

adr_status adr_views_build(const float* dirs, int32_t n, float dist, float fov_deg, int32_t width,
                           int32_t height, float* mvp, float* eye) {
  if (n < 0 || (n > 0 && (!dirs || !mvp || !eye)) || width < 1 || height < 1 || !(dist > 0.f) ||
      !(fov_deg > 0.f && fov_deg < 180.f))
    return fail(ADR_E_INVALID, "bad arguments");
  const double nearp = 0.1, farp = 10.0;
  double fy = 1.0 / tan(fov_deg * M_PI / 360.0);
  double aspect = (double)width / (double)height;
  double P[4][4] = {{fy / aspect, 0, 0, 0},
                    {0, fy, 0, 0},
                    {0, 0, (farp + nearp) / (nearp - farp), 2 * farp * nearp / (nearp - farp)},
                    {0, 0, -1, 0}};
  for (int b = 0; b < n; ++b) {
    double d[3] = {dirs[3 * b], dirs[3 * b + 1], dirs[3 * b + 2]};
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(len > 0.0)) return fail(ADR_E_INVALID, "direction %d is zero", b);
    double e[3] = {dist * d[0] / len, dist * d[1] / len, dist * d[2] / len};
    double el = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    double f[3] = {-e[0] / el, -e[1] / el, -e[2] / el};
    double up[3] = {0, 1, 0};
    if (fabs(f[1]) > 0.999) { up[1] = 0; up[2] = 1; }
    double s[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    double sl = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    for (double& x : s) x /= sl;
    double u[3] = {s[1] * f[2] - s[2] * f[1], s[2] * f[0] - s[0] * f[2], s[0] * f[1] - s[1] * f[0]};
    double V[4][4] = {{s[0], s[1], s[2], -(s[0] * e[0] + s[1] * e[1] + s[2] * e[2])},
                      {u[0], u[1], u[2], -(u[0] * e[0] + u[1] * e[1] + u[2] * e[2])},
                      {-f[0], -f[1], -f[2], f[0] * e[0] + f[1] * e[1] + f[2] * e[2]},
                      {0, 0, 0, 1}};
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        double acc = 0;
        for (int k = 0; k < 4; ++k) acc += P[r][k] * V[k][c];
        mvp[16 * b + 4 * r + c] = (float)acc;
      }
    for (int k = 0; k < 3; ++k) eye[3 * b + k] = (float)e[k];
  }
  return ADR_OK;
}

adr_status adr_job_submit(adr_ctx* ctx, const adr_job_desc* desc, uint64_t* job_id) {
  if (ctx) ctx->geom_ok = false;
  if (!ctx || !desc || !job_id) return fail(ADR_E_INVALID, "ctx, desc and job_id are required");
  if (!ctx->jobs) {
    ctx->jobs = adr::jobs_create(ctx, ctx->device, ctx->budget);
    if (!ctx->jobs) return fail(ADR_E_NOMEM, "job server");
  }
  char msg[256] = "";
  adr_status r = adr::jobs_submit(ctx->jobs, desc, job_id, msg, sizeof(msg));
  if (r != ADR_OK) return fail(r, "%s", msg);
  return ADR_OK;
}

adr_status adr_job_poll(adr_ctx* ctx, uint64_t job_id, adr_job_status* st, adr_job_result* out) {
  if (ctx) ctx->geom_ok = false;
  if (!ctx || !st) return fail(ADR_E_INVALID, "ctx and st are required");
  if (!ctx->jobs) return fail(ADR_E_NOTFOUND, "no jobs");
  char msg[256] = "";
  adr_status r = adr::jobs_poll(ctx->jobs, job_id, st, out, msg, sizeof(msg));
  if (r < 0) return fail(r, "%s", msg);
  return r;
}

}  // extern "C"

// ---- batches: one launch per stage over the work of every item ----
//
// Each item keeps its own scratch (one device allocation for the batch,
// carved per item); at creation every stage's launch is planned per item
// (argument block and grid, as the single entry points plan it) and the
// non-empty plans are written to device tables: the argument blocks, and the
// first block of each item's range with the launch's total at the end.  A
// call then launches each stage once over all items.

namespace {

template <class A>
struct HostStage {
  std::vector<A> args;
  std::vector<int> start{0};
  size_t tab_off = 0, start_off = 0;
  bool too_big = false;
  void add(const Plan<A>& p) {
    if (p.blocks == 0) return;
    const int64_t total = (int64_t)start.back() + p.blocks;
    if (total > 0x7fffffffLL) {
      too_big = true;
      return;
    }
    args.push_back(p.a);
    start.push_back((int)total);
  }
  // offsets of the two tables from `off` (256-byte aligned); the bytes used
  size_t place(size_t off) {
    tab_off = (off + 255) & ~(size_t)255;
    start_off = (tab_off + sizeof(A) * args.size() + 255) & ~(size_t)255;
    return start_off + sizeof(int) * start.size();
  }
  void write(std::vector<unsigned char>& host) const {
    if (!args.empty()) memcpy(host.data() + tab_off, args.data(), sizeof(A) * args.size());
    memcpy(host.data() + start_off, start.data(), sizeof(int) * start.size());
  }
  Stage<A> device(unsigned char* base) const {
    Stage<A> s;
    s.tab = reinterpret_cast<const A*>(base + tab_off);
    s.start = reinterpret_cast<const int*>(base + start_off);
    s.n = (int)args.size();
    s.total = start.back();
    return s;
  }
};

struct BatchItem {
  MeshD m;
  ViewsD v;
  Tex kd, nm, orm;
  int model = 0;
  const float* ref = nullptr;
  int32_t loss_kind = 0;
  const float* dloss = nullptr;
  adr_fwd_out out{};
  adr_grads grads{};
  bool bwd = false;
  int32_t flags = 0;
  int slots = 0;
  Scratch s{};
};

// The scratch of one item carved from `base` (nullptr: sizes only); returns
// the bytes used.  Sizes as prepare_scratch allocates them.
size_t batch_carve(const MeshD& m, const ViewsD& v, bool bwd, int slots, bool det, unsigned char* base, Scratch* s) {
  const size_t B = v.B, V = m.n_pos > 0 ? m.n_pos : 1, T = m.n_tri > 0 ? m.n_tri : 1;
  const size_t px = B * (size_t)v.W * v.H;
  const size_t tiles = (size_t)((v.W + 15) / 16) * ((v.H + 15) / 16) * B;
  size_t off = 0;
  auto take = [&](size_t bytes) -> unsigned char* {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return base ? base + o : nullptr;
  };
  Scratch t{};
  t.snap = (int*)take(B * V * 16);
  t.orient = (int8_t*)take(B * T);
  t.nacc = (double*)take(V * 24);
  t.tacc = (double*)take(V * 24);
  t.nrm = (float*)take(V * 12);
  t.tan = (float*)take(V * 12);
  t.big = (uint32_t*)take(B * T * 4);
  t.big_cnt = (uint32_t*)take((B + 1) * 4);
  t.med = (uint32_t*)take(B * T * 4);
  t.partial = (float*)take(tiles * 4);
  t.mvpd = (double*)take(B * 128);
  t.n_partial = (int)tiles;
  t.det = det;
  if (det) {
    t.fix_n = (unsigned long long*)take(V * 24);
    t.fix_t = (unsigned long long*)take(V * 24);
  }
  if (bwd) {
    t.gcolor = (float*)take(px * 12);
    t.dclip = (float*)take(B * V * 16);
    t.dattr = (float*)take(V * 36);
    if (slots > 0) t.texrec = (float4*)take((size_t)(1 + slots) * px * 16);
    t.fix_attr = (unsigned long long*)take(V * 72);
    t.fix_clip = (unsigned long long*)take(B * V * 32);
    t.fix_pos = (unsigned long long*)take(V * 24);
  }
  if (s) *s = t;
  return off;
}

}  // namespace

struct adr_batch {
  adr_ctx* ctx = nullptr;
  std::vector<BatchItem> items;
  void* arena = nullptr;    // every item's scratch
  void* det_arena = nullptr;  // the deterministic texel sort's buffers, shared by the items in turn
  void* tables = nullptr;
  bool fwd_done = false, any_bwd = false;
  uint64_t scratch_bytes = 0;  // device bytes the batch holds
  // forward
  Stage<FillSet> frame_fill;
  Stage<FaceAccumArgs> faces;
  Stage<VertexNormalizeArgs> verts;
  Stage<XformArgs> xform;
  Stage<ClearArgs> clear;
  Stage<RasterArgs> r_small, r_med, r_big;
  Stage<ShadeFwdArgs> shade;
  Stage<AAFwdArgs> aa;
  Stage<LossReduceArgs> loss;
  // backward
  Stage<FillSet> bwd_fill;
  Stage<AABwdArgs> aa_bwd;
  Stage<ShadeBwdArgs> shade_bwd;
  Stage<FixToF32Args> conv;
  Stage<TexBwdArgs> tex;
  Stage<VertexBwdArgs> vbwd;
  Stage<FaceBwdArgs> fbwd;
  Stage<FixAddArgs> fadd;
  std::vector<int> det_tex;  // items whose texel adjoint is the deterministic sort
  std::vector<int> mips;     // items whose mip adjoint runs in the backward
};

static void batch_free(adr_batch* b) {
  if (!b) return;
  if (b->arena) (void)hipFree(b->arena);
  if (b->det_arena) (void)hipFree(b->det_arena);
  if (b->tables) (void)hipFree(b->tables);
  delete b;
}

extern "C" {

adr_status adr_batch_create(adr_ctx* ctx, int32_t n, const adr_batch_item* items, adr_batch** out) {
  if (!out) return fail(ADR_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(ADR_E_INVALID, "ctx is NULL");
  ctx->geom_ok = false;
  if (n < 1 || !items) return fail(ADR_E_INVALID, "a batch needs 1 or more items (n = %d)", n);
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  adr_batch* b = new (std::nothrow) adr_batch();
  if (!b) return fail(ADR_E_NOMEM, "batch");
  b->ctx = ctx;
  b->items.resize(n);
  size_t arena = 0, det_bytes = 0;
  int64_t det_E = 0, det_hw = 0;
  std::vector<size_t> offs(n);
  for (int i = 0; i < n; ++i) {
    const adr_batch_item& it = items[i];
    BatchItem& bi = b->items[i];
    adr_status r = check_fwd(ctx, it.mesh, it.mat, it.views, it.ref_image, it.loss_kind, it.out, it.flags, bi.m,
                             bi.v, bi.kd, bi.nm, bi.orm);
    if (r != ADR_OK) {
      batch_free(b);
      return fail(r, "batch item %d: %s", i, adr_last_error());
    }
    if (it.flags & ~(ADR_FWD_NO_AA | ADR_DETERMINISTIC | ADR_INDEPENDENT_MIPS | ADR_BWD_DEFER_MIP_ADJOINT)) {
      batch_free(b);
      return fail(ADR_E_INVALID,
                  "batch item %d: flags 0x%x (a batch takes ADR_FWD_NO_AA, ADR_DETERMINISTIC, "
                  "ADR_INDEPENDENT_MIPS and ADR_BWD_DEFER_MIP_ADJOINT; build mip chains with adr_mip_build)",
                  i, it.flags);
    }
    const bool det = (it.flags & ADR_DETERMINISTIC) != 0;
    bi.model = it.mat->model;
    bi.ref = it.ref_image;
    bi.loss_kind = it.loss_kind;
    bi.dloss = it.dloss;
    bi.out = *it.out;
    bi.flags = it.flags;
    bi.bwd = it.grads != nullptr;
    if (bi.bwd) {
      bi.grads = *it.grads;
      if (!it.ref_image) {
        batch_free(b);
        return fail(ADR_E_INVALID, "batch item %d: gradients need a reference image", i);
      }
      if (bi.grads.kd && bi.kd.fmt != ADR_TEX_F32) {
        batch_free(b);
        return fail(ADR_E_INVALID, "batch item %d: kd gradient needs an F32 kd map", i);
      }
      if (bi.grads.orm && bi.model != ADR_SHADE_GGX) {
        batch_free(b);
        return fail(ADR_E_INVALID, "batch item %d: orm gradient needs GGX", i);
      }
      bi.slots = tex_slots(bi.model, bi.grads.kd, bi.grads.normal, bi.grads.orm);
      b->any_bwd = true;
      if (det && bi.slots > 0) {
        const int64_t E = det_entries(bi.v, bi.slots);
        if (E >= (int64_t)0xFFFFFFFF) {
          batch_free(b);
          return fail(ADR_E_INVALID, "batch item %d: deterministic mode: view batch too large", i);
        }
        det_E = std::max(det_E, E);
        det_hw = std::max(det_hw, radix_hist_words(E));
      }
    }
    offs[i] = arena;
    arena += batch_carve(bi.m, bi.v, bi.bwd, bi.slots, det, nullptr, nullptr);
  }
  hipError_t e = hipMalloc(&b->arena, arena);
  if (e != hipSuccess) {
    batch_free(b);
    return fail(ADR_E_NOMEM, "batch scratch: hipMalloc(%zu): %s", arena, hipGetErrorString(e));
  }
  // the deterministic sort's buffers, sized for the largest item
  Scratch det{};
  if (det_E > 0) {
    const size_t parts[8] = {(size_t)det_E * 4, (size_t)det_E * 4, (size_t)det_E * 4, (size_t)det_E * 4,
                             det_vals_bytes(det_E), (size_t)det_hw * 4, (size_t)scan_tmp_words(det_hw) * 4 + 4,
                             det_part_bytes(det_E)};
    size_t o[8];
    for (int k = 0; k < 8; ++k) {
      o[k] = det_bytes;
      det_bytes += (parts[k] + 255) & ~(size_t)255;
    }
    if ((e = hipMalloc(&b->det_arena, det_bytes)) != hipSuccess) {
      batch_free(b);
      return fail(ADR_E_NOMEM, "batch sort buffers: hipMalloc(%zu): %s", det_bytes, hipGetErrorString(e));
    }
    unsigned char* d = static_cast<unsigned char*>(b->det_arena);
    det.det_k0 = (uint32_t*)(d + o[0]);
    det.det_v0 = (uint32_t*)(d + o[1]);
    det.det_k1 = (uint32_t*)(d + o[2]);
    det.det_v1 = (uint32_t*)(d + o[3]);
    det_carve(d + o[4], det_E, det);
    det.det_hist = (uint32_t*)(d + o[5]);
    det.det_tmp = (uint32_t*)(d + o[6]);
    det.det_part = (float4*)(d + o[7]);
  }
  // plan every stage of every item
  HostStage<FillSet> frame_fill, bwd_fill;
  HostStage<FaceAccumArgs> faces;
  HostStage<VertexNormalizeArgs> verts;
  HostStage<XformArgs> xform;
  HostStage<ClearArgs> clear;
  HostStage<RasterArgs> r_small, r_med, r_big;
  HostStage<ShadeFwdArgs> shade;
  HostStage<AAFwdArgs> aa;
  HostStage<LossReduceArgs> loss;
  HostStage<AABwdArgs> aa_bwd;
  HostStage<ShadeBwdArgs> shade_bwd;
  HostStage<FixToF32Args> conv;
  HostStage<TexBwdArgs> tex;
  HostStage<VertexBwdArgs> vbwd;
  HostStage<FaceBwdArgs> fbwd;
  HostStage<FixAddArgs> fadd;
  for (int i = 0; i < n; ++i) {
    BatchItem& bi = b->items[i];
    const adr_batch_item& it = items[i];
    const bool det_i = (bi.flags & ADR_DETERMINISTIC) != 0;
    batch_carve(bi.m, bi.v, bi.bwd, bi.slots, det_i, static_cast<unsigned char*>(b->arena) + offs[i], &bi.s);
    Scratch& s = bi.s;
    s.tiny_bbox = it.tiny_bbox > 0 ? it.tiny_bbox : ctx->tiny_bbox;
    s.med_bbox = it.med_bbox > 0 ? it.med_bbox : ctx->med_bbox;
    if (s.tiny_bbox > s.med_bbox) {
      batch_free(b);
      return fail(ADR_E_INVALID, "batch item %d: raster split %d > %d", i, s.tiny_bbox, s.med_bbox);
    }
    if (det_i && bi.slots > 0) {
      s.det_k0 = det.det_k0;
      s.det_v0 = det.det_v0;
      s.det_k1 = det.det_k1;
      s.det_v1 = det.det_v1;
      s.det_vals = det.det_vals;
      s.det_fy = det.det_fy;
      s.det_gsum = det.det_gsum;
      s.det_hist = det.det_hist;
      s.det_tmp = det.det_tmp;
      s.det_part = det.det_part;
    }
    bi.v.mvpd = s.mvpd;
    const MeshD& m = bi.m;
    const ViewsD& v = bi.v;
    const int64_t npx = (int64_t)v.B * v.W * v.H;
    // a forward-only item with a precomputed frame skips the frame stage
    if (!bi.bwd && it.mesh->nrm && it.mesh->tan) {
      s.nrm = const_cast<float*>(it.mesh->nrm);
      s.tan = const_cast<float*>(it.mesh->tan);
    } else {
      const FramePlans fp = plan_vertex_frame(m, s);
      frame_fill.add(fp.fill);
      faces.add(fp.faces);
      verts.add(fp.verts);
    }
    xform.add(plan_xform(m, v, s));
    clear.add(plan_clear_vis(bi.out.vis, bi.out.coverage, npx, s.big_cnt, v.B));
    const RasterPlans rp = plan_raster(m, v, s, bi.out.vis, bi.out.coverage, nullptr);
    r_small.add({rp.a, rp.small});
    r_med.add({rp.a, rp.med});
    r_big.add({rp.a, rp.big});
    shade.add(plan_shade_fwd(m, v, bi.model, bi.kd, bi.nm, bi.orm, s, bi.out.vis, bi.out.color, bi.out.tri_id,
                             nullptr, nullptr));
    aa.add(plan_aa_fwd(m, v, s, bi.out.vis, bi.out.color, bi.ref, bi.loss_kind, (bi.flags & ADR_FWD_NO_AA) ? 1 : 0,
                       bi.out.image, bi.out.dimage, bi.out.aa));
    if (bi.ref) loss.add(plan_loss_reduce(v, bi.ref, s, bi.out.loss));
    if (!bi.bwd) continue;
    const adr_grads& g = bi.grads;
    const int64_t V = m.n_pos > 0 ? m.n_pos : 1;
    const int64_t n_clip = 4 * (int64_t)v.B * V, n_attr = 9 * V;
    FillSet f{};
    f.add(s.fix_clip, n_clip);
    f.add(s.fix_attr, n_attr);
    f.add(s.fix_pos, 3 * V);
    bwd_fill.add(plan_fill_multi(f));
    aa_bwd.add(plan_aa_bwd(m, v, s, bi.out.vis, bi.out.color, bi.out.dimage, bi.dloss,
                           (bi.flags & ADR_FWD_NO_AA) ? 1 : 0, bi.out.aa));
    shade_bwd.add(plan_shade_bwd(m, v, bi.model, bi.kd, bi.nm, bi.orm, g.kd, g.normal, g.orm, s, bi.out.vis, nullptr,
                                 nullptr, nullptr));
    conv.add(plan_fix_to_f32(s.fix_clip, s.dclip, n_clip, det_i, s.fix_attr, s.dattr, n_attr));
    if (det_i) {
      if (bi.slots > 0) b->det_tex.push_back(i);
    } else {
      tex.add(plan_tex_bwd(v, bi.model, bi.kd, bi.nm, bi.orm, g.kd, g.normal, g.orm, s, nullptr, nullptr));
    }
    if (!(bi.flags & (ADR_INDEPENDENT_MIPS | ADR_BWD_DEFER_MIP_ADJOINT))) b->mips.push_back(i);
    const MeshBwdPlans mp = plan_mesh_bwd(m, v, s, g.pos, g.vnormal);
    vbwd.add(mp.verts);
    fbwd.add(mp.faces);
    fadd.add(mp.add);
  }
  // the tables, uploaded once
  bool too_big = false;
  size_t bytes = 0;
  auto place = [&](auto& hs) {
    too_big |= hs.too_big;
    bytes = hs.place(bytes);
  };
  place(frame_fill), place(faces), place(verts), place(xform), place(clear), place(r_small), place(r_med);
  place(r_big), place(shade), place(aa), place(loss), place(bwd_fill), place(aa_bwd), place(shade_bwd);
  place(conv), place(tex), place(vbwd), place(fbwd), place(fadd);
  if (too_big) {
    batch_free(b);
    return fail(ADR_E_INVALID, "batch: a stage needs 2^31 or more blocks");
  }
  std::vector<unsigned char> host(bytes);
  auto write = [&](const auto& hs) { hs.write(host); };
  write(frame_fill), write(faces), write(verts), write(xform), write(clear), write(r_small), write(r_med);
  write(r_big), write(shade), write(aa), write(loss), write(bwd_fill), write(aa_bwd), write(shade_bwd);
  write(conv), write(tex), write(vbwd), write(fbwd), write(fadd);
  if ((e = hipMalloc(&b->tables, bytes)) != hipSuccess) {
    batch_free(b);
    return fail(ADR_E_NOMEM, "batch tables: hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  if ((e = hipMemcpy(b->tables, host.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "batch tables: hipMemcpy");
  }
  unsigned char* t = static_cast<unsigned char*>(b->tables);
  b->frame_fill = frame_fill.device(t);
  b->faces = faces.device(t);
  b->verts = verts.device(t);
  b->xform = xform.device(t);
  b->clear = clear.device(t);
  b->r_small = r_small.device(t);
  b->r_med = r_med.device(t);
  b->r_big = r_big.device(t);
  b->shade = shade.device(t);
  b->aa = aa.device(t);
  b->loss = loss.device(t);
  b->bwd_fill = bwd_fill.device(t);
  b->aa_bwd = aa_bwd.device(t);
  b->shade_bwd = shade_bwd.device(t);
  b->conv = conv.device(t);
  b->tex = tex.device(t);
  b->vbwd = vbwd.device(t);
  b->fbwd = fbwd.device(t);
  b->fadd = fadd.device(t);
  b->scratch_bytes = arena + det_bytes + bytes;
  *out = b;
  return ADR_OK;
}

adr_status adr_batch_fwd(adr_batch* b, adr_stream stream) {
  if (!b) return fail(ADR_E_INVALID, "batch is NULL");
  adr_ctx* ctx = b->ctx;
  ctx->geom_ok = false;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  TIMED(0, launch_fill_multi_n(b->frame_fill, st), "vertex frame");
  TIMED(0, launch_face_accum_n(b->faces, st), "vertex frame");
  TIMED(0, launch_vertex_normalize_n(b->verts, st), "vertex frame");
  TIMED(1, launch_xform_n(b->xform, st), "transform");
  TIMED(12, launch_clear_vis_n(b->clear, st), "clear");
  TIMED(2, launch_raster_n(b->r_small, b->r_med, b->r_big, st), "raster");
  TIMED(3, launch_shade_fwd_n(b->shade, st), "shade");
  TIMED(4, launch_aa_fwd_n(b->aa, st), "antialias/loss");
  TIMED(18, launch_loss_reduce_n(b->loss, st), "loss reduction");
  b->fwd_done = true;
  return ADR_OK;
}

adr_status adr_batch_bwd(adr_batch* b, adr_stream stream) {
  if (!b) return fail(ADR_E_INVALID, "batch is NULL");
  adr_ctx* ctx = b->ctx;
  ctx->geom_ok = false;
  if (!b->any_bwd) return fail(ADR_E_INVALID, "batch: no item has gradients");
  if (!b->fwd_done) return fail(ADR_E_INVALID, "batch: the backward needs a forward of the batch first");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device), "hipSetDevice");
  TIMED(12, launch_fill_multi_n(b->bwd_fill, st), "clear");
  TIMED(5, launch_aa_bwd_n(b->aa_bwd, st), "antialias adjoint");
  TIMED(6, launch_shade_bwd_n(b->shade_bwd, st), "shading adjoint");
  TIMED(12, launch_fix_to_f32_n(b->conv, st), "accumulator conversion");
  TIMED(11, launch_tex_bwd_n(b->tex, st), "texel adjoint");
  for (int i : b->det_tex) {
    const BatchItem& bi = b->items[i];
    TIMED(11, launch_tex_bwd(bi.v, bi.model, bi.kd, bi.nm, bi.orm, bi.grads.kd, bi.grads.normal, bi.grads.orm,
                             bi.s, st),
          "texel adjoint");
  }
  for (int i : b->mips) {
    const BatchItem& bi = b->items[i];
    MipSet ms{};
    const Tex* maps[3] = {&bi.kd, &bi.nm, &bi.orm};
    float* gs[3] = {bi.grads.kd, bi.grads.normal, bi.grads.orm};
    for (int k = 0; k < 3; ++k)
      if (gs[k] && maps[k]->levels > 1 && (k < 2 || bi.model == ADR_SHADE_GGX)) {
        ms.t[ms.n] = *maps[k];
        ms.g[ms.n++] = gs[k];
      }
    if (ms.n) TIMED(7, launch_mip_adjoint_set(ms, st), "mip adjoint");
  }
  TIMED(8, launch_vertex_bwd_n(b->vbwd, st), "mesh adjoint");
  TIMED(8, launch_face_bwd_n(b->fbwd, st), "mesh adjoint");
  TIMED(8, launch_fix_add_n(b->fadd, st), "mesh adjoint");
  return ADR_OK;
}

adr_status adr_batch_info(const adr_batch* b, int32_t* n_items, uint64_t* scratch_bytes) {
  if (!b) return fail(ADR_E_INVALID, "batch is NULL");
  if (n_items) *n_items = (int32_t)b->items.size();
  if (scratch_bytes) *scratch_bytes = b->scratch_bytes;
  return ADR_OK;
}

adr_status adr_batch_destroy(adr_batch* b) {
  if (!b) return ADR_OK;
  HIPCHK(hipSetDevice(b->ctx->device), "hipSetDevice");
  batch_free(b);  // hipFree waits for the device
  return ADR_OK;
}

}  // extern "C"
