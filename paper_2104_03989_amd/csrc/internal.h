// Internal declarations shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adr.h"

namespace adr {

constexpr uint64_t kKeyEmpty = 0xFFFFFFFF00000000ull;
constexpr int kZMax = 16777215;
constexpr int kMaxLevels = 15;
constexpr int kTinyBBox = 64;      // default: pixel bbox up to this walked by one thread
constexpr int kMedBBox = 4096;     // default: up to this walked by a whole wave; larger: tile-binned
constexpr int kBigTile = 16;       // big-triangle tiles are kBigTile x kBigTile pixels
constexpr int kBigBlocks = 1024;   // most blocks of one big-triangle raster launch (4 per CU)

// Texture as the kernels see it: level offsets in texels precomputed.
struct Tex {
  const void* data;
  int size, levels, channels, fmt;
  int off[kMaxLevels + 1];
};

struct MeshD {
  const float* pos;
  const int* tri;
  const float* uv;
  const int* uv_tri;
  const int* adj;
  int n_pos, n_tri, n_uv;
};

struct ViewsD {
  const float* mvp;
  const float* eye;
  const float* light_dir;
  const float* light_rgb;
  int B, W, H;  // W, H: visibility samples per row / column (pixels x ms)
  int ms;       // multisampling: ms x ms visibility samples per pixel (1: none)
  // derived on the host (views_derive): log2 ms, the pixel grid, and the NDC
  // step of one pixel and of one sample (uniform divisions kept out of the
  // per-pixel code)
  int msh, Wp, Hp;
  double pxs, pys, sxs, sys;
  // [B,16] the view matrices in float64 (exact), written by the transform
  // stage into the call's scratch for the kernels that rebuild float64 clip
  // coordinates (NULL outside the render calls)
  const double* mvpd;
};

// Fills the derived fields of v from B, W, H and ms (ms 1, 2 or 4).
inline void views_derive(ViewsD& v) {
  v.msh = v.ms == 4 ? 2 : (v.ms == 2 ? 1 : 0);
  v.Wp = v.W >> v.msh;
  v.Hp = v.H >> v.msh;
  v.pxs = v.Wp > 0 ? 2.0 / v.Wp : 0.0;
  v.pys = v.Hp > 0 ? 2.0 / v.Hp : 0.0;
  v.sxs = v.W > 0 ? 2.0 / v.W : 0.0;
  v.sys = v.H > 0 ? 2.0 / v.H : 0.0;
}

// Per-call scratch owned by the context.
struct Scratch {
  int* snap;          // [B,V,4]
  int8_t* orient;     // [B,T]
  double* nacc;       // [V,3] unnormalised vertex normals (float64)
  double* tacc;       // [V,3] unnormalised vertex tangents (float64)
  float* nrm;         // [V,3]
  float* tan;         // [V,3]
  uint32_t* big;      // [B,T] big-triangle lists (per view segments of T)
  uint32_t* big_cnt;  // [B + 1]: per-view big-triangle counts, then the medium-queue count
  uint32_t* med;      // [B * n_tri] medium-triangle queue (view * n_tri + triangle)
  int tiny_bbox, med_bbox;  // raster work split (the context's settings)
  float* partial;     // loss partials
  float* gcolor;      // [B,H,W,3] dL/d(colour before AA)
  float* dclip;       // [B,V,4]
  float* dattr;       // [V,9] d(world pos), d(normal), d(tangent)
  float4* texrec;     // [1 + maps, B,H,W] texture-sample records of the adjoint
  float* image_s;     // [B,H,W,3] antialiased samples before the multisample resolve
  double* mvpd;       // [B,16] the view matrices in float64
  int n_partial;
  // vertex-side adjoint accumulators (float64, or fixed point in
  // deterministic mode) and the deterministic mode's sort buffers
  bool det;
  unsigned long long* fix_n;     // [V,3] frame accumulators (deterministic mode)
  unsigned long long* fix_t;     // [V,3]
  unsigned long long* fix_attr;  // [V,9]
  unsigned long long* fix_clip;  // [B,V,4]
  unsigned long long* fix_pos;   // [V,3]
  uint32_t *det_k0, *det_v0, *det_k1, *det_v1, *det_hist, *det_tmp;
  float4* det_vals;              // [entries] (level-weighted adjoint, fx)
  float* det_fy;                 // [entries]
  float4* det_gsum;              // [3 entries] corner sums of the groups, at their first positions
  float4* det_part;              // [3 x 2 tiles]
};

// Up to four texture chains (a material's maps) and their gradient buffers.
struct MipSet {
  Tex t[4];
  float* g[4];
  int n;
};

// Optimised maps for the fused adjoint + Adam + rebuild of their chains: the
// maps and gradient chains, and the Adam moments of each map's level 0.
struct AdamMapSet {
  MipSet ms;
  float* m[4];
  float* v[4];
};

struct TessD {
  const int* vidx;    // [Vt,3]
  const float* w;     // [Vt,3]
  const float* duv;   // [Vt,2]
  int n;
};

// Zero-fill of several ranges of 8-byte words in one launch.
constexpr int kFillRanges = 6;
struct FillSet {
  unsigned long long* p[kFillRanges];
  int64_t len[kFillRanges];
  int n;
  void add(unsigned long long* q, int64_t l) {
    if (q && l > 0 && n < kFillRanges) {
      p[n] = q;
      len[n++] = l;
    }
  }
};
// ---- batched launches ----
// A kernel launch as a batch takes it: the kernel's argument block and its
// grid (0 blocks: nothing to launch).
template <class A>
struct Plan {
  A a;
  unsigned blocks;
};
// One stage of a batch: the argument blocks of n items in device memory and
// the first block of each item's range, start[n] = the launch's blocks.
template <class A>
struct Stage {
  const A* tab = nullptr;
  const int* start = nullptr;
  int n = 0, total = 0;
};

// Argument blocks of the kernels a batch launches.
struct FaceAccumArgs {
  MeshD m;
  double *nacc, *tacc;
  unsigned long long *fn, *ft;
};
struct VertexNormalizeArgs {
  int n;
  double *nacc, *tacc;
  const unsigned long long *fn, *ft;
  float *nrm, *tan;
};
struct FixToF32Args {
  const unsigned long long* src;
  float* dst;
  int64_t n;
  const unsigned long long* src2;
  float* dst2;
  int64_t n2;
  bool det;
};
struct FixAddArgs {
  const unsigned long long* src;
  float* dst;
  int64_t n;
  bool det;
};
struct VertexBwdArgs {
  MeshD m;
  ViewsD v;
  const float* dclip;
  float* dattr;
  const double *nacc, *tacc;
  float *gpos, *gvn;
};
struct FaceBwdArgs {
  MeshD m;
  const float* dattr;
  unsigned long long* fpos;
  bool det;
};
struct FramePlans {
  Plan<FillSet> fill;
  Plan<FaceAccumArgs> faces;
  Plan<VertexNormalizeArgs> verts;
};
struct MeshBwdPlans {
  Plan<VertexBwdArgs> verts;
  Plan<FaceBwdArgs> faces;
  Plan<FixAddArgs> add;
};
struct XformArgs {
  MeshD m;
  ViewsD v;
  int4* snap;
  double* mvpd;
};
struct ClearArgs {
  uint64_t* vis;
  uint32_t* cov;
  int64_t n;
  uint32_t* big_cnt;
  int B;
};
// The three raster kernels share one argument block.
struct RasterArgs {
  MeshD m;
  ViewsD v;
  const int4* snap;
  int8_t* orient;
  uint32_t *big, *big_cnt, *med;
  unsigned long long* vis;
  uint32_t* cov;
  const unsigned long long* floor;
  int tiny, med_max;
  int tiles_x, tiles_y;  // kBigTile tiles
};
struct RasterPlans {
  RasterArgs a;
  unsigned small, med, big;  // blocks of the three kernels
};
struct ShadeArgs {
  MeshD m;
  ViewsD v;
  int model;
  Tex kd, nm, orm;
  Tex al;                 // alpha map (data NULL: none)
  const float* galpha;    // dL/d alpha per pixel (adjoint of a depth-peeled layer), or NULL
  const float* nrm;
  const float* tan;
  const uint64_t* vis;
  int tiles_x, tiles_y;
};
struct ShadeFwdArgs {
  ShadeArgs s;
  float* color;
  int32_t* tri_id;
  float* alpha;
};
// Gradient slots of the texture-sample records (maps with a gradient buffer).
struct TexSlots {
  int kd, nm, orm, al;  // slot of each map, -1 without a gradient buffer
  int n;
};
struct ShadeBwdArgs {
  ShadeArgs s;
  TexSlots sl;
  const float* gcolor;
  float4* rec;
  unsigned long long *fclip, *fattr;
  bool det;
};
struct TexBwdArgs {
  Tex t[4];
  float* g[4];
  int n;
  int pair;   // slots 0 and 1 are 3-channel maps of one size and layout: one window serves both
  const float4* rec;
  ViewsD v;
  int tiles_x, tiles_y;
};
struct AAArgs {
  MeshD m;
  ViewsD v;
  const int4* snap;
  const int8_t* orient;
  const uint64_t* vis;
  const float* color;
  int tiles_x, tiles_y;
  int no_aa;
  float4* stats;  // per (sample) pixel (W, acc) of the received antialiasing: written by the
                  // forward, read by the adjoint instead of re-evaluating pairs (NULL: none)
  float* codes;   // per pixel, codes of the pairs with the right and the upper neighbour
  int code_stride;  // floats between two pixels' code pairs (pixel o's at codes[code_stride * o])
};
struct AAFwdArgs {
  AAArgs a;
  const float* ref;
  int loss_kind;
  float *image, *dimage, *partial;
};
struct AABwdArgs {
  AAArgs a;
  const float *dimage, *dloss;
  float* gcolor;
  unsigned long long* fclip;
  bool det;
};
struct LossReduceArgs {
  const float* partial;
  int n;
  float inv_n;
  float* loss;
};

// Records `msg` as the calling thread's last error and returns `code`.
adr_status report(adr_status code, const char* msg);

// ---- launchers (stream-ordered, no host sync) ----
hipError_t launch_tess_fwd(const MeshD& base, const TessD& ts, const double* nacc, const Tex& disp,
                           float* out, hipStream_t st);
hipError_t launch_tess_bwd(const MeshD& base, const TessD& ts, const double* nacc, const Tex& disp,
                           float* gout, float* gbase, float* dattr, float* gdisp, hipStream_t st);
hipError_t launch_vertex_frame(const MeshD& m, const Scratch& s, hipStream_t st);
hipError_t launch_xform(const MeshD& m, const ViewsD& v, const Scratch& s, hipStream_t st);
hipError_t launch_clear_vis(uint64_t* vis, uint32_t* cov, int64_t n, uint32_t* big_cnt, int B,
                            hipStream_t st);
hipError_t launch_orient(const MeshD& m, const ViewsD& v, const Scratch& s, hipStream_t st);
// floor: keys of the previous depth-peeling layer (NULL: no lower bound).
hipError_t launch_raster(const MeshD& m, const ViewsD& v, const Scratch& s, uint64_t* vis,
                         uint32_t* cov, hipStream_t st, const uint64_t* floor = nullptr);
// al / alpha: the alpha map and the per-pixel alpha output of a depth-peeled
// layer (both optional).
hipError_t launch_shade_fwd(const MeshD& m, const ViewsD& v, int model, const Tex& kd,
                            const Tex& nm, const Tex& orm, const Scratch& s, const uint64_t* vis,
                            float* color, int32_t* tri_id, hipStream_t st, const Tex* al = nullptr,
                            float* alpha = nullptr);
// stats: per-pixel (W, acc) of the received antialiasing, written by the
// forward and read by the adjoint (optional).
hipError_t launch_aa_loss_fwd(const MeshD& m, const ViewsD& v, const Scratch& s,
                              const uint64_t* vis, const float* color, const float* ref,
                              int loss_kind, int no_aa, float* image, float* dimage, float* loss,
                              hipStream_t st, float* stats = nullptr);
// The image loss from the partials the forward above left (ref non-NULL).
hipError_t launch_loss_reduce(const ViewsD& v, const float* ref, const Scratch& s, float* loss, hipStream_t st);
hipError_t launch_aa_bwd(const MeshD& m, const ViewsD& v, const Scratch& s, const uint64_t* vis,
                         const float* color, const float* dimage, const float* dloss, int no_aa,
                         hipStream_t st, const float* stats = nullptr);
hipError_t launch_oit_blend(int64_t n, const uint64_t* vis, const float* color, const float* alpha,
                            const float* behind, float* blend, hipStream_t st);
hipError_t launch_oit_blend_bwd(int64_t n, const uint64_t* vis, const float* color, const float* alpha,
                                const float* behind, float* g, float* galpha, float* gbehind, hipStream_t st);
hipError_t launch_skin_fwd(int n, int nb, const float* pos, const float* w, const float* bones, float* out,
                           float* blend, hipStream_t st);
hipError_t launch_skin_bwd(int n, int nb, const float* pos, const float* bones, const float* blend, float* gout,
                           float* gpos, float* gw, hipStream_t st);
hipError_t launch_downsample(const float* in, int B, int H, int W, int k, float* out, hipStream_t st);
hipError_t launch_laplacian(int n, const float* pos, const int* offs, const int* nbr, const float* dref,
                            float lambda, float* r, double* part, float* dout, float* loss, float* gpos,
                            hipStream_t st);

// Deterministic-mode sizes and helpers.
int64_t det_entries(const ViewsD& v, int slots);
// Bytes of the value buffers of E entries (det_vals, det_fy and det_gsum,
// carved from one allocation by det_carve) and of the tile partials.
size_t det_vals_bytes(int64_t E);
size_t det_part_bytes(int64_t E);
void det_carve(void* p, int64_t E, Scratch& s);
int64_t radix_hist_words(int64_t n);
int64_t scan_tmp_words(int64_t n);
hipError_t launch_exscan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st);
hipError_t launch_fill_multi(const FillSet& f, hipStream_t st);
// src2/dst2 (optional): a second array converted in the same launch.
hipError_t launch_fix_to_f32(const unsigned long long* src, float* dst, int64_t n, bool det, hipStream_t st,
                             const unsigned long long* src2 = nullptr, float* dst2 = nullptr, int64_t n2 = 0);

// Number of texture-gradient slots (maps with a gradient buffer).
int tex_slots(int model, const float* gkd, const float* gnm, const float* gorm, const float* gal = nullptr);
// al / gal / galpha: the alpha map, its gradient and dL/d alpha per pixel of
// a depth-peeled layer (all optional; galpha selects the alpha variant).
hipError_t launch_shade_bwd(const MeshD& m, const ViewsD& v, int model, const Tex& kd,
                            const Tex& nm, const Tex& orm, float* gkd, float* gnm, float* gorm,
                            const Scratch& s, const uint64_t* vis, hipStream_t st, const Tex* al = nullptr,
                            float* gal = nullptr, const float* galpha = nullptr);
hipError_t launch_tex_bwd(const ViewsD& v, int model, const Tex& kd, const Tex& nm, const Tex& orm,
                          float* gkd, float* gnm, float* gorm, const Scratch& s, hipStream_t st,
                          const Tex* al = nullptr, float* gal = nullptr);
hipError_t launch_mip_adjoint_set(const MipSet& ms, hipStream_t st);
hipError_t launch_mip_build_set(const MipSet& ms, hipStream_t st);
// pos_cleared: the face-term accumulator (fix_pos) was zeroed by the caller.
hipError_t launch_mesh_bwd(const MeshD& m, const ViewsD& v, const Scratch& s, float* gpos,
                           float* gvnormal, hipStream_t st, bool pos_cleared = false);
hipError_t launch_mip_build(const Tex& t, hipStream_t st);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st);
// Map Adam in two launches: the level-0 tiles (adjoint of the tile levels,
// Adam, rebuild of the tile levels), then the levels above the tiles.
hipError_t launch_adam_maps_tiles(const AdamMapSet& a, int t, float lr, float b1, float b2, float eps,
                                  hipStream_t st);
hipError_t launch_adam_maps_top(const AdamMapSet& a, hipStream_t st);
hipError_t launch_adam(const adr_param* params, int n, int t, float lr, float b1, float b2,
                       float eps, hipStream_t st);

// ---- plans (argument block and grid of one launch) and batched launchers ----
Plan<FillSet> plan_fill_multi(const FillSet& f);
Plan<FixToF32Args> plan_fix_to_f32(const unsigned long long* src, float* dst, int64_t n, bool det,
                                   const unsigned long long* src2, float* dst2, int64_t n2);
FramePlans plan_vertex_frame(const MeshD& m, const Scratch& s);
MeshBwdPlans plan_mesh_bwd(const MeshD& m, const ViewsD& v, const Scratch& s, float* gpos, float* gvnormal);
Plan<XformArgs> plan_xform(const MeshD& m, const ViewsD& v, const Scratch& s);
Plan<ClearArgs> plan_clear_vis(uint64_t* vis, uint32_t* cov, int64_t n, uint32_t* big_cnt, int B);
RasterPlans plan_raster(const MeshD& m, const ViewsD& v, const Scratch& s, uint64_t* vis, uint32_t* cov,
                        const uint64_t* floor);
Plan<ShadeFwdArgs> plan_shade_fwd(const MeshD& m, const ViewsD& v, int model, const Tex& kd, const Tex& nm,
                                   const Tex& orm, const Scratch& s, const uint64_t* vis, float* color,
                                   int32_t* tri_id, const Tex* al, float* alpha);
Plan<ShadeBwdArgs> plan_shade_bwd(const MeshD& m, const ViewsD& v, int model, const Tex& kd, const Tex& nm,
                                   const Tex& orm, float* gkd, float* gnm, float* gorm, const Scratch& s,
                                   const uint64_t* vis, const Tex* al, float* gal, const float* galpha);
Plan<TexBwdArgs> plan_tex_bwd(const ViewsD& v, int model, const Tex& kd, const Tex& nm, const Tex& orm, float* gkd,
                              float* gnm, float* gorm, const Scratch& s, const Tex* al, float* gal);
Plan<AAFwdArgs> plan_aa_fwd(const MeshD& m, const ViewsD& v, const Scratch& s, const uint64_t* vis,
                            const float* color, const float* ref, int loss_kind, int no_aa, float* image,
                            float* dimage, float* stats);
Plan<LossReduceArgs> plan_loss_reduce(const ViewsD& v, const float* ref, const Scratch& s, float* loss);
Plan<AABwdArgs> plan_aa_bwd(const MeshD& m, const ViewsD& v, const Scratch& s, const uint64_t* vis,
                            const float* color, const float* dimage, const float* dloss, int no_aa,
                            const float* stats);

hipError_t launch_fill_multi_n(const Stage<FillSet>& s, hipStream_t st);
hipError_t launch_face_accum_n(const Stage<FaceAccumArgs>& s, hipStream_t st);
hipError_t launch_vertex_normalize_n(const Stage<VertexNormalizeArgs>& s, hipStream_t st);
hipError_t launch_fix_to_f32_n(const Stage<FixToF32Args>& s, hipStream_t st);
hipError_t launch_vertex_bwd_n(const Stage<VertexBwdArgs>& s, hipStream_t st);
hipError_t launch_face_bwd_n(const Stage<FaceBwdArgs>& s, hipStream_t st);
hipError_t launch_fix_add_n(const Stage<FixAddArgs>& s, hipStream_t st);
hipError_t launch_xform_n(const Stage<XformArgs>& s, hipStream_t st);
hipError_t launch_clear_vis_n(const Stage<ClearArgs>& s, hipStream_t st);
hipError_t launch_raster_n(const Stage<RasterArgs>& small, const Stage<RasterArgs>& med,
                           const Stage<RasterArgs>& big, hipStream_t st);
hipError_t launch_shade_fwd_n(const Stage<ShadeFwdArgs>& s, hipStream_t st);
hipError_t launch_shade_bwd_n(const Stage<ShadeBwdArgs>& s, hipStream_t st);
hipError_t launch_tex_bwd_n(const Stage<TexBwdArgs>& s, hipStream_t st);
hipError_t launch_aa_fwd_n(const Stage<AAFwdArgs>& s, hipStream_t st);
hipError_t launch_loss_reduce_n(const Stage<LossReduceArgs>& s, hipStream_t st);
hipError_t launch_aa_bwd_n(const Stage<AABwdArgs>& s, hipStream_t st);

}  // namespace adr
