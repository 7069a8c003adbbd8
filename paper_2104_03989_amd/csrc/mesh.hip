// Mesh operations (Sec. 5.1, "Tangent space"): smooth vertex normals and
// UV tangents recomputed from the positions every step, and the adjoint that
// folds gradients w.r.t. clip coordinates, interpolated attributes, normals
// and tangents back into vertex positions.
//   n_v = normalize(sum_{f at v} (p1 - p0) x (p2 - p0))
//   t_f = (e1 dv2 - e2 dv1) / (du1 dv2 - du2 dv1)   (skipped if |r| < 1e-12)
//   t_v = normalize(sum_{f at v} t_f)
#include "dev.h"

namespace adr {

// The frame stage runs in float64 (d3 helpers): around a UV pole the per-face
// tangents nearly cancel, and a float32 sum there loses the tangent's
// direction.  The stage is per face and per vertex, so float64 costs nothing
// measurable.
struct FaceFrame {
  d3 e1, e2, fn, tf;
  bool tan_ok;
  double r, d1v, d2v;
};

__device__ __forceinline__ FaceFrame face_frame(const MeshD& m, int t) {
  int i0 = m.tri[3 * t], i1 = m.tri[3 * t + 1], i2 = m.tri[3 * t + 2];
  int u0 = m.uv_tri[3 * t], u1 = m.uv_tri[3 * t + 1], u2 = m.uv_tri[3 * t + 2];
  d3 p0 = dld3f(m.pos, i0), p1 = dld3f(m.pos, i1), p2 = dld3f(m.pos, i2);
  FaceFrame f;
  f.e1 = p1 - p0;
  f.e2 = p2 - p0;
  f.fn = dcross(f.e1, f.e2);
  double d1u = (double)m.uv[2 * u1] - (double)m.uv[2 * u0], d1v = (double)m.uv[2 * u1 + 1] - (double)m.uv[2 * u0 + 1];
  double d2u = (double)m.uv[2 * u2] - (double)m.uv[2 * u0], d2v = (double)m.uv[2 * u2 + 1] - (double)m.uv[2 * u0 + 1];
  f.r = d1u * d2v - d2u * d1v;
  f.d1v = d1v;
  f.d2v = d2v;
  f.tan_ok = fabs(f.r) >= 1e-12;
  f.tf = f.tan_ok ? (1.0 / f.r) * (d2v * f.e1 - d1v * f.e2) : dmk(0.0, 0.0, 0.0);
  return f;
}

// fn/ft non-null: deterministic mode, fixed-point accumulators.
__device__ __forceinline__ void face_accum_body(const FaceAccumArgs& a, int bid, int) {
  const MeshD& m = a.m;
  int t = bid * 256 + threadIdx.x;
  if (t >= m.n_tri) return;
  FaceFrame f = face_frame(m, t);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int v = m.tri[3 * t + k];
    if (a.fn) {
      fix_add3(a.fn, v, f.fn);
      if (f.tan_ok) fix_add3(a.ft, v, f.tf);
    } else {
      datomic3(a.nacc, v, f.fn);
      if (f.tan_ok) datomic3(a.tacc, v, f.tf);
    }
  }
}
ADR_KERNEL(__launch_bounds__(256), k_face_accum, FaceAccumArgs, face_accum_body)

__device__ __forceinline__ void vertex_normalize_body(const VertexNormalizeArgs& a, int bid, int) {
  int v = bid * 256 + threadIdx.x;
  if (v >= a.n) return;
  if (a.fn) {  // the adjoint reads the unnormalised sums as float64
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a.nacc[3 * v + k] = fix_val(a.fn[3 * v + k]);
      a.tacc[3 * v + k] = fix_val(a.ft[3 * v + k]);
    }
  }
  d3 x = dnormalize(dld3(a.nacc, v)), y = dnormalize(dld3(a.tacc, v));
  st3(a.nrm, v, mk((float)x.x, (float)x.y, (float)x.z));
  st3(a.tan, v, mk((float)y.x, (float)y.y, (float)y.z));
}
ADR_KERNEL(__launch_bounds__(256), k_vertex_normalize, VertexNormalizeArgs, vertex_normalize_body)

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0ull;
}

// Zero-fill of up to kFillRanges ranges of 8-byte words in one launch.
__device__ __forceinline__ void fill_multi_body(const FillSet& f, int bid, int nb) {
  const int64_t stride = (int64_t)nb * 256;
  for (int r = 0; r < f.n; ++r)
    for (int64_t i = (int64_t)bid * 256 + threadIdx.x; i < f.len[r]; i += stride) f.p[r][i] = 0ull;
}
ADR_KERNEL(__launch_bounds__(256), k_fill_multi, FillSet, fill_multi_body)

// Two accumulator arrays converted in one launch (the second may be empty).
__device__ __forceinline__ void fix_to_f32_body(const FixToF32Args& a, int bid, int nb) {
  int64_t i = (int64_t)bid * 256 + threadIdx.x;
  const int64_t stride = (int64_t)nb * 256;
  for (; i < a.n + a.n2; i += stride) {
    if (i < a.n) a.dst[i] = (float)acc_val(a.src[i], a.det);
    else a.dst2[i - a.n] = (float)acc_val(a.src2[i - a.n], a.det);
  }
}
ADR_KERNEL(__launch_bounds__(256), k_fix_to_f32, FixToF32Args, fix_to_f32_body)

__device__ __forceinline__ void fix_add_body(const FixAddArgs& a, int bid, int nb) {
  int64_t i = (int64_t)bid * 256 + threadIdx.x;
  const int64_t stride = (int64_t)nb * 256;
  for (; i < a.n; i += stride) a.dst[i] += (float)acc_val(a.src[i], a.det);
}
ADR_KERNEL(__launch_bounds__(256), k_fix_add_f32, FixAddArgs, fix_add_body)

static unsigned grid_for(int64_t n) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

Plan<FillSet> plan_fill_multi(const FillSet& f) {
  int64_t most = 0;
  for (int r = 0; r < f.n; ++r) most = f.len[r] > most ? f.len[r] : most;
  return {f, most == 0 ? 0u : grid_for(most)};
}

hipError_t launch_fill_multi(const FillSet& f, hipStream_t st) {
  ADR_LAUNCH_1(k_fill_multi, plan_fill_multi(f), st);
  return hipGetLastError();
}

Plan<FixToF32Args> plan_fix_to_f32(const unsigned long long* src, float* dst, int64_t n, bool det,
                                   const unsigned long long* src2, float* dst2, int64_t n2) {
  if (n < 0) n = 0;
  if (n2 < 0 || !src2) n2 = 0;
  return {FixToF32Args{src, dst, n, src2, dst2, n2, det}, n + n2 <= 0 ? 0u : grid_for(n + n2)};
}

hipError_t launch_fix_to_f32(const unsigned long long* src, float* dst, int64_t n, bool det, hipStream_t st,
                             const unsigned long long* src2, float* dst2, int64_t n2) {
  ADR_LAUNCH_1(k_fix_to_f32, plan_fix_to_f32(src, dst, n, det, src2, dst2, n2), st);
  return hipGetLastError();
}

__global__ void k_fill(float* __restrict__ p, int64_t n, float val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = val;
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// The vertex frame in three launches: clear the accumulators, sum the face
// terms, normalize.
FramePlans plan_vertex_frame(const MeshD& m, const Scratch& s) {
  const int64_t n = 3 * (int64_t)m.n_pos;
  unsigned long long* fn = s.det ? s.fix_n : nullptr;
  unsigned long long* ft = s.det ? s.fix_t : nullptr;
  FramePlans p;
  FillSet f{};
  f.add(s.det ? fn : reinterpret_cast<unsigned long long*>(s.nacc), n);
  f.add(s.det ? ft : reinterpret_cast<unsigned long long*>(s.tacc), n);
  p.fill = plan_fill_multi(f);
  p.faces = {FaceAccumArgs{m, s.nacc, s.tacc, fn, ft}, (unsigned)((m.n_tri + 255) / 256)};
  p.verts = {VertexNormalizeArgs{m.n_pos, s.nacc, s.tacc, fn, ft, s.nrm, s.tan}, (unsigned)((m.n_pos + 255) / 256)};
  return p;
}

hipError_t launch_vertex_frame(const MeshD& m, const Scratch& s, hipStream_t st) {
  const FramePlans p = plan_vertex_frame(m, s);
  ADR_LAUNCH_1(k_fill_multi, p.fill, st);
  ADR_LAUNCH_1(k_face_accum, p.faces, st);
  ADR_LAUNCH_1(k_vertex_normalize, p.verts, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------- adjoint

// Per vertex: the clip-space gradient of every view through its MVP, the
// gradient of the interpolated world position, and the normalize adjoints
// of the vertex normal and tangent (stored back into dattr for the face pass).
__device__ __forceinline__ void vertex_bwd_body(const VertexBwdArgs& a, int bid, int) {
  const MeshD& m = a.m;
  const ViewsD& v = a.v;
  float* __restrict__ dattr = a.dattr;
  int vi = bid * 256 + threadIdx.x;
  if (vi >= m.n_pos) return;
  f3 g = ld3(dattr, 3 * vi);  // d(world position)
  for (int b = 0; b < v.B; ++b) {
    const float* M = v.mvp + 16 * b;
    const float* dc = a.dclip + 4 * ((int64_t)b * m.n_pos + vi);
    float c0 = dc[0], c1 = dc[1], c2 = dc[2], c3 = dc[3];
    g.x += M[0] * c0 + M[4] * c1 + M[8] * c2 + M[12] * c3;
    g.y += M[1] * c0 + M[5] * c1 + M[9] * c2 + M[13] * c3;
    g.z += M[2] * c0 + M[6] * c1 + M[10] * c2 + M[14] * c3;
  }
  if (a.gpos) atomic_add3(a.gpos, vi, g);
  f3 gn = ld3(dattr, 3 * vi + 1);
  f3 gt = ld3(dattr, 3 * vi + 2);
  if (a.gvn) st3(a.gvn, vi, gn);
  d3 an = dnormalize_bwd(dld3(a.nacc, vi), dmk(gn.x, gn.y, gn.z));
  d3 at = dnormalize_bwd(dld3(a.tacc, vi), dmk(gt.x, gt.y, gt.z));
  st3(dattr, 3 * vi + 1, mk((float)an.x, (float)an.y, (float)an.z));
  st3(dattr, 3 * vi + 2, mk((float)at.x, (float)at.y, (float)at.z));
}
ADR_KERNEL(__launch_bounds__(256), k_vertex_bwd, VertexBwdArgs, vertex_bwd_body)

// Per face: adjoint of the face normal (cross product) and face tangent.
__device__ __forceinline__ void face_bwd_body(const FaceBwdArgs& a, int bid, int) {
  const MeshD& m = a.m;
  const float* __restrict__ dattr = a.dattr;
  int t = bid * 256 + threadIdx.x;
  if (t >= m.n_tri) return;
  int i0 = m.tri[3 * t], i1 = m.tri[3 * t + 1], i2 = m.tri[3 * t + 2];
  FaceFrame f = face_frame(m, t);
  d3 gfn = dld3f(dattr, 3 * i0 + 1) + dld3f(dattr, 3 * i1 + 1) + dld3f(dattr, 3 * i2 + 1);
  d3 g1 = dcross(f.e2, gfn);   // d/d e1 of e1 x e2
  d3 g2 = dcross(gfn, f.e1);   // d/d e2
  if (f.tan_ok) {
    d3 gtf = dld3f(dattr, 3 * i0 + 2) + dld3f(dattr, 3 * i1 + 2) + dld3f(dattr, 3 * i2 + 2);
    double inv = 1.0 / f.r;
    g1 = g1 + (f.d2v * inv) * gtf;
    g2 = g2 - (f.d1v * inv) * gtf;
  }
  const d3 g0 = dmk(-(g1.x + g2.x), -(g1.y + g2.y), -(g1.z + g2.z));
  acc_add3(a.fpos, i1, g1, a.det);
  acc_add3(a.fpos, i2, g2, a.det);
  acc_add3(a.fpos, i0, g0, a.det);
}
ADR_KERNEL(__launch_bounds__(256), k_face_bwd, FaceBwdArgs, face_bwd_body)

// The mesh adjoint in three launches: per vertex, per face (face terms summed
// in float64, fixed point in deterministic mode, into s.fix_pos, which the
// caller has cleared), then the face sums added once per vertex.
MeshBwdPlans plan_mesh_bwd(const MeshD& m, const ViewsD& v, const Scratch& s, float* gpos, float* gvnormal) {
  MeshBwdPlans p;
  const bool any = m.n_pos > 0 && (gpos || gvnormal);
  p.verts = {VertexBwdArgs{m, v, s.dclip, s.dattr, s.nacc, s.tacc, gpos, gvnormal},
             any ? (unsigned)((m.n_pos + 255) / 256) : 0u};
  const bool faces = gpos && m.n_pos > 0 && m.n_tri > 0;
  const int64_t n = 3 * (int64_t)m.n_pos;
  p.faces = {FaceBwdArgs{m, s.dattr, s.fix_pos, s.det}, faces ? (unsigned)((m.n_tri + 255) / 256) : 0u};
  p.add = {FixAddArgs{s.fix_pos, gpos, n, s.det}, faces ? grid_for(n) : 0u};
  return p;
}

hipError_t launch_mesh_bwd(const MeshD& m, const ViewsD& v, const Scratch& s, float* gpos,
                           float* gvnormal, hipStream_t st, bool pos_cleared) {
  const MeshBwdPlans p = plan_mesh_bwd(m, v, s, gpos, gvnormal);
  ADR_LAUNCH_1(k_vertex_bwd, p.verts, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.faces.blocks == 0) return e;
  if (!pos_cleared && (e = launch_fill_u64(s.fix_pos, p.add.a.n, st)) != hipSuccess) return e;
  ADR_LAUNCH_1(k_face_bwd, p.faces, st);
  ADR_LAUNCH_1(k_fix_add_f32, p.add, st);
  return hipGetLastError();
}

// ---- batched launches ----
hipError_t launch_fill_multi_n(const Stage<FillSet>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_fill_multi, s, st);
  return hipGetLastError();
}
hipError_t launch_face_accum_n(const Stage<FaceAccumArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_face_accum, s, st);
  return hipGetLastError();
}
hipError_t launch_vertex_normalize_n(const Stage<VertexNormalizeArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_vertex_normalize, s, st);
  return hipGetLastError();
}
hipError_t launch_fix_to_f32_n(const Stage<FixToF32Args>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_fix_to_f32, s, st);
  return hipGetLastError();
}
hipError_t launch_vertex_bwd_n(const Stage<VertexBwdArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_vertex_bwd, s, st);
  return hipGetLastError();
}
hipError_t launch_face_bwd_n(const Stage<FaceBwdArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_face_bwd, s, st);
  return hipGetLastError();
}
hipError_t launch_fix_add_n(const Stage<FixAddArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_fix_add_f32, s, st);
  return hipGetLastError();
}

}  // namespace adr
