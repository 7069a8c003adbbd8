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
__global__ void k_face_accum(MeshD m, double* __restrict__ nacc, double* __restrict__ tacc,
                             unsigned long long* __restrict__ fn, unsigned long long* __restrict__ ft) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_tri) return;
  FaceFrame f = face_frame(m, t);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int v = m.tri[3 * t + k];
    if (fn) {
      fix_add3(fn, v, f.fn);
      if (f.tan_ok) fix_add3(ft, v, f.tf);
    } else {
      datomic3(nacc, v, f.fn);
      if (f.tan_ok) datomic3(tacc, v, f.tf);
    }
  }
}

__global__ void k_vertex_normalize(int n, double* __restrict__ nacc, double* __restrict__ tacc,
                                   const unsigned long long* __restrict__ fn,
                                   const unsigned long long* __restrict__ ft, float* __restrict__ nrm,
                                   float* __restrict__ tan) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (fn) {  // the adjoint reads the unnormalised sums as float64
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      nacc[3 * v + k] = fix_val(fn[3 * v + k]);
      tacc[3 * v + k] = fix_val(ft[3 * v + k]);
    }
  }
  d3 a = dnormalize(dld3(nacc, v)), b = dnormalize(dld3(tacc, v));
  st3(nrm, v, mk((float)a.x, (float)a.y, (float)a.z));
  st3(tan, v, mk((float)b.x, (float)b.y, (float)b.z));
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0ull;
}

// Zero-fill of up to kFillRanges ranges of 8-byte words in one launch.
__global__ void k_fill_multi(FillSet f) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int r = 0; r < f.n; ++r)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f.len[r]; i += stride) f.p[r][i] = 0ull;
}

// Two accumulator arrays converted in one launch (the second may be empty).
__global__ void k_fix_to_f32(const unsigned long long* __restrict__ src, float* __restrict__ dst, int64_t n,
                             const unsigned long long* __restrict__ src2, float* __restrict__ dst2, int64_t n2,
                             bool det) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n + n2; i += stride) {
    if (i < n) dst[i] = (float)acc_val(src[i], det);
    else dst2[i - n] = (float)acc_val(src2[i - n], det);
  }
}

__global__ void k_fix_add_f32(const unsigned long long* __restrict__ src, float* __restrict__ dst, int64_t n,
                              bool det) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] += (float)acc_val(src[i], det);
}

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

hipError_t launch_fill_multi(const FillSet& f, hipStream_t st) {
  int64_t most = 0;
  for (int r = 0; r < f.n; ++r) most = f.len[r] > most ? f.len[r] : most;
  if (most == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_multi, dim3(grid_for(most)), dim3(256), 0, st, f);
  return hipGetLastError();
}


hipError_t launch_fix_to_f32(const unsigned long long* src, float* dst, int64_t n, bool det, hipStream_t st,
                             const unsigned long long* src2, float* dst2, int64_t n2) {
  if (n < 0) n = 0;
  if (n2 < 0 || !src2) n2 = 0;
  if (n + n2 <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fix_to_f32, dim3(grid_for(n + n2)), dim3(256), 0, st, src, dst, n, src2, dst2, n2, det);
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

hipError_t launch_vertex_frame(const MeshD& m, const Scratch& s, hipStream_t st) {
  int64_t n = 3 * (int64_t)m.n_pos;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  unsigned long long* fn = s.det ? s.fix_n : nullptr;
  unsigned long long* ft = s.det ? s.fix_t : nullptr;
  FillSet f{};
  f.add(s.det ? fn : reinterpret_cast<unsigned long long*>(s.nacc), n);
  f.add(s.det ? ft : reinterpret_cast<unsigned long long*>(s.tacc), n);
  hipError_t e = launch_fill_multi(f, st);
  if (e != hipSuccess) return e;
  if (m.n_tri > 0) {
    hipLaunchKernelGGL(k_face_accum, dim3((m.n_tri + 255) / 256), dim3(256), 0, st, m, s.nacc, s.tacc, fn, ft);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_vertex_normalize, dim3((m.n_pos + 255) / 256), dim3(256), 0, st, m.n_pos,
                     s.nacc, s.tacc, fn, ft, s.nrm, s.tan);
  return hipGetLastError();
}

// ---------------------------------------------------------------- adjoint

// Per vertex: the clip-space gradient of every view through its MVP, the
// gradient of the interpolated world position, and the normalize adjoints
// of the vertex normal and tangent (stored back into dattr for the face pass).
__global__ void k_vertex_bwd(MeshD m, ViewsD v, const float* __restrict__ dclip,
                             float* __restrict__ dattr, const double* __restrict__ nacc,
                             const double* __restrict__ tacc, float* __restrict__ gpos,
                             float* __restrict__ gvn) {
  int vi = blockIdx.x * blockDim.x + threadIdx.x;
  if (vi >= m.n_pos) return;
  f3 g = ld3(dattr, 3 * vi);  // d(world position)
  for (int b = 0; b < v.B; ++b) {
    const float* M = v.mvp + 16 * b;
    const float* dc = dclip + 4 * ((int64_t)b * m.n_pos + vi);
    float c0 = dc[0], c1 = dc[1], c2 = dc[2], c3 = dc[3];
    g.x += M[0] * c0 + M[4] * c1 + M[8] * c2 + M[12] * c3;
    g.y += M[1] * c0 + M[5] * c1 + M[9] * c2 + M[13] * c3;
    g.z += M[2] * c0 + M[6] * c1 + M[10] * c2 + M[14] * c3;
  }
  if (gpos) atomic_add3(gpos, vi, g);
  f3 gn = ld3(dattr, 3 * vi + 1);
  f3 gt = ld3(dattr, 3 * vi + 2);
  if (gvn) st3(gvn, vi, gn);
  d3 an = dnormalize_bwd(dld3(nacc, vi), dmk(gn.x, gn.y, gn.z));
  d3 at = dnormalize_bwd(dld3(tacc, vi), dmk(gt.x, gt.y, gt.z));
  st3(dattr, 3 * vi + 1, mk((float)an.x, (float)an.y, (float)an.z));
  st3(dattr, 3 * vi + 2, mk((float)at.x, (float)at.y, (float)at.z));
}

// Per face: adjoint of the face normal (cross product) and face tangent.
__global__ void k_face_bwd(MeshD m, const float* __restrict__ dattr, unsigned long long* __restrict__ fpos,
                           bool det) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
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
  acc_add3(fpos, i1, g1, det);
  acc_add3(fpos, i2, g2, det);
  acc_add3(fpos, i0, g0, det);
}

hipError_t launch_mesh_bwd(const MeshD& m, const ViewsD& v, const Scratch& s, float* gpos,
                           float* gvnormal, hipStream_t st, bool pos_cleared) {
  hipLaunchKernelGGL(k_vertex_bwd, dim3((m.n_pos + 255) / 256), dim3(256), 0, st, m, v, s.dclip,
                     s.dattr, s.nacc, s.tacc, gpos, gvnormal);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !gpos || m.n_tri == 0) return e;
  // face terms summed in float64 (fixed point in deterministic mode), then
  // added once per vertex
  const int64_t n = 3 * (int64_t)m.n_pos;
  if (!pos_cleared && (e = launch_fill_u64(s.fix_pos, n, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_face_bwd, dim3((m.n_tri + 255) / 256), dim3(256), 0, st, m, s.dattr, s.fix_pos, s.det);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_fix_add_f32, dim3(grid_for(n)), dim3(256), 0, st, s.fix_pos, gpos, n, s.det);
  return hipGetLastError();
}

}  // namespace adr
