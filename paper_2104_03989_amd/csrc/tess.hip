// Displacement mapping on a tessellated base mesh (Sec. 5.1,
// "Displacement mapping", Eq. 3): every base triangle is split by
// edge-midpoint subdivision, applied `levels` times, into 4^levels
// triangles whose topology is fixed; each step the tessellated positions are
// recomputed from the base mesh and displaced along the interpolated normal:
//   p = sum_c w_c P[v_c],  n = normalize(sum_c w_c N[v_c]),  v_d = p + tex2d(uv) n
// with N the smooth vertex normals of the base mesh and tex2d a bilinear
// lookup in level 0 of the scalar displacement map (wrap u, clamp v).
//
// Canonical numbering (also what the host builder below emits), n = 2^levels:
//   vertices: the base vertices; then, for every base edge (a < b) in
//   lexicographic order, its n-1 interior points ordered from a to b; then,
//   for every base triangle t with corners (c0, c1, c2), its interior lattice
//   points c0 + (i/n)(c1 - c0) + (j/n)(c2 - c0), i, j >= 1, i + j <= n - 1,
//   ordered by i then j;
//   triangles: per base triangle, the "up" triangles (i,j),(i+1,j),(i,j+1)
//   for i + j < n, then the "down" triangles (i+1,j),(i+1,j+1),(i,j+1) for
//   i + j < n - 1, each in i-then-j order (winding kept);
//   UVs: per base triangle its (n+1)(n+2)/2 lattice points (i then j),
//   uv = w0 uv0 + w1 uv1 + w2 uv2 (UV seams stay split);
//   the displacement coordinate of a vertex is its lattice UV in the first
//   base triangle (lowest index) that contains it.
#include <algorithm>
#include <map>
#include <vector>

#include "dev.h"

namespace adr {

// The forward runs in float64 and rounds each displaced position once: the
// rasteriser snaps the float32 positions, so a position that is the correctly
// rounded value of the exact expression keeps the integer coverage
// reproducible.  Normals come straight from the float64 frame accumulators.
struct DBil {
  int idx[4];       // t00, t10, t01, t11
  double fx, fy;
};
__device__ __forceinline__ DBil disp_footprint(const Tex& t, float u, float v) {
  DBil b;
  const int s = t.size;
  double x = (double)u * s - 0.5, y = (double)v * s - 0.5;
  double x0f = floor(x), y0f = floor(y);
  b.fx = x - x0f;
  b.fy = y - y0f;
  int x0 = (int)fmin(fmax(x0f, -1073741824.0), 1073741824.0);
  int y0 = (int)fmin(fmax(y0f, -1073741824.0), 1073741824.0);
  int c0 = x0 & (s - 1);  // x0 mod s (s is a power of two), in [0, s) also for x0 < 0
  int c1 = c0 + 1; if (c1 == s) c1 = 0;
  int r0 = y0 < 0 ? 0 : (y0 > s - 1 ? s - 1 : y0);
  int r1 = y0 + 1 < 0 ? 0 : (y0 + 1 > s - 1 ? s - 1 : y0 + 1);
  b.idx[0] = r0 * s + c0;
  b.idx[1] = r0 * s + c1;
  b.idx[2] = r1 * s + c0;
  b.idx[3] = r1 * s + c1;
  return b;
}

__device__ __forceinline__ double disp_value(const Tex& t, const DBil& b) {
  const float* d = reinterpret_cast<const float*>(t.data);
  double gx = 1.0 - b.fx, gy = 1.0 - b.fy;
  return ((gx * gy * d[b.idx[0]] + b.fx * gy * d[b.idx[1]]) + gx * b.fy * d[b.idx[2]]) +
         b.fx * b.fy * d[b.idx[3]];
}

// Corner weights, base indices and the interpolated unnormalised normal.
struct TessV {
  int k[3];
  double w[3];
  d3 p, m;
};
__device__ __forceinline__ TessV tess_vertex(const MeshD& base, const TessD& ts, const double* nacc, int v) {
  TessV r;
  r.p = dmk(0.0, 0.0, 0.0);
  r.m = r.p;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    r.k[c] = ts.vidx[3 * v + c];
    r.w[c] = ts.w[3 * v + c];
    r.p = r.p + r.w[c] * dld3f(base.pos, r.k[c]);
    r.m = r.m + r.w[c] * dnormalize(dld3(nacc, r.k[c]));
  }
  return r;
}

__global__ void k_tess_fwd(MeshD base, TessD ts, const double* __restrict__ nacc, Tex disp,
                           float* __restrict__ out) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= ts.n) return;
  TessV tv = tess_vertex(base, ts, nacc, v);
  d3 n = dnormalize(tv.m);
  double d = disp_value(disp, disp_footprint(disp, ts.duv[2 * v], ts.duv[2 * v + 1]));
  d3 q = tv.p + d * n;
  out[3 * (int64_t)v] = (float)q.x;
  out[3 * (int64_t)v + 1] = (float)q.y;
  out[3 * (int64_t)v + 2] = (float)q.z;
}

__global__ void k_tess_bwd(MeshD base, TessD ts, const double* __restrict__ nacc, Tex disp,
                           float* __restrict__ gout, float* __restrict__ gbase,
                           float* __restrict__ dattr, float* __restrict__ gdisp) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= ts.n) return;
  d3 g = dld3f(gout, v);
  if (g.x == 0.0 && g.y == 0.0 && g.z == 0.0) return;
  st3(gout, v, mk(0.f, 0.f, 0.f));  // consumed
  TessV tv = tess_vertex(base, ts, nacc, v);
  d3 n = dnormalize(tv.m);
  DBil b = disp_footprint(disp, ts.duv[2 * v], ts.duv[2 * v + 1]);
  double d = disp_value(disp, b);
  d3 gm = dnormalize_bwd(tv.m, d * g);  // d/d(sum w N); N is the normalised vertex normal
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (tv.w[c] == 0.0) continue;
    fatomic3(gbase, tv.k[c], tv.w[c] * g);
    float* da = dattr + 9 * (int64_t)tv.k[c] + 3;
    atomicAdd(da + 0, (float)(tv.w[c] * gm.x));
    atomicAdd(da + 1, (float)(tv.w[c] * gm.y));
    atomicAdd(da + 2, (float)(tv.w[c] * gm.z));
  }
  double gd = ddot(g, n);
  if (gdisp && gd != 0.0) {
    double gx = 1.0 - b.fx, gy = 1.0 - b.fy;
    double ww[4] = {gx * gy, b.fx * gy, gx * b.fy, b.fx * b.fy};
#pragma unroll
    for (int q = 0; q < 4; ++q) atomicAdd(gdisp + b.idx[q], (float)(ww[q] * gd));
  }
}

hipError_t launch_tess_fwd(const MeshD& base, const TessD& ts, const double* nacc, const Tex& disp,
                           float* out, hipStream_t st) {
  if (ts.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tess_fwd, dim3((ts.n + 255) / 256), dim3(256), 0, st, base, ts, nacc, disp, out);
  return hipGetLastError();
}

hipError_t launch_tess_bwd(const MeshD& base, const TessD& ts, const double* nacc, const Tex& disp,
                           float* gout, float* gbase, float* dattr, float* gdisp, hipStream_t st) {
  if (ts.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tess_bwd, dim3((ts.n + 255) / 256), dim3(256), 0, st, base, ts, nacc, disp, gout,
                     gbase, dattr, gdisp);
  return hipGetLastError();
}

// ------------------------------------------------------------- host builder

namespace {

struct Built {
  std::vector<int> vidx, tri, uv_tri;
  std::vector<float> w, duv, uv;
};

// Returns nullptr, or what is wrong with the input.
const char* build(const int32_t* tri, const int32_t* uv_tri, const float* uv, int n_tri, int n_pos, int n_uv,
           int levels, Built* out, int64_t* nv, int64_t* nt, int64_t* nu) {
  if (n_tri < 0 || n_pos < 0) return "negative size";
  if (levels < 0 || levels > 6) return "levels must be in 0..6";
  if (out)
    for (int64_t k = 0; k < 3 * (int64_t)n_tri; ++k)
      if (uv_tri[k] < 0 || uv_tri[k] >= n_uv) return "uv_tri index out of range";
  const int n = 1 << levels;
  std::map<std::pair<int, int>, int> edge_id;
  for (int t = 0; t < n_tri; ++t)
    for (int k = 0; k < 3; ++k) {
      int a = tri[3 * t + k], b = tri[3 * t + (k + 1) % 3];
      if (a < 0 || a >= n_pos || b < 0 || b >= n_pos) return "tri index out of range";
      edge_id.emplace(std::make_pair(std::min(a, b), std::max(a, b)), 0);
    }
  int e = 0;
  for (auto& kv : edge_id) kv.second = e++;
  const int64_t E = (int64_t)edge_id.size();
  const int64_t per_face = (int64_t)(n - 1) * (n - 2) / 2;
  const int64_t npf = (int64_t)(n + 1) * (n + 2) / 2;
  *nv = n_pos + E * (n - 1) + (int64_t)n_tri * per_face;
  *nt = (int64_t)n_tri * n * n;
  *nu = (int64_t)n_tri * npf;
  if (*nv > INT32_MAX || *nt > INT32_MAX || *nu > INT32_MAX) return "tessellated mesh exceeds int32 indexing";
  if (!out) return nullptr;
  out->vidx.assign(3 * *nv, -1);
  out->w.assign(3 * *nv, 0.f);
  out->duv.assign(2 * *nv, 0.f);
  out->tri.resize(3 * *nt);
  out->uv_tri.resize(3 * *nt);
  out->uv.resize(2 * *nu);
  std::vector<char> have_duv(*nv, 0);
  auto local_uv = [&](int i, int j) { return i * (n + 1) - i * (i - 1) / 2 + j; };
  for (int t = 0; t < n_tri; ++t) {
    int c[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
    const float* u0 = uv + 2 * uv_tri[3 * t];
    const float* u1 = uv + 2 * uv_tri[3 * t + 1];
    const float* u2 = uv + 2 * uv_tri[3 * t + 2];
    // vertex of lattice point (i, j) and its weights on (c0, c1, c2)
    auto vertex = [&](int i, int j, int* vi, float* vw) {
      float a = (float)i / n, b = (float)j / n;
      if (i == 0 && j == 0) { vi[0] = vi[1] = vi[2] = c[0]; vw[0] = 1; vw[1] = vw[2] = 0; return c[0]; }
      if (i == n && j == 0) { vi[0] = vi[1] = vi[2] = c[1]; vw[0] = 1; vw[1] = vw[2] = 0; return c[1]; }
      if (i == 0 && j == n) { vi[0] = vi[1] = vi[2] = c[2]; vw[0] = 1; vw[1] = vw[2] = 0; return c[2]; }
      int p = -1, q = -1, kk = 0;
      if (j == 0) { p = c[0]; q = c[1]; kk = i; }
      else if (i == 0) { p = c[0]; q = c[2]; kk = j; }
      else if (i + j == n) { p = c[1]; q = c[2]; kk = j; }
      if (p >= 0) {
        int lo = std::min(p, q), hi = std::max(p, q);
        int k = p == lo ? kk : n - kk;  // steps from lo towards hi
        int id = n_pos + edge_id[std::make_pair(lo, hi)] * (n - 1) + (k - 1);
        vi[0] = lo; vi[1] = hi; vi[2] = hi;
        vw[0] = 1.f - (float)k / n; vw[1] = (float)k / n; vw[2] = 0.f;
        return id;
      }
      int li = 0;
      for (int ii = 1; ii < i; ++ii) li += n - 1 - ii;
      li += j - 1;
      vi[0] = c[0]; vi[1] = c[1]; vi[2] = c[2];
      vw[0] = 1.f - a - b; vw[1] = a; vw[2] = b;
      return (int)(n_pos + E * (n - 1) + (int64_t)t * per_face + li);
    };
    std::vector<int> lat((n + 1) * (n + 1), -1);
    for (int i = 0; i <= n; ++i)
      for (int j = 0; j + i <= n; ++j) {
        int vi[3];
        float vw[3];
        int id = vertex(i, j, vi, vw);
        lat[i * (n + 1) + j] = id;
        // dyadic weights times float32 UVs: the float64 sum is exact, rounded once
        double a = (double)i / n, b = (double)j / n, w0 = 1.0 - a - b;
        float uu = (float)((w0 * u0[0] + a * u1[0]) + b * u2[0]);
        float vv = (float)((w0 * u0[1] + a * u1[1]) + b * u2[1]);
        int64_t lu = (int64_t)t * npf + local_uv(i, j);
        out->uv[2 * lu] = uu;
        out->uv[2 * lu + 1] = vv;
        if (!have_duv[id]) {
          have_duv[id] = 1;
          for (int k = 0; k < 3; ++k) {
            out->vidx[3 * (int64_t)id + k] = vi[k];
            out->w[3 * (int64_t)id + k] = vw[k];
          }
          out->duv[2 * (int64_t)id] = uu;
          out->duv[2 * (int64_t)id + 1] = vv;
        }
      }
    int64_t tb = (int64_t)t * n * n, k = 0;
    auto put = [&](int i0, int j0, int i1, int j1, int i2, int j2) {
      int64_t o = 3 * (tb + k++);
      out->tri[o] = lat[i0 * (n + 1) + j0];
      out->tri[o + 1] = lat[i1 * (n + 1) + j1];
      out->tri[o + 2] = lat[i2 * (n + 1) + j2];
      out->uv_tri[o] = (int)(t * npf + local_uv(i0, j0));
      out->uv_tri[o + 1] = (int)(t * npf + local_uv(i1, j1));
      out->uv_tri[o + 2] = (int)(t * npf + local_uv(i2, j2));
    };
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n - i; ++j) put(i, j, i + 1, j, i, j + 1);
    for (int i = 0; i < n - 1; ++i)
      for (int j = 0; j < n - 1 - i; ++j) put(i + 1, j, i + 1, j + 1, i, j + 1);
  }
  return nullptr;
}

}  // namespace

}  // namespace adr

using namespace adr;

extern "C" adr_status adr_tess_counts(const int32_t* tri, int32_t n_tri, int32_t n_pos, int32_t levels,
                                      int64_t* n_vert, int64_t* n_tri_out, int64_t* n_uv_out) {
  if ((n_tri > 0 && !tri) || !n_vert || !n_tri_out || !n_uv_out)
    return report(ADR_E_INVALID, "tess_counts: tri and the three outputs are required");
  const char* why = build(tri, nullptr, nullptr, n_tri, n_pos, 0, levels, nullptr, n_vert, n_tri_out, n_uv_out);
  return why ? report(ADR_E_INVALID, why) : ADR_OK;
}

extern "C" adr_status adr_tess_build(const int32_t* tri, const int32_t* uv_tri, const float* uv,
                                     int32_t n_tri, int32_t n_pos, int32_t n_uv, int32_t levels, int32_t* vidx,
                                     float* w, float* duv, int32_t* tess_tri, float* tess_uv,
                                     int32_t* tess_uv_tri) {
  if (n_tri > 0 && (!tri || !uv_tri || !uv || !vidx || !w || !duv || !tess_tri || !tess_uv || !tess_uv_tri))
    return report(ADR_E_INVALID, "tess_build: input and output arrays are required");
  Built b;
  int64_t nv, nt, nu;
  if (const char* why = build(tri, uv_tri, uv, n_tri, n_pos, n_uv, levels, &b, &nv, &nt, &nu))
    return report(ADR_E_INVALID, why);
  std::copy(b.vidx.begin(), b.vidx.end(), vidx);
  std::copy(b.w.begin(), b.w.end(), w);
  std::copy(b.duv.begin(), b.duv.end(), duv);
  std::copy(b.tri.begin(), b.tri.end(), tess_tri);
  std::copy(b.uv.begin(), b.uv.end(), tess_uv);
  std::copy(b.uv_tri.begin(), b.uv_tri.end(), tess_uv_tri);
  return ADR_OK;
}
