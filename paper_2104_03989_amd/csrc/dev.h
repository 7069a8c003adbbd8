// Device-side helpers: small vector algebra, the XCD-aware block order and
// texture addressing.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace adr {

struct f3 {
  float x, y, z;
};
__device__ __forceinline__ f3 mk(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator-(f3 a) { return {-a.x, -a.y, -a.z}; }
__device__ __forceinline__ f3 operator*(float s, f3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ f3 operator*(f3 a, f3 b) { return {a.x * b.x, a.y * b.y, a.z * b.z}; }
__device__ __forceinline__ f3& operator+=(f3& a, f3 b) {
  a.x += b.x; a.y += b.y; a.z += b.z;
  return a;
}
__device__ __forceinline__ f3& operator-=(f3& a, f3 b) {
  a.x -= b.x; a.y -= b.y; a.z -= b.z;
  return a;
}
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float sum3(f3 a) { return a.x + a.y + a.z; }
__device__ __forceinline__ f3 ld3(const float* p, int i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }
__device__ __forceinline__ void st3(float* p, int64_t i, f3 v) {
  p[3 * i] = v.x; p[3 * i + 1] = v.y; p[3 * i + 2] = v.z;
}
__device__ __forceinline__ void atomic_add3(float* p, int64_t i, f3 v) {
  atomicAdd(p + 3 * i, v.x);
  atomicAdd(p + 3 * i + 1, v.y);
  atomicAdd(p + 3 * i + 2, v.z);
}

// x / |x|; vectors with |x|^2 <= 1e-20 pass unchanged.
__device__ __forceinline__ f3 safe_normalize(f3 x) {
  float n2 = dot(x, x);
  return n2 > 1e-20f ? rsqrtf(n2) * x : x;
}
// Adjoint of safe_normalize at x for the output gradient g.
__device__ __forceinline__ f3 safe_normalize_bwd(f3 x, f3 g) {
  float n2 = dot(x, x);
  if (!(n2 > 1e-20f)) return g;
  float inv = rsqrtf(n2);
  f3 y = inv * x;
  return inv * (g - dot(g, y) * y);
}

// float64 vectors (vertex frame, displacement).
struct d3 {
  double x, y, z;
};
__device__ __forceinline__ d3 dmk(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 operator*(double s, d3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double ddot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 dcross(d3 a, d3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ d3 dld3f(const float* p, int i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }
__device__ __forceinline__ d3 dld3(const double* p, int i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }
__device__ __forceinline__ void datomic3(double* p, int64_t i, d3 v) {
  atomicAdd(p + 3 * i, v.x);
  atomicAdd(p + 3 * i + 1, v.y);
  atomicAdd(p + 3 * i + 2, v.z);
}
__device__ __forceinline__ void fatomic3(float* p, int64_t i, d3 v) {
  atomicAdd(p + 3 * i, (float)v.x);
  atomicAdd(p + 3 * i + 1, (float)v.y);
  atomicAdd(p + 3 * i + 2, (float)v.z);
}
// x / |x| in float64; |x|^2 <= 1e-20 passes unchanged.
__device__ __forceinline__ d3 dnormalize(d3 x) {
  double n2 = ddot(x, x);
  return n2 > 1e-20 ? (1.0 / sqrt(n2)) * x : x;
}
__device__ __forceinline__ d3 dnormalize_bwd(d3 x, d3 g) {
  double n2 = ddot(x, x);
  if (!(n2 > 1e-20)) return g;
  double inv = 1.0 / sqrt(n2);
  d3 y = inv * x;
  return inv * (g - ddot(g, y) * y);
}

// Deterministic accumulation: a value is scaled by 2^40, rounded to a 64-bit
// integer and added with an integer atomic; integer (wrap-around) addition
// does not depend on the order of the additions, so the sum is the same on
// every run.  Resolution 2^-40 (9.1e-13), range +-2^23 (8.4e6) per sum.
constexpr double kFixScale = 1099511627776.0;
__device__ __forceinline__ void fix_add(unsigned long long* p, double v) {
  atomicAdd(p, (unsigned long long)__double2ll_rn(v * kFixScale));
}
__device__ __forceinline__ double fix_val(unsigned long long x) { return (double)(long long)x / kFixScale; }
__device__ __forceinline__ void fix_add3(unsigned long long* p, int64_t i, d3 v) {
  fix_add(p + 3 * i, v.x);
  fix_add(p + 3 * i + 1, v.y);
  fix_add(p + 3 * i + 2, v.z);
}

// Vertex-side adjoint accumulators: 8-byte slots holding fixed point in
// deterministic mode and float64 otherwise (float32 sums of per-pixel terms
// cancel badly where the tangent frame is ill-conditioned, e.g. at UV poles).
__device__ __forceinline__ void acc_add(unsigned long long* p, double v, bool det) {
  if (det) fix_add(p, v);
  else atomicAdd(reinterpret_cast<double*>(p), v);
}
__device__ __forceinline__ void acc_add3(unsigned long long* p, int64_t i, d3 v, bool det) {
  acc_add(p + 3 * i, v.x, det);
  acc_add(p + 3 * i + 1, v.y, det);
  acc_add(p + 3 * i + 2, v.z, det);
}
__device__ __forceinline__ double acc_val(unsigned long long x, bool det) {
  return det ? fix_val(x) : __longlong_as_double((long long)x);
}

// Batched launches: one grid over the blocks of n items, item k owning
// blocks [start[k], start[k+1]) (an item may own none).  The item of block
// bid is the last k with start[k] <= bid, found by a binary search on
// values that are the same for the whole block.  The tables are read through
// the constant address space (they do not change while a kernel runs), so
// the argument blocks load into scalar registers once and the pointers in
// them are known to be global, as with kernel arguments.
#define ADR_CONST __attribute__((address_space(4)))
__device__ __forceinline__ int batch_item(const ADR_CONST int* start, int n, int bid) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= bid) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <class T>
inline const ADR_CONST T* const_tab(const T* p) {
  return (const ADR_CONST T*)p;
}

// A kernel written as a body BODY(args, block, blocks) with two entry
// points: NAME runs one argument block over its grid, NAME_n the batched
// launch over the items of a stage (each block runs its item's body with
// the block's index within the item's range).
#define ADR_KERNEL(ATTR, NAME, ARGS, BODY)                                                             \
  __global__ ATTR void NAME(ARGS a) { BODY(a, (int)blockIdx.x, (int)gridDim.x); }                   \
  __global__ ATTR void NAME##_n(const ADR_CONST ARGS* tab, const ADR_CONST int* start, int n) {     \
    const int it_ = batch_item(start, n, (int)blockIdx.x);                                            \
    const int s0_ = start[it_];                                                                       \
    BODY(*(const ARGS*)&tab[it_], (int)blockIdx.x - s0_, start[it_ + 1] - s0_);                       \
  }

// Launches the single entry point of a kernel with a plan's argument block.
#define ADR_LAUNCH_1(NAME, PLAN, ST)                                                          \
  do {                                                                                        \
    if ((PLAN).blocks > 0) hipLaunchKernelGGL(NAME, dim3((PLAN).blocks), dim3(256), 0, ST, (PLAN).a); \
  } while (0)

// Launches the batched entry point of a kernel over a stage.
#define ADR_LAUNCH_N(NAME, STAGE, ST)                                                                 \
  do {                                                                                                 \
    if ((STAGE).total > 0)                                                                             \
      hipLaunchKernelGGL(NAME##_n, dim3((unsigned)(STAGE).total), dim3(256), 0, ST,                    \
                         const_tab((STAGE).tab), const_tab((STAGE).start), (STAGE).n);                 \
  } while (0)

// Blocks are dispatched round-robin over the 8 XCDs of an MI355X; each XCD
// has its own L2.  This maps the hardware block id to a logical tile id so
// that every XCD works through one contiguous range of tiles (neighbouring
// pixels share texels and triangles through that XCD's L2).
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  int xcd = bid & 7, idx = bid >> 3;
  int per = nb >> 3, rem = nb & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// Pixel of thread `tid` (0..255) in 16x16 tile `tile`: each 64-wide wave
// covers an 8x8 block.
struct Pix {
  int b, i, j;
  bool ok;
};
__device__ __forceinline__ Pix tile_pixel(int tile, int tid, int tiles_x, int tiles_y, int W, int H) {
  int per_view = tiles_x * tiles_y;
  Pix p;
  p.b = tile / per_view;
  int r = tile - p.b * per_view;
  int ty = r / tiles_x, tx = r - ty * tiles_x;
  int wave = tid >> 6, lane = tid & 63;
  p.i = tx * 16 + (wave & 1) * 8 + (lane & 7);
  p.j = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
  p.ok = p.i < W && p.j < H;
  return p;
}

// Nontemporal float4 accesses (the streaming cache policy) for data that is
// touched once per step or handed to the next kernel only: they keep such
// streams from evicting the working sets of the other kernels.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_nt(const float4* p) {
  const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_nt(float4* p, float4 x) {
  const nt_f4 v = {x.x, x.y, x.z, x.w};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_f4*>(p));
}

// ---- textures ----

__device__ __forceinline__ f3 tex_fetch(const Tex& t, int texel) {
  if (t.fmt == ADR_TEX_RGBA8) {
    uchar4 q = reinterpret_cast<const uchar4*>(t.data)[texel];
    const float s = 1.0f / 255.0f;
    return {q.x * s, q.y * s, q.z * s};
  }
  const float* d = reinterpret_cast<const float*>(t.data);
  if (t.channels == 3) return ld3(d, texel);
  float v = d[texel];
  return {v, 0.f, 0.f};
}

// Texture coordinates travel as float32 pairs (u, ul) with u + ul the
// coordinate to about float64 precision: on a 2048^2 map one float32 unit of
// u is 1.2e-4 texels, which moves a lookup of a high-frequency map by more
// than the forward tolerance.  Texel coordinate of u + ul on a level of s
// texels: the cell x0 and the fraction fx of u s - 1/2 + ul s.  u s is exact
// (a power-of-two scale) and so is u s - 1/2 when u s >= 1 (otherwise the
// result is below 1 in magnitude and within 2^-25 of it, or u lies outside
// the map and wraps); the fraction then gains the low part and is moved back
// into [0, 1] across a cell boundary.
__device__ __forceinline__ void texel_coord(float u, float ul, int s, int& x0, float& fx) {
  const float x = u * (float)s - 0.5f;
  float xf = floorf(x);
  float f = (x - xf) + ul * (float)s;
  const float adj = floorf(f);  // -1 or 0 (or 1 at the upper boundary)
  f -= adj;
  xf += adj;
  fx = f;
  x0 = (int)fminf(fmaxf(xf, -1073741824.f), 1073741824.f);
}

// Bilinear footprint of (u + ul, v + vl) at level l: four texel indices and
// weights.
struct Bil {
  int idx[4];      // t00, t10, t01, t11
  float fx, fy;    // fractional position
  int s;           // level size
};
__device__ __forceinline__ Bil bil_footprint(const Tex& t, int l, float u, float v, float ul, float vl) {
  Bil b;
  int s = t.size >> l;
  if (s < 1) s = 1;
  b.s = s;
  int x0, y0;
  texel_coord(u, ul, s, x0, b.fx);
  texel_coord(v, vl, s, y0, b.fy);
  int c0 = x0 & (s - 1);  // x0 mod s (s is a power of two), in [0, s) also for x0 < 0
  int c1 = c0 + 1; if (c1 == s) c1 = 0;
  int r0 = y0 < 0 ? 0 : (y0 > s - 1 ? s - 1 : y0);
  int r1 = y0 + 1 < 0 ? 0 : (y0 + 1 > s - 1 ? s - 1 : y0 + 1);
  int o = t.off[l];
  b.idx[0] = o + r0 * s + c0;
  b.idx[1] = o + r0 * s + c1;
  b.idx[2] = o + r1 * s + c0;
  b.idx[3] = o + r1 * s + c1;
  return b;
}

// The low parts of a coordinate pair in one float (texture-sample records):
// two int16 of ul 2^38 and vl 2^38.  |ul| is at most half a float32 unit of
// u, 2^-25 for u in [0, 1): the scale keeps 2^-38 (1.5e-8 texels of a 4096^2
// level) and saturates only for coordinates beyond [-2, 2].
__device__ __forceinline__ float pack_lo(float ul, float vl) {
  const float k = 274877906944.f;  // 2^38
  const int a = (int)rintf(fminf(fmaxf(ul * k, -32767.f), 32767.f));
  const int b = (int)rintf(fminf(fmaxf(vl * k, -32767.f), 32767.f));
  return __uint_as_float(((uint32_t)a & 0xFFFFu) | ((uint32_t)b << 16));
}
__device__ __forceinline__ void unpack_lo(float x, float& ul, float& vl) {
  const uint32_t q = __float_as_uint(x);
  const float k = 1.f / 274877906944.f;
  ul = (float)(int)(int16_t)(q & 0xFFFFu) * k;
  vl = (float)(int)(int16_t)(q >> 16) * k;
}

struct BilVal {
  f3 val, du, dv;  // value and derivatives w.r.t. u and v
};
__device__ __forceinline__ BilVal bil_eval(const Tex& t, const Bil& b) {
  f3 t00 = tex_fetch(t, b.idx[0]), t10 = tex_fetch(t, b.idx[1]);
  f3 t01 = tex_fetch(t, b.idx[2]), t11 = tex_fetch(t, b.idx[3]);
  float fx = b.fx, fy = b.fy;
  BilVal r;
  f3 a = t00 + fx * (t10 - t00);
  f3 c = t01 + fx * (t11 - t01);
  r.val = a + fy * (c - a);
  float s = (float)b.s;
  r.du = s * ((1.f - fy) * (t10 - t00) + fy * (t11 - t01));
  r.dv = s * ((1.f - fx) * (t01 - t00) + fx * (t11 - t10));
  return r;
}

// Level selection of a trilinear lookup.
struct Lod {
  int l0;
  float f;         // weight of level l0 + 1
  bool has1;       // l0 + 1 exists
  bool grad;       // the LOD is differentiable here (not clamped, max > 0)
  bool use_x;      // max taken from the x derivative
  float m;         // max(|duv/dx|^2, |duv/dy|^2) in level-0 texels
};
__device__ __forceinline__ Lod lod_select(const Tex& t, float ux, float vx, float uy, float vy) {
  float S = (float)t.size;
  float sx2 = (ux * S) * (ux * S) + (vx * S) * (vx * S);
  float sy2 = (uy * S) * (uy * S) + (vy * S) * (vy * S);
  Lod r;
  r.use_x = sx2 >= sy2;
  float m = r.use_x ? sx2 : sy2;
  r.m = m;
  float lod_raw = m > 0.f ? 0.5f * log2f(m) : 0.f;
  float L1 = (float)(t.levels - 1);
  r.grad = m > 0.f && lod_raw >= 0.f && lod_raw <= L1;
  float lod = fminf(fmaxf(lod_raw, 0.f), L1);
  int l0 = (int)floorf(lod);
  if (l0 > t.levels - 1) l0 = t.levels - 1;
  r.l0 = l0;
  r.has1 = l0 + 1 < t.levels;
  r.f = r.has1 ? lod - (float)l0 : 0.f;
  return r;
}

struct TriSample {
  f3 val;
  f3 du, dv;       // d value / d(u, v)
  f3 dl;           // value at level l0 + 1 minus value at l0 (zero without a second level)
};
// The bilinear footprints of a trilinear lookup: level l0, and l0 + 1 when
// the lookup has it.  They depend on the map's size and level count only, so
// maps of one size share them.
struct TriFoot {
  Bil b0, b1;
};
__device__ __forceinline__ TriFoot tri_foot(const Tex& t, float u, float v, float ul, float vl, const Lod& L) {
  TriFoot F;
  F.b0 = bil_footprint(t, L.l0, u, v, ul, vl);
  if (L.has1) F.b1 = bil_footprint(t, L.l0 + 1, u, v, ul, vl);
  return F;
}
__device__ __forceinline__ TriSample tri_eval(const Tex& t, const TriFoot& F, const Lod& L) {
  // a one-texel map (a constant material channel): every footprint is that
  // texel, with zero derivatives and no second level -- what the general
  // path computes, without its arithmetic
  if (t.size == 1) return TriSample{tex_fetch(t, t.off[0]), mk(0.f, 0.f, 0.f), mk(0.f, 0.f, 0.f), mk(0.f, 0.f, 0.f)};
  BilVal a = bil_eval(t, F.b0);
  TriSample r{a.val, a.du, a.dv, mk(0.f, 0.f, 0.f)};
  if (L.has1) {
    BilVal c = bil_eval(t, F.b1);
    float f = L.f;
    r.dl = c.val - a.val;
    r.val = a.val + f * (c.val - a.val);
    r.du = a.du + f * (c.du - a.du);
    r.dv = a.dv + f * (c.dv - a.dv);
  }
  return r;
}
__device__ __forceinline__ TriSample tex_trilinear(const Tex& t, float u, float v, float ul, float vl,
                                                   const Lod& L) {
  if (t.size == 1) return tri_eval(t, TriFoot{}, L);
  return tri_eval(t, tri_foot(t, u, v, ul, vl, L), L);
}
// Two maps of one size and level count share their level selection and
// footprints.
__device__ __forceinline__ bool same_layout(const Tex& a, const Tex& b) {
  return a.size == b.size && a.levels == b.levels;
}

// One bias-corrected Adam update (Sec. 5.3); c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__device__ __forceinline__ float adam1(float& p, float g, float& m, float& v, float b1, float b2,
                                       float c1, float c2, float lr, float eps) {
  m = b1 * m + (1.f - b1) * g;
  v = b2 * v + (1.f - b2) * g * g;
  float mh = m * c1, vh = v * c2;
  p = p - lr * mh / (sqrtf(vh) + eps);
  return p;
}

// Clip coordinates of vertex vi in view b in float64 from the float32
// position and the view matrix (in float64, converted once per call by the
// transform stage), as the transform stage computes them for the
// rasterizer: each product of two float32 values is exact in float64, so
// the sums round the same way whether or not a multiply is fused with them.
// Recomputed where needed (3 vertices per pixel) instead of gathered from a
// [views, vertices] float64 array.
__device__ __forceinline__ double4 clip_from(const double* __restrict__ M, double px, double py, double pz) {
  double d[4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    d[r] = ((M[4 * r] * px + M[4 * r + 1] * py) + M[4 * r + 2] * pz) + M[4 * r + 3];
  return make_double4(d[0], d[1], d[2], d[3]);
}
__device__ __forceinline__ double4 clip_d(const float* __restrict__ pos, const double* __restrict__ mvpd, int b,
                                          int vi) {
  return clip_from(mvpd + 16 * b, pos[3 * vi], pos[3 * vi + 1], pos[3 * vi + 2]);
}

}  // namespace adr
