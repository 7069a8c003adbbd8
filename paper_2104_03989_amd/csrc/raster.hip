// Fixed-point rasterization of B views of a triangle mesh (the visibility
// stage of the paper's pipeline, Sec. 3 and Sec. 5.2, which the paper runs on
// fixed-function hardware through Laine et al. 2020).  Integer rules:
//   clip = MVP [p,1] in float32 as ((m0 x + m1 y) + m2 z) + m3, no contraction;
//   X = rint(((x/w) 0.5 + 0.5) W 256), Y likewise, Z = clamp(rint(((z/w) 0.5 +
//   0.5) 2^24), 0, 2^24-1), every step rounded to float32;
//   a vertex with w <= 1e-6 or |x/w|, |y/w| > 8 drops its triangles, as does a
//   zero integer area; clockwise triangles are reoriented, nothing is culled;
//   coverage at pixel centres (256 i + 128, 256 j + 128) by integer edge
//   functions with the top-left rule; depth = clamp(rint((Z0 + a dx) + b dy))
//   from the float32 plane a = (dz1 dy2 - dz2 dy1)/A, b = (dz2 dx1 - dz1 dx2)/A;
//   key = depth << 32 | (triangle + 1), smallest key wins.
// Everything here is integer or correctly rounded float32 in a fixed order,
// so the visibility buffer is bit-exact and independent of launch order.
//
// Work split: a triangle whose pixel bounding box holds at most `tiny` (64
// by default, a per-context setting) pixel centres is walked by one thread
// (most triangles of dense meshes are pixel-sized); one of up to `med` (4096)
// goes to a queue whose entries a second
// kernel spreads over all waves of the chip, one triangle per wave at a time;
// larger ones go to a per-view list that a third kernel bins against 16x16
// tiles in LDS and resolves one pixel per thread.
//
// Depth peeling (Sec. 5.2, "Order-independent transparency"): with a floor
// buffer (the previous layer's keys) a fragment counts only if its key is
// strictly greater than the floor key of its pixel, so a pass keeps the
// nearest fragment behind the previous layer.
// This file is compiled with -ffp-contract=off.
#include "dev.h"

#pragma clang fp contract(off)

namespace adr {

__device__ __forceinline__ float fmul(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ float fadd(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ float fsub(float a, float b) { return __fsub_rn(a, b); }

// Snapped integer coordinates (from the float32 clip coordinates of the
// rules above) and float64 clip coordinates for interpolation.
__device__ __forceinline__ void xform_body(const XformArgs& a, int bid, int) {
  const MeshD& m = a.m;
  const ViewsD& v = a.v;
  int gid = bid * 256 + threadIdx.x;
  if (gid < 16 * v.B) a.mvpd[gid] = (double)v.mvp[gid];
  if (gid >= v.B * m.n_pos) return;
  int b = gid / m.n_pos, vi = gid - b * m.n_pos;
  const float* M = v.mvp + 16 * b;
  float px = m.pos[3 * vi], py = m.pos[3 * vi + 1], pz = m.pos[3 * vi + 2];
  float c[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float t = fadd(fmul(M[4 * r + 0], px), fmul(M[4 * r + 1], py));
    t = fadd(t, fmul(M[4 * r + 2], pz));
    c[r] = fadd(t, M[4 * r + 3]);
  }
  int4 s = make_int4(0, 0, 0, 0);
  float w = c[3];
  if (w > 1e-6f) {
    float qx = __fdiv_rn(c[0], w), qy = __fdiv_rn(c[1], w), qz = __fdiv_rn(c[2], w);
    if (fabsf(qx) <= 8.0f && fabsf(qy) <= 8.0f && !isnan(qz)) {
      float sx = fmul(fadd(fmul(qx, 0.5f), 0.5f), (float)(v.W * 256));
      float sy = fmul(fadd(fmul(qy, 0.5f), 0.5f), (float)(v.H * 256));
      float sz = fmul(fadd(fmul(qz, 0.5f), 0.5f), 16777216.0f);
      float rz = rintf(sz);
      s.x = (int)rintf(sx);
      s.y = (int)rintf(sy);
      s.z = rz <= 0.0f ? 0 : (rz >= (float)kZMax ? kZMax : (int)rz);
      s.w = 1;
    }
  }
  a.snap[gid] = s;
}
ADR_KERNEL(__launch_bounds__(256), k_xform, XformArgs, xform_body)

// Oriented integer setup of one triangle in one view.
struct Setup {
  int X[3], Y[3], Z0;
  float a, b;
  int64_t eA[3], eB[3], eC[3];  // E_k(P) = eA P.x + eB P.y + eC
  int bias[3];                  // 0 for top-left edges, 1 otherwise
  int flip;
};

__device__ __forceinline__ bool setup_tri(const int4* __restrict__ snapv, int3 c, Setup& s) {
  int4 v0 = snapv[c.x], v1 = snapv[c.y], v2 = snapv[c.z];
  if (!v0.w || !v1.w || !v2.w) return false;
  int64_t A = (int64_t)(v1.x - v0.x) * (v2.y - v0.y) - (int64_t)(v1.y - v0.y) * (v2.x - v0.x);
  if (A == 0) return false;
  s.flip = A < 0;
  if (s.flip) {
    int4 t = v1; v1 = v2; v2 = t;
  }
  s.X[0] = v0.x; s.X[1] = v1.x; s.X[2] = v2.x;
  s.Y[0] = v0.y; s.Y[1] = v1.y; s.Y[2] = v2.y;
  s.Z0 = v0.z;
  float dx1 = (float)(v1.x - v0.x), dy1 = (float)(v1.y - v0.y);
  float dx2 = (float)(v2.x - v0.x), dy2 = (float)(v2.y - v0.y);
  float dz1 = (float)(v1.z - v0.z), dz2 = (float)(v2.z - v0.z);
  float Af = fsub(fmul(dx1, dy2), fmul(dy1, dx2));
  float nx = fsub(fmul(dz1, dy2), fmul(dz2, dy1));
  float ny = fsub(fmul(dz2, dx1), fmul(dz1, dx2));
  s.a = __fdiv_rn(nx, Af);
  s.b = __fdiv_rn(ny, Af);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int j = k == 2 ? 0 : k + 1, l = k == 0 ? 2 : k - 1;
    int64_t dx = (int64_t)s.X[l] - s.X[j], dy = (int64_t)s.Y[l] - s.Y[j];
    // E = dx (Py - Yj) - dy (Px - Xj)
    s.eA[k] = -dy;
    s.eB[k] = dx;
    s.eC[k] = dy * s.X[j] - dx * s.Y[j];
    s.bias[k] = (dy < 0 || (dy == 0 && dx < 0)) ? 0 : 1;
  }
  return true;
}

__device__ __forceinline__ uint32_t depth_at(const Setup& s, int px, int py) {
  float t = fadd((float)s.Z0, fmul(s.a, (float)(px - s.X[0])));
  t = fadd(t, fmul(s.b, (float)(py - s.Y[0])));
  float r = rintf(t);
  if (!(r > 0.0f)) return 0u;
  if (r >= (float)kZMax) return (uint32_t)kZMax;
  return (uint32_t)r;
}

__device__ __forceinline__ bool covers(const Setup& s, int64_t px, int64_t py) {
  bool in = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) in &= (s.eA[k] * px + s.eB[k] * py + s.eC[k]) >= s.bias[k];
  return in;
}

__device__ __forceinline__ int floor_div256(int a) { return a >= 0 ? a >> 8 : -((-a + 255) >> 8); }

struct BBox {
  int i0, i1, j0, j1;
};
__device__ __forceinline__ BBox pixel_bbox(const Setup& s, int W, int H) {
  int mnx = min(s.X[0], min(s.X[1], s.X[2])), mxx = max(s.X[0], max(s.X[1], s.X[2]));
  int mny = min(s.Y[0], min(s.Y[1], s.Y[2])), mxy = max(s.Y[0], max(s.Y[1], s.Y[2]));
  BBox b;
  b.i0 = max(floor_div256(mnx - 128 + 255), 0);
  b.i1 = min(floor_div256(mxx - 128), W - 1);
  b.j0 = max(floor_div256(mny - 128 + 255), 0);
  b.j1 = min(floor_div256(mxy - 128), H - 1);
  return b;
}

__device__ __forceinline__ void clear_body(const ClearArgs& a, int bid, int nb) {
  int64_t gid = (int64_t)bid * 256 + threadIdx.x;
  int64_t stride = (int64_t)nb * 256;
  for (int64_t i = gid; i < a.n; i += stride) {
    a.vis[i] = kKeyEmpty;
    if (a.cov) a.cov[i] = 0u;
  }
  if (gid <= a.B) a.big_cnt[gid] = 0u;   // B per-view big counts and the medium-queue count
}
ADR_KERNEL(__launch_bounds__(256), k_clear, ClearArgs, clear_body)

__device__ __forceinline__ void raster_pixel(const Setup& s, int t, int i, int j, int W,
                                             unsigned long long* __restrict__ vv, uint32_t* __restrict__ cv,
                                             const unsigned long long* __restrict__ fl) {
  const int px = 256 * i + 128, py = 256 * j + 128;
  if (!covers(s, px, py)) return;
  unsigned long long key = ((unsigned long long)depth_at(s, px, py) << 32) | (uint32_t)(t + 1);
  int64_t o = (int64_t)j * W + i;
  if (fl && key <= fl[o]) return;
  if (cv) atomicAdd(cv + o, 1u);
  atomicMin(vv + o, key);
}

// One thread per triangle and view.  A triangle whose pixel bounding box
// holds at most `tiny` pixel centres is walked by its thread; up to `med`
// it is queued for k_raster_med (big_cnt[B] counts the queue);
// larger ones go to the view's list for the tile kernel.
__device__ __forceinline__ void raster_small_body(const RasterArgs& a, int bid, int) {
  const MeshD& m = a.m;
  const ViewsD& v = a.v;
  const int4* __restrict__ snap = a.snap;
  uint32_t* __restrict__ big_cnt = a.big_cnt;
  unsigned long long* __restrict__ vis = a.vis;
  uint32_t* __restrict__ cov = a.cov;
  const unsigned long long* __restrict__ floor = a.floor;
  const int tiny = a.tiny, med_max = a.med_max;
  const int gid = bid * 256 + threadIdx.x;
  int area = 0, b = 0, t = 0;
  Setup s;
  BBox bb{0, -1, 0, -1};
  if (gid < v.B * m.n_tri) {
    b = gid / m.n_tri;
    t = gid - b * m.n_tri;
    int3 c = make_int3(m.tri[3 * t], m.tri[3 * t + 1], m.tri[3 * t + 2]);
    if (setup_tri(snap + (int64_t)b * m.n_pos, c, s)) {
      a.orient[gid] = s.flip ? -1 : 1;
      bb = pixel_bbox(s, v.W, v.H);
      if (bb.i1 >= bb.i0 && bb.j1 >= bb.j0) area = (bb.i1 - bb.i0 + 1) * (bb.j1 - bb.j0 + 1);
    } else {
      a.orient[gid] = 0;
    }
  }
  const int64_t HW = (int64_t)v.W * v.H;
  if (area > med_max) {
    uint32_t slot = atomicAdd(big_cnt + b, 1u);
    a.big[(int64_t)b * m.n_tri + slot] = (uint32_t)t;
  } else if (area > 0 && area <= tiny) {
    unsigned long long* vv = vis + b * HW;
    uint32_t* cv = cov ? cov + b * HW : nullptr;
    const unsigned long long* fl = floor ? floor + b * HW : nullptr;
    for (int j = bb.j0; j <= bb.j1; ++j)
      for (int i = bb.i0; i <= bb.i1; ++i) raster_pixel(s, t, i, j, v.W, vv, cv, fl);
  }
  // medium triangles of this wave: one queue reservation per wave
  const int lane = threadIdx.x & 63;
  const bool is_med = area > tiny && area <= med_max;
  const unsigned long long mm = __ballot(is_med);
  if (mm) {
    const int leader = __ffsll((long long)mm) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(big_cnt + v.B, (uint32_t)__popcll(mm));
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
    if (is_med) a.med[base + (uint32_t)__popcll(mm & ((1ull << lane) - 1ull))] = (uint32_t)gid;
  }
}
ADR_KERNEL(__launch_bounds__(256), k_raster_small, RasterArgs, raster_small_body)

// Queued medium triangles, one per wave at a time (a grid-stride loop over
// the queue).  The wave walks the triangle's bounding box in blocks of
// bw x (64 / bw) pixels, bw in 8..64 chosen per triangle to waste the fewest
// lanes.
__device__ __forceinline__ void raster_med_body(const RasterArgs& a, int bid, int nb) {
  const MeshD& m = a.m;
  const ViewsD& v = a.v;
  const int4* __restrict__ snap = a.snap;
  unsigned long long* __restrict__ vis = a.vis;
  uint32_t* __restrict__ cov = a.cov;
  const unsigned long long* __restrict__ floor = a.floor;
  const int lane = threadIdx.x & 63;
  const uint32_t n_waves = (uint32_t)nb * 4u;
  const uint32_t cnt = a.big_cnt[v.B];
  const int64_t HW = (int64_t)v.W * v.H;
  for (uint32_t q = (uint32_t)bid * 4u + (threadIdx.x >> 6); q < cnt; q += n_waves) {
    const int g = (int)a.med[q];
    const int b = g / m.n_tri, t = g - b * m.n_tri;
    const int3 c = make_int3(m.tri[3 * t], m.tri[3 * t + 1], m.tri[3 * t + 2]);
    Setup s;
    if (!setup_tri(snap + (int64_t)b * m.n_pos, c, s)) continue;  // queued triangles always set up
    const BBox bb = pixel_bbox(s, v.W, v.H);
    const int nx = bb.i1 - bb.i0 + 1, ny = bb.j1 - bb.j0 + 1;
    int lb = 3, fewest = 0x7fffffff;
#pragma unroll
    for (int l = 3; l <= 6; ++l) {
      const int bh = 64 >> l;
      const int blocks = ((nx + (1 << l) - 1) >> l) * ((ny + bh - 1) / bh);
      if (blocks < fewest) {
        fewest = blocks;
        lb = l;
      }
    }
    const int bw = 1 << lb, bh = 64 >> lb;
    const int lx = lane & (bw - 1), ly = lane >> lb;
    unsigned long long* vv = vis + b * HW;
    uint32_t* cv = cov ? cov + b * HW : nullptr;
    const unsigned long long* fl = floor ? floor + b * HW : nullptr;
    for (int y0 = bb.j0; y0 <= bb.j1; y0 += bh) {
      const int y = y0 + ly;
      for (int x0 = bb.i0; x0 <= bb.i1; x0 += bw) {
        const int x = x0 + lx;
        if (x <= bb.i1 && y <= bb.j1) raster_pixel(s, t, x, y, v.W, vv, cv, fl);
      }
    }
  }
}
ADR_KERNEL(__launch_bounds__(256), k_raster_med, RasterArgs, raster_med_body)

// One 16x16 tile of one view per block: stage the view's big triangles that
// overlap the tile into LDS, then resolve one pixel per thread.
__device__ __forceinline__ void raster_big_body(const RasterArgs& a, int bid, int nb) {
  __shared__ Setup lds[256];
  __shared__ int lds_t[256];
  __shared__ int lds_n;
  const MeshD& m = a.m;
  const ViewsD& v = a.v;
  const uint32_t* __restrict__ big = a.big;
  unsigned long long* __restrict__ vis = a.vis;
  uint32_t* __restrict__ cov = a.cov;
  const unsigned long long* __restrict__ floor = a.floor;
  const int tiles_x = a.tiles_x, tiles_y = a.tiles_y;
  const int per_view = tiles_x * tiles_y, n_tiles = per_view * v.B;
  // a grid-stride loop over the tiles of all views: a view without big
  // triangles is stepped over at once instead of costing a block per tile
  for (int tile = bid; tile < n_tiles; tile += nb) {
    const int b = tile / per_view;
    const uint32_t n_big = a.big_cnt[b];
    if (n_big == 0) {
      // on to this block's first tile in a later view
      tile += ((b + 1) * per_view - tile + nb - 1) / nb * nb - nb;
      continue;
    }
    int r = tile - b * per_view;
    int ty = r / tiles_x, tx = r - ty * tiles_x;
    int i = tx * kBigTile + (threadIdx.x & 15), j = ty * kBigTile + (threadIdx.x >> 4);
    int ti0 = tx * kBigTile, ti1 = min(ti0 + kBigTile, v.W) - 1;
    int tj0 = ty * kBigTile, tj1 = min(tj0 + kBigTile, v.H) - 1;
    const int4* sv = a.snap + (int64_t)b * m.n_pos;
    unsigned long long best = kKeyEmpty;
    uint32_t hits = 0;
    int64_t px = 256 * (int64_t)i + 128, py = 256 * (int64_t)j + 128;
    const unsigned long long fk =
        (floor && i < v.W && j < v.H) ? floor[(int64_t)b * v.W * v.H + (int64_t)j * v.W + i] : 0ull;
    for (uint32_t base = 0; base < n_big; base += 256) {
      if (threadIdx.x == 0) lds_n = 0;
      __syncthreads();
      uint32_t q = base + threadIdx.x;
      if (q < n_big) {
        int t = (int)big[(int64_t)b * m.n_tri + q];
        int3 c = make_int3(m.tri[3 * t], m.tri[3 * t + 1], m.tri[3 * t + 2]);
        Setup s;
        if (setup_tri(sv, c, s)) {
          BBox bb = pixel_bbox(s, v.W, v.H);
          if (bb.i0 <= ti1 && bb.i1 >= ti0 && bb.j0 <= tj1 && bb.j1 >= tj0) {
            int slot = atomicAdd(&lds_n, 1);
            lds[slot] = s;
            lds_t[slot] = t;
          }
        }
      }
      __syncthreads();
      int n = lds_n;
      if (i < v.W && j < v.H) {
        for (int k = 0; k < n; ++k) {
          if (!covers(lds[k], px, py)) continue;
          unsigned long long key =
              ((unsigned long long)depth_at(lds[k], (int)px, (int)py) << 32) | (uint32_t)(lds_t[k] + 1);
          if (floor && key <= fk) continue;
          ++hits;
          best = key < best ? key : best;
        }
      }
      __syncthreads();
    }
    if (i < v.W && j < v.H) {
      int64_t o = (int64_t)b * v.W * v.H + (int64_t)j * v.W + i;
      if (best != kKeyEmpty) atomicMin(vis + o, best);
      if (cov && hits) atomicAdd(cov + o, hits);
    }
  }
}
ADR_KERNEL(__launch_bounds__(256), k_raster_big, RasterArgs, raster_big_body)

Plan<XformArgs> plan_xform(const MeshD& m, const ViewsD& v, const Scratch& s) {
  // one thread per (view, vertex), at least 16 per view for the matrices
  const int n = m.n_pos > 0 ? (m.n_pos < 16 ? 16 : m.n_pos) * v.B : 0;
  return {XformArgs{m, v, reinterpret_cast<int4*>(s.snap), s.mvpd}, (unsigned)((n + 255) / 256)};
}

hipError_t launch_xform(const MeshD& m, const ViewsD& v, const Scratch& s, hipStream_t st) {
  ADR_LAUNCH_1(k_xform, plan_xform(m, v, s), st);
  return hipGetLastError();
}

Plan<ClearArgs> plan_clear_vis(uint64_t* vis, uint32_t* cov, int64_t n, uint32_t* big_cnt, int B) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < (B + 256) / 256) blocks = (B + 256) / 256;   // threads for the B + 1 counters
  return {ClearArgs{vis, cov, n, big_cnt, B}, (unsigned)blocks};
}

hipError_t launch_clear_vis(uint64_t* vis, uint32_t* cov, int64_t n, uint32_t* big_cnt, int B,
                            hipStream_t st) {
  ADR_LAUNCH_1(k_clear, plan_clear_vis(vis, cov, n, big_cnt, B), st);
  return hipGetLastError();
}

RasterPlans plan_raster(const MeshD& m, const ViewsD& v, const Scratch& s, uint64_t* vis, uint32_t* cov,
                        const uint64_t* floor) {
  RasterArgs a{};
  a.m = m;
  a.v = v;
  a.snap = reinterpret_cast<const int4*>(s.snap);
  a.orient = s.orient;
  a.big = s.big;
  a.big_cnt = s.big_cnt;
  a.med = s.med;
  a.vis = reinterpret_cast<unsigned long long*>(vis);
  a.cov = cov;
  a.floor = reinterpret_cast<const unsigned long long*>(floor);
  a.tiny = s.tiny_bbox;
  a.med_max = s.med_bbox;
  a.tiles_x = (v.W + kBigTile - 1) / kBigTile;
  a.tiles_y = (v.H + kBigTile - 1) / kBigTile;
  const int n = v.B * m.n_tri;
  RasterPlans p;
  p.a = a;
  p.small = n > 0 ? (unsigned)((n + 255) / 256) : 0u;
  // enough waves to fill the chip; each loops over the queue
  p.med = n > 0 ? (unsigned)std::min((n + 3) / 4, 4096) : 0u;
  // the big-triangle tiles: at most kBigBlocks blocks, each looping over tiles
  p.big = n > 0 ? (unsigned)std::min(a.tiles_x * a.tiles_y * v.B, kBigBlocks) : 0u;
  return p;
}

hipError_t launch_raster(const MeshD& m, const ViewsD& v, const Scratch& s, uint64_t* vis,
                         uint32_t* cov, hipStream_t st, const uint64_t* floor) {
  const RasterPlans p = plan_raster(m, v, s, vis, cov, floor);
  ADR_LAUNCH_1(k_raster_small, (Plan<RasterArgs>{p.a, p.small}), st);
  ADR_LAUNCH_1(k_raster_med, (Plan<RasterArgs>{p.a, p.med}), st);
  ADR_LAUNCH_1(k_raster_big, (Plan<RasterArgs>{p.a, p.big}), st);
  return hipGetLastError();
}

// ---- batched launches ----
hipError_t launch_xform_n(const Stage<XformArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_xform, s, st);
  return hipGetLastError();
}
hipError_t launch_clear_vis_n(const Stage<ClearArgs>& s, hipStream_t st) {
  ADR_LAUNCH_N(k_clear, s, st);
  return hipGetLastError();
}
hipError_t launch_raster_n(const Stage<RasterArgs>& small, const Stage<RasterArgs>& med,
                           const Stage<RasterArgs>& big, hipStream_t st) {
  ADR_LAUNCH_N(k_raster_small, small, st);
  ADR_LAUNCH_N(k_raster_med, med, st);
  ADR_LAUNCH_N(k_raster_big, big, st);
  return hipGetLastError();
}

}  // namespace adr

namespace adr {

// Screen orientation of every triangle in every view (+1, -1, 0 dropped);
// the backward pass needs it for the silhouette test without re-rasterizing.
__global__ void k_orient(MeshD m, ViewsD v, const int4* __restrict__ snap, int8_t* __restrict__ orient) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= v.B * m.n_tri) return;
  int b = gid / m.n_tri, t = gid - b * m.n_tri;
  const int4* sv = snap + (int64_t)b * m.n_pos;
  int4 v0 = sv[m.tri[3 * t]], v1 = sv[m.tri[3 * t + 1]], v2 = sv[m.tri[3 * t + 2]];
  int8_t o = 0;
  if (v0.w && v1.w && v2.w) {
    int64_t A = (int64_t)(v1.x - v0.x) * (v2.y - v0.y) - (int64_t)(v1.y - v0.y) * (v2.x - v0.x);
    o = A > 0 ? 1 : (A < 0 ? -1 : 0);
  }
  orient[gid] = o;
}

hipError_t launch_orient(const MeshD& m, const ViewsD& v, const Scratch& s, hipStream_t st) {
  int n = v.B * m.n_tri;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_orient, dim3((n + 255) / 256), dim3(256), 0, st, m, v,
                     reinterpret_cast<const int4*>(s.snap), s.orient);
  return hipGetLastError();
}

}  // namespace adr
