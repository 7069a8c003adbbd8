// Mip chains of the optimised maps (each level a 2x2 box average of the one
// below; Sec. 4.2 treats the mip chain as the texture representation) and
// the adjoint that pushes coarse-level texel gradients down to level 0.
// RGBA8: (a + b + c + d + 2) >> 2 per channel; F32: ((a + b) + (c + d)) / 4.
#include "dev.h"

namespace adr {

__global__ void k_mip_down_rgba8(uchar4* __restrict__ d, int src_off, int dst_off, int s_dst) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  int n = s_dst * s_dst;
  if (idx >= n) return;
  int r = idx / s_dst, c = idx - r * s_dst;
  int s_src = 2 * s_dst;
  const uchar4* src = d + src_off;
  int64_t t00 = (int64_t)(2 * r) * s_src + 2 * c;
  uchar4 a = src[t00], b = src[t00 + 1], e = src[t00 + s_src], f = src[t00 + s_src + 1];
  uchar4 o;
  o.x = (unsigned char)(((int)a.x + b.x + e.x + f.x + 2) >> 2);
  o.y = (unsigned char)(((int)a.y + b.y + e.y + f.y + 2) >> 2);
  o.z = (unsigned char)(((int)a.z + b.z + e.z + f.z + 2) >> 2);
  o.w = (unsigned char)(((int)a.w + b.w + e.w + f.w + 2) >> 2);
  d[dst_off + idx] = o;
}

// ------------------------------------------------------------------ F32 chains
// Float chains are built and differentiated in two launches for all maps of
// a material: a tile kernel in which each block owns a kMipTile^2 tile of
// level 0 and the levels 1..log2(kMipTile) above it (kept in LDS between
// levels), and a one-block-per-map kernel for the few coarse levels above.
// Both produce exactly the per-level box filter and its adjoint.
constexpr int kMipTile = 32;
constexpr int kMipTileLevels = 5;  // log2(kMipTile)

__device__ __forceinline__ int ilog2i(int x) { return 31 - __clz(x); }

// Row-major copy of a tile region between global memory and LDS with
// consecutive threads on consecutive floats: rows of `w` floats, global row
// stride `gs`; float4 when both are multiples of 4 and the base is aligned.
template <bool LOAD>
__device__ __forceinline__ void tile_copy(float* g, int64_t gs, float* l, int rows, int w, bool vec) {
  const int tid = threadIdx.x;
  if (vec) {
    const int w4 = w >> 2, n = rows * w4;
    for (int e = tid; e < n; e += blockDim.x) {
      const int r = e / w4, x = e - r * w4;
      float4* gp = reinterpret_cast<float4*>(g + r * gs) + x;
      float4* lp = reinterpret_cast<float4*>(l + r * w) + x;
      if (LOAD) *lp = *gp;
      else *gp = *lp;
    }
  } else {
    const int n = rows * w;
    for (int e = tid; e < n; e += blockDim.x) {
      const int r = e / w, x = e - r * w;
      if (LOAD) l[e] = g[r * gs + x];
      else g[r * gs + x] = l[e];
    }
  }
}

__device__ __forceinline__ bool vec_ok(const float* p, int w, int64_t gs) {
  return (w & 3) == 0 && (gs & 3) == 0 && ((uintptr_t)p & 15) == 0;
}

// Levels 1..L of a tile from its level 0 held in LDS (`base`, T rows of
// T*C floats), each level kept in LDS for the next and written to the chain.
__device__ __forceinline__ void tile_build_levels(const Tex& t, float* d, int by, int bx, int T, int L,
                                                  const float* base, float* odd, float* even) {
  const int S = t.size, C = t.channels, tid = threadIdx.x;
  int s = T >> 1;
  if (tid < s * s) {
    int r = tid / s, c = tid - r * s;
    int k00 = 2 * r * T + 2 * c;
    for (int ch = 0; ch < C; ++ch) {
      float a = base[k00 * C + ch], b = base[(k00 + 1) * C + ch];
      float e = base[(k00 + T) * C + ch], f = base[(k00 + T + 1) * C + ch];
      odd[tid * C + ch] = ((a + b) + (e + f)) * 0.25f;
    }
  }
  __syncthreads();
  float* g1 = d + ((int64_t)t.off[1] + (int64_t)(by * s) * (S >> 1) + bx * s) * C;
  tile_copy<false>(g1, (int64_t)(S >> 1) * C, odd, s, s * C, vec_ok(g1, s * C, (int64_t)(S >> 1) * C));
  for (int l = 2; l <= L; ++l) {
    const int sp = s;
    s >>= 1;
    __syncthreads();
    const float* src = (l & 1) ? even : odd;
    float* dst = (l & 1) ? odd : even;
    if (tid < s * s) {
      int r = tid / s, c = tid - r * s;
      int k00 = 2 * r * sp + 2 * c;
      int64_t o = (int64_t)t.off[l] + (int64_t)(by * s + r) * (S >> l) + bx * s + c;
      for (int ch = 0; ch < C; ++ch) {
        float a = src[k00 * C + ch], b = src[(k00 + 1) * C + ch];
        float e = src[(k00 + sp) * C + ch], f = src[(k00 + sp + 1) * C + ch];
        float v = ((a + b) + (e + f)) * 0.25f;
        dst[tid * C + ch] = v;
        d[o * C + ch] = v;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_mip_build_tiles(MipSet ms) {
  const Tex& t = ms.t[blockIdx.y];
  const int S = t.size, T = S < kMipTile ? S : kMipTile, nt = S / T;
  const int L = min(t.levels - 1, ilog2i(T));
  if ((int)blockIdx.x >= nt * nt || L <= 0) return;
  const int C = t.channels;
  const int by = blockIdx.x / nt, bx = blockIdx.x - by * nt;
  __shared__ __align__(16) float base[kMipTile * kMipTile * 3];
  __shared__ __align__(16) float lds[2][256 * 4];
  float* d = (float*)t.data;
  // level 0 of the tile into LDS, coalesced
  float* g0 = d + ((int64_t)(by * T) * S + bx * T) * C;
  tile_copy<true>(g0, (int64_t)S * C, base, T, T * C, vec_ok(g0, T * C, (int64_t)S * C));
  __syncthreads();
  tile_build_levels(t, d, by, bx, T, L, base, lds[0], lds[1]);
}

// Levels above the tile range of map k, level by level (one block).
__device__ __forceinline__ void build_top(const Tex& t) {
  const int S = t.size, C = t.channels;
  float* d = (float*)t.data;
  for (int l = kMipTileLevels + 1; l < t.levels; ++l) {
    const int s = S >> l, sp = 2 * s;
    for (int idx = threadIdx.x; idx < s * s; idx += blockDim.x) {
      int r = idx / s, c = idx - r * s;
      int64_t t00 = (int64_t)t.off[l - 1] + (int64_t)(2 * r) * sp + 2 * c;
      int64_t o = (int64_t)t.off[l] + idx;
      for (int ch = 0; ch < C; ++ch) {
        float a = d[t00 * C + ch], b = d[(t00 + 1) * C + ch];
        float e = d[(t00 + sp) * C + ch], f = d[(t00 + sp + 1) * C + ch];
        d[o * C + ch] = ((a + b) + (e + f)) * 0.25f;
      }
    }
    __syncthreads();
  }
}

// Clears the gradients of the levels above the tile range (one block).
__device__ __forceinline__ void clear_top(const Tex& t, float* g) {
  if (t.levels - 1 <= kMipTileLevels) return;
  const int64_t a = (int64_t)t.off[kMipTileLevels + 1] * t.channels, b = (int64_t)t.off[t.levels] * t.channels;
  for (int64_t k = a + threadIdx.x; k < b; k += blockDim.x) g[k] = 0.f;
}

__global__ __launch_bounds__(256) void k_mip_build_top(MipSet ms) { build_top(ms.t[blockIdx.x]); }

// Run once every tile has folded the levels above the tiles.
__global__ __launch_bounds__(256) void k_mip_clear_top(MipSet ms) { clear_top(ms.t[blockIdx.x], ms.g[blockIdx.x]); }

// Adjoint within a level-0 tile: the tile's levels 1..L (L <= 5) are read
// into LDS in one round (and cleared), folded down (each level adds a
// quarter of its parent's folded value), and a quarter of the folded level 1
// is added to level 0.
constexpr int kPyrFloats = (256 + 64 + 16 + 4 + 1) * 3;  // levels 1..5 of a 32^2 tile, 3 channels
constexpr int kAncFloats = (kMaxLevels - 1 - kMipTileLevels) * 3;  // one texel per level above a tile
constexpr int kPyrLds = kPyrFloats + kAncFloats;

// Reads the tile's gradient levels 1..L into `pyr` (kPyrLds floats) in one
// round (clearing them) together with the tile's ancestors above level L
// (one texel per level), adds the ancestors folded from the top and folds
// down, so that pyr holds the folded level 1 at offset 0 on return (after a
// barrier).  Level l of the tile (T >> l texels a side) sits at pyr + po[l].
__device__ __forceinline__ void tile_fold_grads(const Tex& t, float* g, int by, int bx, int T, int L, float* pyr) {
  const int S = t.size, C = t.channels, tid = threadIdx.x;
  int po[kMipTileLevels + 2];
  po[1] = 0;
  for (int l = 1; l <= L; ++l) po[l + 1] = po[l] + (T >> l) * (T >> l) * C;
  const int total = po[L + 1];
  constexpr int kPer = (kPyrFloats + 255) / 256;
  float v[kPer];
  int64_t addr[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = tid + 256 * u;
    addr[u] = -1;
    if (e < total) {
      int l = 1;
      while (e >= po[l + 1]) ++l;
      const int sl = T >> l, w = sl * C, k = e - po[l], r = k / w, x = k - r * w;
      addr[u] = ((int64_t)t.off[l] + (int64_t)(by * sl + r) * (S >> l) + bx * sl) * C + x;
      v[u] = g[addr[u]];
    }
  }
  // ancestors (levels L+1.. of a full 32^2 tile), one per thread, cleared
  // only once every tile has read them (a separate launch)
  const int na = (T == kMipTile && L == kMipTileLevels) ? (t.levels - 1 - L) * C : 0;
  float anc = 0.f;
  if (tid < na) {
    const int l = L + 1 + tid / C, ch = tid - (tid / C) * C, sl = S >> l, sh = l - L;
    anc = g[((int64_t)t.off[l] + (int64_t)(by >> sh) * sl + (bx >> sh)) * C + ch];
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    if (addr[u] >= 0) {
      pyr[tid + 256 * u] = v[u];
      g[addr[u]] = 0.f;
    }
  }
  if (tid < na) pyr[kPyrFloats + tid] = anc;
  // levels above the tile (a 32^2 tile's level 5 is one texel): its
  // ancestors' gradients folded from the top, f = g_l + f / 4, added to it
  // as a quarter of the folded parent (the same arithmetic as level by level)
  __syncthreads();
  if (tid < C && na > 0) {
    float f = 0.f;
    for (int l = t.levels - 1; l > L; --l) f = pyr[kPyrFloats + (l - L - 1) * C + tid] + 0.25f * f;
    pyr[po[L] + tid] += 0.25f * f;
  }
  // fold down: level l += a quarter of level l + 1
  for (int l = L - 1; l >= 1; --l) {
    __syncthreads();
    const int sl = T >> l, sp = sl >> 1;
    for (int k = tid; k < sl * sl * C; k += blockDim.x) {
      const int texel = k / C, ch = k - texel * C, r = texel / sl, c = texel - r * sl;
      pyr[po[l] + k] += 0.25f * pyr[po[l + 1] + ((r >> 1) * sp + (c >> 1)) * C + ch];
    }
  }
  __syncthreads();
}

// Adjoint within a level-0 tile: the folded level 1 (tile_fold_grads), a
// quarter of which is added to level 0.
__global__ __launch_bounds__(256) void k_mip_adjoint_tiles(MipSet ms) {
  const Tex& t = ms.t[blockIdx.y];
  const int S = t.size, T = S < kMipTile ? S : kMipTile, nt = S / T;
  const int L = min(t.levels - 1, ilog2i(T));
  if ((int)blockIdx.x >= nt * nt || L <= 0) return;
  const int C = t.channels, tid = threadIdx.x;
  const int by = blockIdx.x / nt, bx = blockIdx.x - by * nt;
  float* g = ms.g[blockIdx.y];
  __shared__ float pyr[kPyrLds];
  tile_fold_grads(t, g, by, bx, T, L, pyr);
  // level 0 += a quarter of the folded level 1, row by row with consecutive
  // threads on consecutive floats (float4 where aligned)
  const float* par = pyr;
  const int sp = T >> 1, w = T * C;
  float* g0 = g + ((int64_t)(by * T) * S + bx * T) * C;
  const int64_t gs = (int64_t)S * C;
  if (vec_ok(g0, w, gs)) {
    const int w4 = w >> 2;
    for (int e = tid; e < T * w4; e += blockDim.x) {
      const int r = e / w4, x4 = e - r * w4;
      float4* gp = reinterpret_cast<float4*>(g0 + r * gs) + x4;
      float4 q4 = *gp;
      float q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int x = 4 * x4 + u, c = x / C, ch = x - c * C;
        q[u] = 0.25f * par[((r >> 1) * sp + (c >> 1)) * C + ch];
      }
      q4.x += q[0];
      q4.y += q[1];
      q4.z += q[2];
      q4.w += q[3];
      *gp = q4;
    }
  } else {
    for (int e = tid; e < T * w; e += blockDim.x) {
      const int r = e / w, x = e - r * w, c = x / C, ch = x - c * C;
      g0[r * gs + x] += 0.25f * par[((r >> 1) * sp + (c >> 1)) * C + ch];
    }
  }
}

// Adam on level 0 of optimised maps fused with the chain's adjoint before it
// and the chain's rebuild after it (one block per level-0 tile): the tile's
// level-0 gradient is completed by the folded coarser levels exactly as
// k_mip_adjoint_tiles does, Adam updates the tile's texels, the gradient
// chain of the tile is cleared, and levels 1..5 of the tile are rebuilt from
// the new level 0 exactly as k_mip_build_tiles does.  The levels above the
// tiles follow in k_adam_maps_top.  The same bits as the adjoint, Adam and
// build launched one after another.
constexpr int kTileF4 = kMipTile * kMipTile * 3 / 4 / 256;  // float4 per thread of a 32^2 x 3 tile

__global__ __launch_bounds__(256) void k_adam_maps_tiles(AdamMapSet a, float b1, float b2, float c1, float c2,
                                                         float lr, float eps) {
  const Tex& t = a.ms.t[blockIdx.y];
  const int S = t.size, T = S < kMipTile ? S : kMipTile, nt = S / T;
  if ((int)blockIdx.x >= nt * nt) return;
  const int L = min(t.levels - 1, ilog2i(T));
  const int C = t.channels, tid = threadIdx.x;
  const int by = blockIdx.x / nt, bx = blockIdx.x - by * nt;
  // LDS: the gradient pyramid, reused for the odd levels of the rebuild once
  // the level-0 update has read it; the new level 0, reused for the even
  // levels once level 1 is built from it
  __shared__ __align__(16) float pyr[kPyrLds];
  __shared__ __align__(16) float base[kMipTile * kMipTile * 3];
  const int64_t o0 = ((int64_t)(by * T) * S + bx * T) * C, gs = (int64_t)S * C;
  float* d = (float*)t.data;
  float* g = a.ms.g[blockIdx.y];
  float *P = d + o0, *G = g + o0, *M = a.m[blockIdx.y] + o0, *V = a.v[blockIdx.y] + o0;
  const int sp = T >> 1, w = T * C;
  const bool vec = vec_ok(P, w, gs) && vec_ok(G, w, gs) && vec_ok(M, w, gs) && vec_ok(V, w, gs);
  const int w4 = w >> 2, n4 = vec ? T * w4 : 0;
  // the tile's level-0 loads are issued before the fold
  float4 p4[kTileF4], g4[kTileF4], m4[kTileF4], v4[kTileF4];
#pragma unroll
  for (int u = 0; u < kTileF4; ++u) {
    const int e = tid + 256 * u;
    if (e < n4) {
      const int r = e / w4, x4 = e - r * w4;
      const int64_t q = r * gs + 4 * x4;
      p4[u] = ld_nt(reinterpret_cast<const float4*>(P + q));
      g4[u] = ld_nt(reinterpret_cast<const float4*>(G + q));
      m4[u] = ld_nt(reinterpret_cast<const float4*>(M + q));
      v4[u] = ld_nt(reinterpret_cast<const float4*>(V + q));
    }
  }
  if (L > 0) tile_fold_grads(t, g, by, bx, T, L, pyr);
  // level 0: g += a quarter of the folded level 1, then Adam; the new
  // texels also go to LDS for the rebuild
#pragma unroll
  for (int u = 0; u < kTileF4; ++u) {
    const int e = tid + 256 * u;
    if (e < n4) {
      const int r = e / w4, x4 = e - r * w4;
      const int64_t q = r * gs + 4 * x4;
      float gg[4] = {g4[u].x, g4[u].y, g4[u].z, g4[u].w};
      if (L > 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int x = 4 * x4 + j, c = x / C, ch = x - c * C;
          gg[j] += 0.25f * pyr[((r >> 1) * sp + (c >> 1)) * C + ch];
        }
      }
      adam1(p4[u].x, gg[0], m4[u].x, v4[u].x, b1, b2, c1, c2, lr, eps);
      adam1(p4[u].y, gg[1], m4[u].y, v4[u].y, b1, b2, c1, c2, lr, eps);
      adam1(p4[u].z, gg[2], m4[u].z, v4[u].z, b1, b2, c1, c2, lr, eps);
      adam1(p4[u].w, gg[3], m4[u].w, v4[u].w, b1, b2, c1, c2, lr, eps);
      st_nt(reinterpret_cast<float4*>(P + q), p4[u]);
      st_nt(reinterpret_cast<float4*>(M + q), m4[u]);
      st_nt(reinterpret_cast<float4*>(V + q), v4[u]);
      st_nt(reinterpret_cast<float4*>(G + q), make_float4(0.f, 0.f, 0.f, 0.f));
      *reinterpret_cast<float4*>(base + r * w + 4 * x4) = p4[u];
    }
  }
  if (!vec) {
    for (int e = tid; e < T * w; e += blockDim.x) {
      const int r = e / w, x = e - r * w, c = x / C, ch = x - c * C;
      const int64_t q = r * gs + x;
      float gg = G[q];
      if (L > 0) gg += 0.25f * pyr[((r >> 1) * sp + (c >> 1)) * C + ch];
      float p = P[q], m = M[q], v = V[q];
      adam1(p, gg, m, v, b1, b2, c1, c2, lr, eps);
      P[q] = p;
      M[q] = m;
      V[q] = v;
      G[q] = 0.f;
      base[e] = p;
    }
  }
  if (L <= 0) return;
  __syncthreads();
  tile_build_levels(t, d, by, bx, T, L, base, pyr, base);
}

// After k_adam_maps_tiles: clears the gradient levels above the tiles and
// rebuilds the data levels above the tiles (one block per map).
__global__ __launch_bounds__(256) void k_adam_maps_top(MipSet ms) {
  clear_top(ms.t[blockIdx.x], ms.g[blockIdx.x]);
  build_top(ms.t[blockIdx.x]);
}

static int max_tiles(const MipSet& ms) {
  int n = 0;
  for (int k = 0; k < ms.n; ++k) {
    int T = ms.t[k].size < kMipTile ? ms.t[k].size : kMipTile;
    int nt = ms.t[k].size / T;
    n = nt * nt > n ? nt * nt : n;
  }
  return n;
}

static bool has_top(const MipSet& ms) {
  for (int k = 0; k < ms.n; ++k)
    if (ms.t[k].levels > kMipTileLevels + 1) return true;
  return false;
}

hipError_t launch_mip_build_set(const MipSet& ms, hipStream_t st) {
  if (ms.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mip_build_tiles, dim3(max_tiles(ms), ms.n), dim3(256), 0, st, ms);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !has_top(ms)) return e;
  hipLaunchKernelGGL(k_mip_build_top, dim3(ms.n), dim3(256), 0, st, ms);
  return hipGetLastError();
}

hipError_t launch_mip_adjoint_set(const MipSet& ms, hipStream_t st) {
  if (ms.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mip_adjoint_tiles, dim3(max_tiles(ms), ms.n), dim3(256), 0, st, ms);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !has_top(ms)) return e;
  // the levels above the tiles, read by every tile, are cleared afterwards
  hipLaunchKernelGGL(k_mip_clear_top, dim3(ms.n), dim3(256), 0, st, ms);
  return hipGetLastError();
}

hipError_t launch_adam_maps_tiles(const AdamMapSet& a, int t, float lr, float b1, float b2, float eps,
                                  hipStream_t st) {
  if (a.ms.n == 0) return hipSuccess;
  const double c1 = 1.0 / (1.0 - pow((double)b1, t)), c2 = 1.0 / (1.0 - pow((double)b2, t));
  hipLaunchKernelGGL(k_adam_maps_tiles, dim3(max_tiles(a.ms), a.ms.n), dim3(256), 0, st, a, b1, b2, (float)c1,
                     (float)c2, lr, eps);
  return hipGetLastError();
}

hipError_t launch_adam_maps_top(const AdamMapSet& a, hipStream_t st) {
  if (a.ms.n == 0 || !has_top(a.ms)) return hipSuccess;
  hipLaunchKernelGGL(k_adam_maps_top, dim3(a.ms.n), dim3(256), 0, st, a.ms);
  return hipGetLastError();
}

// Box filter of a supersampled image: out[b, j, i] = mean of in[b, k j + y,
// k i + x] over x, y < k, summed row by row.  Renders the reference of the
// prefiltering application (Sec. 4.2) with k^2 samples per pixel.
__global__ __launch_bounds__(256) void k_downsample(const float* __restrict__ in, int B, int H, int W, int k,
                                                   float* __restrict__ out) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= (int64_t)B * H * W) return;
  const int64_t b = o / ((int64_t)H * W);
  const int64_t r = o - b * H * W;
  const int j = (int)(r / W), i = (int)(r - (int64_t)j * W);
  const int64_t Ws = (int64_t)W * k;
  float ax = 0.f, ay = 0.f, az = 0.f;
  for (int y = 0; y < k; ++y) {
    const float* row = in + 3 * ((b * H * k + (int64_t)j * k + y) * Ws + (int64_t)i * k);
    for (int x = 0; x < k; ++x) {
      ax += row[3 * x];
      ay += row[3 * x + 1];
      az += row[3 * x + 2];
    }
  }
  const float s = 1.0f / (float)(k * k);
  out[3 * o] = ax * s;
  out[3 * o + 1] = ay * s;
  out[3 * o + 2] = az * s;
}

hipError_t launch_downsample(const float* in, int B, int H, int W, int k, float* out, hipStream_t st) {
  const int64_t n = (int64_t)B * H * W;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_downsample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, B, H, W, k, out);
  return hipGetLastError();
}

// RGBA8 chains (read-only maps, built once): one launch per level.
hipError_t launch_mip_build(const Tex& t, hipStream_t st) {
  if (t.fmt != ADR_TEX_RGBA8) {
    MipSet ms{};
    ms.t[0] = t;
    ms.n = 1;
    return launch_mip_build_set(ms, st);
  }
  for (int l = 1; l < t.levels; ++l) {
    int s = t.size >> l;
    if (s < 1) break;
    int n = s * s;
    hipLaunchKernelGGL(k_mip_down_rgba8, dim3((n + 255) / 256), dim3(256), 0, st,
                       (uchar4*)t.data, t.off[l - 1], t.off[l], s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace adr
