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

__global__ __launch_bounds__(256) void k_mip_build_tiles(MipSet ms) {
  const Tex& t = ms.t[blockIdx.y];
  const int S = t.size, T = S < kMipTile ? S : kMipTile, nt = S / T;
  const int L = min(t.levels - 1, ilog2i(T));
  if ((int)blockIdx.x >= nt * nt || L <= 0) return;
  const int C = t.channels, tid = threadIdx.x;
  const int by = blockIdx.x / nt, bx = blockIdx.x - by * nt;
  __shared__ float lds[2][256 * 4];
  float* d = (float*)t.data;
  int s = T >> 1;
  if (tid < s * s) {
    int r = tid / s, c = tid - r * s;
    int64_t t00 = (int64_t)(by * T + 2 * r) * S + bx * T + 2 * c;
    int64_t o = (int64_t)t.off[1] + (int64_t)(by * s + r) * (S >> 1) + bx * s + c;
    for (int ch = 0; ch < C; ++ch) {
      float a = d[t00 * C + ch], b = d[(t00 + 1) * C + ch];
      float e = d[(t00 + S) * C + ch], f = d[(t00 + S + 1) * C + ch];
      float v = ((a + b) + (e + f)) * 0.25f;
      lds[0][tid * C + ch] = v;
      d[o * C + ch] = v;
    }
  }
  for (int l = 2; l <= L; ++l) {
    const int sp = s;
    s >>= 1;
    __syncthreads();
    const float* src = lds[l & 1];
    float* dst = lds[(l + 1) & 1];
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

// Levels above the tile range, one block per map, level by level.
__global__ __launch_bounds__(256) void k_mip_build_top(MipSet ms) {
  const Tex& t = ms.t[blockIdx.x];
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

// Adjoint of the coarse levels above the tile range: level l pushes a
// quarter of each texel's gradient to its four children and is cleared.
__global__ __launch_bounds__(256) void k_mip_adjoint_top(MipSet ms) {
  const Tex& t = ms.t[blockIdx.x];
  const int S = t.size, C = t.channels;
  float* g = ms.g[blockIdx.x];
  for (int l = t.levels - 1; l > kMipTileLevels; --l) {
    const int s = S >> l, sc = 2 * s;
    for (int idx = threadIdx.x; idx < s * s; idx += blockDim.x) {
      int r = idx / s, c = idx - r * s;
      int64_t k00 = (int64_t)t.off[l - 1] + (int64_t)(2 * r) * sc + 2 * c;
      int64_t kids[4] = {k00, k00 + 1, k00 + sc, k00 + sc + 1};
      int64_t o = (int64_t)t.off[l] + idx;
      for (int ch = 0; ch < C; ++ch) {
        float w = 0.25f * g[o * C + ch];
        for (int k = 0; k < 4; ++k) g[kids[k] * C + ch] += w;
        g[o * C + ch] = 0.f;
      }
    }
    __syncthreads();
  }
}

// Adjoint within a level-0 tile: the tile's levels L..1 (L <= 5) folded
// down through LDS (each level adds a quarter of its parent's folded value)
// and added to level 0; the tile's coarse texels are cleared.
__global__ __launch_bounds__(256) void k_mip_adjoint_tiles(MipSet ms) {
  const Tex& t = ms.t[blockIdx.y];
  const int S = t.size, T = S < kMipTile ? S : kMipTile, nt = S / T;
  const int L = min(t.levels - 1, ilog2i(T));
  if ((int)blockIdx.x >= nt * nt || L <= 0) return;
  const int C = t.channels, tid = threadIdx.x;
  const int by = blockIdx.x / nt, bx = blockIdx.x - by * nt;
  float* g = ms.g[blockIdx.y];
  __shared__ float lds[2][256 * 4];
  // level L of the tile has no parent inside it
  int s = T >> L;
  float* cur = lds[L & 1];
  if (tid < s * s) {
    int r = tid / s, c = tid - r * s;
    int64_t o = (int64_t)t.off[L] + (int64_t)(by * s + r) * (S >> L) + bx * s + c;
    for (int ch = 0; ch < C; ++ch) {
      cur[tid * C + ch] = g[o * C + ch];
      g[o * C + ch] = 0.f;
    }
  }
  for (int l = L - 1; l >= 1; --l) {
    const int sp = s;
    s <<= 1;
    __syncthreads();
    const float* par = lds[(l + 1) & 1];
    float* dst = lds[l & 1];
    if (tid < s * s) {
      int r = tid / s, c = tid - r * s;
      int kp = (r >> 1) * sp + (c >> 1);
      int64_t o = (int64_t)t.off[l] + (int64_t)(by * s + r) * (S >> l) + bx * s + c;
      for (int ch = 0; ch < C; ++ch) {
        float v = g[o * C + ch] + 0.25f * par[kp * C + ch];
        dst[tid * C + ch] = v;
        g[o * C + ch] = 0.f;
      }
    }
  }
  __syncthreads();
  const float* par = lds[1];
  const int sp = T >> 1;
  for (int k = tid; k < T * T; k += blockDim.x) {
    int r = k / T, c = k - r * T;
    int kp = (r >> 1) * sp + (c >> 1);
    int64_t o = (int64_t)(by * T + r) * S + bx * T + c;
    for (int ch = 0; ch < C; ++ch) g[o * C + ch] += 0.25f * par[kp * C + ch];
  }
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
  if (has_top(ms)) {
    hipLaunchKernelGGL(k_mip_adjoint_top, dim3(ms.n), dim3(256), 0, st, ms);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_mip_adjoint_tiles, dim3(max_tiles(ms), ms.n), dim3(256), 0, st, ms);
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
