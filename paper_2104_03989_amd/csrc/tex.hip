// Mip chains of the optimised maps (each level a 2x2 box average of the one
// below; Sec. 4.2 treats the mip chain as the texture representation) and
// the adjoint that pushes coarse-level texel gradients down to level 0.
#include "dev.h"

namespace adr {

__global__ void k_mip_down_f32(float* __restrict__ d, int src_off, int dst_off, int s_dst, int C) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  int n = s_dst * s_dst;
  if (idx >= n) return;
  int r = idx / s_dst, c = idx - r * s_dst;
  int s_src = 2 * s_dst;
  const float* src = d + (int64_t)src_off * C;
  float* dst = d + (int64_t)dst_off * C;
  int64_t t00 = (int64_t)(2 * r) * s_src + 2 * c, t01 = t00 + 1, t10 = t00 + s_src, t11 = t10 + 1;
  for (int ch = 0; ch < C; ++ch) {
    float a = src[t00 * C + ch], b = src[t01 * C + ch], e = src[t10 * C + ch], f = src[t11 * C + ch];
    dst[(int64_t)idx * C + ch] = ((a + b) + (e + f)) * 0.25f;
  }
}

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

hipError_t launch_mip_build(const Tex& t, hipStream_t st) {
  for (int l = 1; l < t.levels; ++l) {
    int s = t.size >> l;
    if (s < 1) break;
    int n = s * s;
    if (t.fmt == ADR_TEX_RGBA8) {
      hipLaunchKernelGGL(k_mip_down_rgba8, dim3((n + 255) / 256), dim3(256), 0, st,
                         (uchar4*)t.data, t.off[l - 1], t.off[l], s);
    } else {
      hipLaunchKernelGGL(k_mip_down_f32, dim3((n + 255) / 256), dim3(256), 0, st, (float*)t.data,
                         t.off[l - 1], t.off[l], s, t.channels);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Level l -> l-1: every texel of level l adds a quarter of its gradient to
// its four children and is cleared.
__global__ void k_mip_adjoint(float* __restrict__ g, int par_off, int child_off, int s_par, int C) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= s_par * s_par) return;
  int r = idx / s_par, c = idx - r * s_par;
  int s_ch = 2 * s_par;
  float* par = g + (int64_t)par_off * C;
  float* ch = g + (int64_t)child_off * C;
  int64_t t00 = (int64_t)(2 * r) * s_ch + 2 * c;
  int64_t kids[4] = {t00, t00 + 1, t00 + s_ch, t00 + s_ch + 1};
  for (int q = 0; q < C; ++q) {
    float v = par[(int64_t)idx * C + q];
    if (v != 0.f) {
      float w = 0.25f * v;
      for (int k = 0; k < 4; ++k) ch[kids[k] * C + q] += w;
      par[(int64_t)idx * C + q] = 0.f;
    }
  }
}

hipError_t launch_mip_adjoint(const Tex& t, float* g, hipStream_t st) {
  for (int l = t.levels - 1; l >= 1; --l) {
    int s = t.size >> l;
    int n = s * s;
    hipLaunchKernelGGL(k_mip_adjoint, dim3((n + 255) / 256), dim3(256), 0, st, g, t.off[l],
                       t.off[l - 1], s, t.channels);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace adr
