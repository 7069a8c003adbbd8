// Back-to-front blending of depth-peeled layers (Sec. 5.2, "Order-independent
// transparency") and its adjoint, per pixel of the view batch:
//   B_k = a_k c_k + (1 - a_k) C_{k+1}   where layer k covers the pixel,
//   B_k = C_{k+1}                       elsewhere,
// with C_{k+1} the antialiased composite of the layers behind (black behind
// the last).  The antialiasing of each layer runs in between (aa.hip).
#include "dev.h"

namespace adr {

__device__ __forceinline__ f3 ld3l(const float* p, int64_t o) { return mk(p[3 * o], p[3 * o + 1], p[3 * o + 2]); }

__global__ __launch_bounds__(256) void k_oit_blend(int64_t n, const uint64_t* __restrict__ vis,
                                                   const float* __restrict__ color, const float* __restrict__ alpha,
                                                   const float* __restrict__ behind, float* __restrict__ blend) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const f3 cb = behind ? ld3l(behind, o) : mk(0.f, 0.f, 0.f);
  f3 out = cb;
  if ((uint32_t)vis[o] != 0u) {
    const float a = alpha[o];
    out = a * ld3l(color, o) + (1.f - a) * cb;
  }
  st3(blend, o, out);
}

// g (in: dL/dB_k, out: dL/dc_k), galpha (out: dL/da_k) and gbehind (out:
// dL/dC_{k+1}; NULL behind the last layer).  Each pixel reads and writes
// only its own entries.
__global__ __launch_bounds__(256) void k_oit_blend_bwd(int64_t n, const uint64_t* __restrict__ vis,
                                                       const float* __restrict__ color,
                                                       const float* __restrict__ alpha,
                                                       const float* __restrict__ behind, float* __restrict__ g,
                                                       float* __restrict__ galpha, float* __restrict__ gbehind) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const f3 gB = ld3l(g, o);
  if ((uint32_t)vis[o] != 0u) {
    const float a = alpha[o];
    const f3 cb = behind ? ld3l(behind, o) : mk(0.f, 0.f, 0.f);
    st3(g, o, a * gB);
    galpha[o] = dot(gB, ld3l(color, o) - cb);
    if (gbehind) st3(gbehind, o, (1.f - a) * gB);
  } else {
    st3(g, o, mk(0.f, 0.f, 0.f));
    galpha[o] = 0.f;
    if (gbehind) st3(gbehind, o, gB);
  }
}

hipError_t launch_oit_blend(int64_t n, const uint64_t* vis, const float* color, const float* alpha,
                            const float* behind, float* blend, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_oit_blend, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, vis, color, alpha, behind,
                     blend);
  return hipGetLastError();
}

hipError_t launch_oit_blend_bwd(int64_t n, const uint64_t* vis, const float* color, const float* alpha,
                                const float* behind, float* g, float* galpha, float* gbehind, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_oit_blend_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, vis, color, alpha,
                     behind, g, galpha, gbehind);
  return hipGetLastError();
}

}  // namespace adr
