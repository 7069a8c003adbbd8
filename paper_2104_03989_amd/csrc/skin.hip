// Dense linear blend skinning (Sec. 5.1, "Animation & skinning", Eq. 2):
//   v_i^s = sum_b w_ib M_b (v_i, 1)     M_b: top three rows of an affine map
//
// Written as two small contractions on the matrix cores (float64 MFMA
// 16x16x4, one wave per 16 vertices):
//   forward   A[V,12]  = W[V,nb] x M[nb,12]      blended matrix of each vertex
//             v^s_i    = A_i (v_i, 1)            4-term dot per output row
//   adjoint   dW[V,nb] = U[V,12] x M[nb,12]^T    U_i = g_i (v_i, 1)^T
//             g_v_i    = A_i[:, :3]^T g_i
// Every product of float32 inputs is exact in float64, so the skinned
// positions are the float64 result rounded once to float32.  Each vertex row
// (of A, W, dW) belongs to one wave: the adjoint accumulates without atomics.
//
// MFMA f64 16x16x4 operand layout (lane l of a wave, i/j/k the row, column
// and reduction indices): A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// D[i][j] in element i / 4 of lane j + 16 (i % 4) (rows interleaved over the
// four lane groups, unlike the float32 16x16x4 form).
#include "dev.h"

namespace adr {

typedef double dx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dx4 mfma_f64(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Bone k of chunk q..q+15 seen by lane (row/col n, k-slot kk) at sub-step e.
// Forward: A lane (i, kk) holds the weights of bones q + 4 kk + e, e = 0..3,
// loaded as one float4 when the row is 16-byte aligned.
template <bool VEC>
__global__ __launch_bounds__(64) void k_skin_fwd(int n, int nb, const float* __restrict__ pos,
                                                 const float* __restrict__ w, const float* __restrict__ bones,
                                                 float* __restrict__ out, float* __restrict__ blend) {
  const int lane = threadIdx.x;
  const int64_t v0 = (int64_t)blockIdx.x * 16;
  const int i = lane & 15, kk = lane >> 4;
  const int64_t va = v0 + i;
  const bool rin = va < n;
  const float* wrow = w + va * nb;
  dx4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int q = 0; q < nb; q += 16) {
    const int b0 = q + 4 * kk;
    float a[4];
    if (VEC && rin && b0 + 3 < nb) {
      const float4 t = *reinterpret_cast<const float4*>(wrow + b0);
      a[0] = t.x;
      a[1] = t.y;
      a[2] = t.z;
      a[3] = t.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = (rin && b0 + e < nb) ? wrow[b0 + e] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int b = b0 + e;
      const double m = (b < nb && i < 12) ? (double)bones[(int64_t)b * 12 + i] : 0.0;
      acc = mfma_f64((double)a[e], m, acc);
    }
  }
  // lane (j = lane & 15, g = lane >> 4) holds A[v0 + g + 4 r][j]
  const int j = lane & 15, c = j >> 2, m = j & 3;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t v = v0 + kk + 4 * r;
    const bool in = v < n;
    double x = 1.0;
    if (m < 3) x = in ? (double)pos[v * 3 + m] : 0.0;
    if (blend && in && j < 12) blend[v * 12 + j] = (float)acc[r];
    double p = acc[r] * x;
    p += __shfl_xor(p, 1);
    p += __shfl_xor(p, 2);
    if (in && m == 0 && c < 3) out[v * 3 + c] = (float)p;
  }
}

// Adjoint.  A operand: U[v0 + i][4 s + kk] = g[c = s] x[m = kk]; B operand:
// M[bone 16 t + n][4 s + kk]; D: dW[v0 + g + 4 r][16 t + j].
__global__ __launch_bounds__(64) void k_skin_bwd(int n, int nb, const float* __restrict__ pos,
                                                 const float* __restrict__ bones, const float* __restrict__ blend,
                                                 float* __restrict__ gout, float* __restrict__ gpos,
                                                 float* __restrict__ gw) {
  const int lane = threadIdx.x;
  const int64_t v0 = (int64_t)blockIdx.x * 16;
  const int i = lane & 15, kk = lane >> 4;
  const int64_t va = v0 + i;
  const bool rin = va < n;
  double g[3] = {0.0, 0.0, 0.0};
  double x = 0.0;
  if (rin) {
#pragma unroll
    for (int s = 0; s < 3; ++s) g[s] = (double)gout[va * 3 + s];
    x = kk < 3 ? (double)pos[va * 3 + kk] : 1.0;
  }
  if (gw) {
    for (int t = 0; t < nb; t += 16) {
      const int b = t + i;
      dx4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const double m = b < nb ? (double)bones[(int64_t)b * 12 + 4 * s + kk] : 0.0;
        acc = mfma_f64(g[s] * x, m, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t v = v0 + kk + 4 * r;
        if (v < n && b < nb) gw[v * nb + b] += (float)acc[r];
      }
    }
  }
  // lanes with kk < 3: g_v[va][kk] = sum_c A[va][c][kk] g[c]
  if (rin && kk < 3) {
    if (gpos) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) s += (double)blend[va * 12 + 4 * c + kk] * g[c];
      gpos[va * 3 + kk] += (float)s;
    }
    gout[va * 3 + kk] = 0.f;   // consumed: every read of this row is above, in this wave
  }
}

hipError_t launch_skin_fwd(int n, int nb, const float* pos, const float* w, const float* bones, float* out,
                           float* blend, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 15) / 16));
  const bool vec = (nb % 4 == 0) && ((uintptr_t)w % 16 == 0);
  if (vec)
    hipLaunchKernelGGL(k_skin_fwd<true>, grid, dim3(64), 0, st, n, nb, pos, w, bones, out, blend);
  else
    hipLaunchKernelGGL(k_skin_fwd<false>, grid, dim3(64), 0, st, n, nb, pos, w, bones, out, blend);
  return hipGetLastError();
}

hipError_t launch_skin_bwd(int n, int nb, const float* pos, const float* bones, const float* blend, float* gout,
                           float* gpos, float* gw, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_skin_bwd, dim3((unsigned)((n + 15) / 16)), dim3(64), 0, st, n, nb, pos, bones, blend, gout,
                     gpos, gw);
  return hipGetLastError();
}

}  // namespace adr
