// Adam with bias correction (Sec. 5.3: "Adam with default parameters"),
// several tensors per launch:
//   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
//   p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps);  g = 0.
// Pure streaming: 16 bytes read and 16 written per parameter.
#include "dev.h"

namespace adr {

constexpr int kAdamMax = 8;

struct AdamTable {
  float* p[kAdamMax];
  float* g[kAdamMax];
  float* m[kAdamMax];
  float* v[kAdamMax];
  int64_t n4[kAdamMax];    // float4 chunks
  int64_t start[kAdamMax + 1];  // prefix of n4 (in float4 chunks)
  int count;
};

__global__ __launch_bounds__(256) void k_adam(AdamTable T, float b1, float b2, float c1, float c2,
                                              float lr, float eps) {
  int64_t total = T.start[T.count];
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
    int k = 0;
    while (k + 1 < T.count && q >= T.start[k + 1]) ++k;
    int64_t i = q - T.start[k];
    float4* P = reinterpret_cast<float4*>(T.p[k]);
    float4* G = reinterpret_cast<float4*>(T.g[k]);
    float4* M = reinterpret_cast<float4*>(T.m[k]);
    float4* V = reinterpret_cast<float4*>(T.v[k]);
    float4 p = P[i], g = G[i], m = M[i], v = V[i];
    adam1(p.x, g.x, m.x, v.x, b1, b2, c1, c2, lr, eps);
    adam1(p.y, g.y, m.y, v.y, b1, b2, c1, c2, lr, eps);
    adam1(p.z, g.z, m.z, v.z, b1, b2, c1, c2, lr, eps);
    adam1(p.w, g.w, m.w, v.w, b1, b2, c1, c2, lr, eps);
    P[i] = p;
    M[i] = m;
    V[i] = v;
    G[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// Remainder elements (n not a multiple of 4, or unaligned tensors).
__global__ void k_adam_scalar(float* p, float* g, float* m, float* v, int64_t n, float b1, float b2,
                              float c1, float c2, float lr, float eps) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float pp = p[i], mm = m[i], vv = v[i];
    adam1(pp, g[i], mm, vv, b1, b2, c1, c2, lr, eps);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
    g[i] = 0.f;
  }
}

hipError_t launch_adam(const adr_param* params, int n, int t, float lr, float b1, float b2, float eps,
                       hipStream_t st) {
  double c1 = 1.0 / (1.0 - pow((double)b1, t));
  double c2 = 1.0 / (1.0 - pow((double)b2, t));
  AdamTable T;
  T.count = 0;
  T.start[0] = 0;
  auto flush = [&]() -> hipError_t {
    if (T.count == 0) return hipSuccess;
    int64_t total = T.start[T.count];
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks > 0)
      hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, st, T, b1, b2, (float)c1,
                         (float)c2, lr, eps);
    T.count = 0;
    T.start[0] = 0;
    return hipGetLastError();
  };
  for (int k = 0; k < n; ++k) {
    const adr_param& a = params[k];
    bool aligned = ((uintptr_t)a.param | (uintptr_t)a.grad | (uintptr_t)a.m | (uintptr_t)a.v) % 16 == 0;
    int64_t n4 = aligned ? a.n / 4 : 0;
    int64_t rem = a.n - 4 * n4;
    if (n4 > 0) {
      T.p[T.count] = a.param;
      T.g[T.count] = a.grad;
      T.m[T.count] = a.m;
      T.v[T.count] = a.v;
      T.n4[T.count] = n4;
      T.start[T.count + 1] = T.start[T.count] + n4;
      ++T.count;
      if (T.count == kAdamMax) {
        hipError_t e = flush();
        if (e != hipSuccess) return e;
      }
    }
    if (rem > 0) {
      int64_t o = 4 * n4;
      int64_t blocks = (rem + 255) / 256;
      if (blocks > 4096) blocks = 4096;
      hipLaunchKernelGGL(k_adam_scalar, dim3((unsigned)blocks), dim3(256), 0, st, a.param + o,
                         a.grad + o, a.m + o, a.v + o, rem, b1, b2, (float)c1, (float)c2, lr, eps);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return flush();
}

}  // namespace adr
