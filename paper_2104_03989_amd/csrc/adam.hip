// Adam with bias correction (Sec. 5.3: "Adam with default parameters"),
// several tensors per launch:
//   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
//   p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps);  g = 0.
// Pure streaming: 16 bytes read and 16 written per parameter.
#include "dev.h"

namespace adr {

constexpr int kAdamMax = 16;

// Up to kAdamMax tensors per launch, each cut into chunks of four floats
// (the last chunk may be partial); a tensor whose four pointers are 16-byte
// aligned moves its whole chunks as float4, the rest element by element.
struct AdamTable {
  float* p[kAdamMax];
  float* g[kAdamMax];
  float* m[kAdamMax];
  float* v[kAdamMax];
  int64_t n[kAdamMax];           // floats
  int64_t start[kAdamMax + 1];   // prefix of the chunk counts
  int vec;                       // bit k: tensor k is 16-byte aligned
  int count;
};

__global__ __launch_bounds__(256) void k_adam(AdamTable T, float b1, float b2, float c1, float c2,
                                              float lr, float eps) {
  int64_t total = T.start[T.count];
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
    int k = 0;
    while (k + 1 < T.count && q >= T.start[k + 1]) ++k;
    const int64_t i = q - T.start[k];
    if (((T.vec >> k) & 1) && 4 * i + 4 <= T.n[k]) {
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
    } else {
      const int64_t e1 = min(4 * i + 4, T.n[k]);
      for (int64_t e = 4 * i; e < e1; ++e) {
        float pp = T.p[k][e], mm = T.m[k][e], vv = T.v[k][e];
        adam1(pp, T.g[k][e], mm, vv, b1, b2, c1, c2, lr, eps);
        T.p[k][e] = pp;
        T.m[k][e] = mm;
        T.v[k][e] = vv;
        T.g[k][e] = 0.f;
      }
    }
  }
}

hipError_t launch_adam(const adr_param* params, int n, int t, float lr, float b1, float b2, float eps,
                       hipStream_t st) {
  double c1 = 1.0 / (1.0 - pow((double)b1, t));
  double c2 = 1.0 / (1.0 - pow((double)b2, t));
  AdamTable T;
  T.count = 0;
  T.vec = 0;
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
    T.vec = 0;
    T.start[0] = 0;
    return hipGetLastError();
  };
  for (int k = 0; k < n; ++k) {
    const adr_param& a = params[k];
    if (a.n <= 0) continue;
    const bool aligned = ((uintptr_t)a.param | (uintptr_t)a.grad | (uintptr_t)a.m | (uintptr_t)a.v) % 16 == 0;
    T.p[T.count] = a.param;
    T.g[T.count] = a.grad;
    T.m[T.count] = a.m;
    T.v[T.count] = a.v;
    T.n[T.count] = a.n;
    if (aligned) T.vec |= 1 << T.count;
    T.start[T.count + 1] = T.start[T.count] + (a.n + 3) / 4;
    ++T.count;
    if (T.count == kAdamMax) {
      hipError_t e = flush();
      if (e != hipSuccess) return e;
    }
  }
  return flush();
}

}  // namespace adr
