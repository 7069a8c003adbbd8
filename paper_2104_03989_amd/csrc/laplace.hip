// Uniform Laplacian regularizer of the latent mesh (Sec. 5.3, "Objective
// function"):
//   delta_i = v_i - (1/|N_i|) sum_{j in N_i} v_j      (N_i: one-ring of i)
//   L_delta = (1/n) sum_i |delta_i - delta'_i|^2
//   dL/dv_v = (2/n) (r_v - sum_{i in N_v} r_i / |N_i|),  r = delta - delta'
// The one-ring is symmetric, so the adjoint is a gather over the same
// neighbour lists: no atomics, and the same bits on every run.
#include <algorithm>
#include <vector>

#include "dev.h"

namespace adr {

__global__ __launch_bounds__(256) void k_lap_delta(int n, const float* __restrict__ pos,
                                                   const int* __restrict__ offs, const int* __restrict__ nbr,
                                                   const float* __restrict__ dref, float* __restrict__ r,
                                                   float* __restrict__ dout, double* __restrict__ part) {
  __shared__ double red[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < n) {
    const int a = offs[i], b = offs[i + 1];
    d3 s = dmk(0.0, 0.0, 0.0);
    for (int k = a; k < b; ++k) s = s + dld3f(pos, nbr[k]);
    d3 d = dld3f(pos, i);
    if (b > a) d = d - (1.0 / (b - a)) * s;
    else d = dmk(0.0, 0.0, 0.0);
    if (dout) st3(dout, i, mk((float)d.x, (float)d.y, (float)d.z));
    if (dref) d = d - dld3f(dref, i);
    st3(r, i, mk((float)d.x, (float)d.y, (float)d.z));
    e = ddot(d, d);
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_lap_loss(const double* __restrict__ part, int nb, int n,
                                                  float* __restrict__ loss) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) acc += part[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(red[0] / n);
}

__global__ __launch_bounds__(256) void k_lap_grad(int n, const int* __restrict__ offs, const int* __restrict__ nbr,
                                                  const float* __restrict__ r, float scale,
                                                  float* __restrict__ gpos) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  d3 g = dld3f(r, v);
  for (int k = offs[v]; k < offs[v + 1]; ++k) {
    const int i = nbr[k];
    const int c = offs[i + 1] - offs[i];
    g = g - (1.0 / c) * dld3f(r, i);
  }
  g = (double)scale * g;
  gpos[3 * v] += (float)g.x;
  gpos[3 * v + 1] += (float)g.y;
  gpos[3 * v + 2] += (float)g.z;
}

hipError_t launch_laplacian(int n, const float* pos, const int* offs, const int* nbr, const float* dref,
                            float lambda, float* r, double* part, float* dout, float* loss, float* gpos,
                            hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_lap_delta, dim3(nb), dim3(256), 0, st, n, pos, offs, nbr, dref, r, dout, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (loss) {
    hipLaunchKernelGGL(k_lap_loss, dim3(1), dim3(256), 0, st, part, nb, n, loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (gpos) {
    hipLaunchKernelGGL(k_lap_grad, dim3(nb), dim3(256), 0, st, n, offs, nbr, r, 2.0f * lambda / n, gpos);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace adr

using namespace adr;

// Host: sorted one-ring neighbour lists in CSR form.
extern "C" adr_status adr_mesh_one_ring(const int32_t* tri, int32_t n_tri, int32_t n_pos, int32_t* offs,
                                        int32_t* nbr, int64_t* n_nbr) {
  if (n_tri < 0 || n_pos < 0 || (n_tri > 0 && !tri) || !offs || !n_nbr)
    return report(ADR_E_INVALID, "one_ring: bad arguments");
  std::vector<std::vector<int32_t>> ring(n_pos);
  for (int64_t t = 0; t < n_tri; ++t)
    for (int k = 0; k < 3; ++k) {
      const int32_t a = tri[3 * t + k], b = tri[3 * t + (k + 1) % 3];
      if (a < 0 || a >= n_pos || b < 0 || b >= n_pos) return report(ADR_E_INVALID, "one_ring: index out of range");
      if (a == b) continue;
      ring[a].push_back(b);
      ring[b].push_back(a);
    }
  int64_t total = 0;
  offs[0] = 0;
  for (int32_t i = 0; i < n_pos; ++i) {
    std::vector<int32_t>& r = ring[i];
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    if (nbr) std::copy(r.begin(), r.end(), nbr + total);
    total += (int64_t)r.size();
    if (total > INT32_MAX) return report(ADR_E_INVALID, "one_ring: too many entries");
    offs[i + 1] = (int32_t)total;
  }
  *n_nbr = total;
  return ADR_OK;
}
