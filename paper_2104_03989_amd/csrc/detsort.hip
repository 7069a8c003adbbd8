// Building blocks of the deterministic gradient mode: a device-wide
// exclusive scan of 32-bit counts and a stable LSD radix sort of
// (key, index) pairs.  Texel-gradient contributions are written at positions
// fixed by (pixel, map, level, corner); sorting them stably by texel key
// puts each texel's contributions next to each other in that fixed order, so
// a segmented sum gives the same bits on every run, whatever the scheduling.
#include "dev.h"

namespace adr {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;  // 2048 values per block

// Exclusive scan of the 256 values of a block (one per thread), in LDS.
// Returns this thread's exclusive prefix; *total receives the block's sum.
__device__ __forceinline__ uint32_t block_exscan(uint32_t x, uint32_t* lds, uint32_t* total) {
  const int t = threadIdx.x;
  lds[t] = x;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    uint32_t y = t >= off ? lds[t - off] : 0u;
    __syncthreads();
    lds[t] += y;
    __syncthreads();
  }
  uint32_t incl = lds[t];
  *total = lds[kScanBlock - 1];
  __syncthreads();
  return incl - x;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                            uint32_t* __restrict__ sums) {
  __shared__ uint32_t lds[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) s += base + k < n ? in[base + k] : 0u;
  uint32_t total;
  block_exscan(s, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block scans the block sums (any count, in chunks of the block size).
__global__ __launch_bounds__(kScanBlock) void k_scan_top(uint32_t* __restrict__ sums, int64_t n) {
  __shared__ uint32_t lds[kScanBlock];
  uint32_t carry = 0;
  for (int64_t c = 0; c < n; c += kScanBlock) {
    const int64_t i = c + threadIdx.x;
    uint32_t x = i < n ? sums[i] : 0u, total;
    uint32_t ex = block_exscan(x, lds, &total);
    if (i < n) sums[i] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_down(const uint32_t* __restrict__ in, int64_t n,
                                                          const uint32_t* __restrict__ sums,
                                                          uint32_t* __restrict__ out) {
  __shared__ uint32_t lds[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems], s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = sums[blockIdx.x] + block_exscan(s, lds, &total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

int64_t scan_tmp_words(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

// out[i] = sum of in[0..i) (in and out may alias); tmp: scan_tmp_words(n) words.
hipError_t launch_exscan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = scan_tmp_words(n);
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, st, tmp, nb);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, tmp, out);
  return hipGetLastError();
}

// ------------------------------------------------------------- radix sort
// One pass per 8-bit digit.  Tiles of 2048 pairs per block, in array order.
//  hist:    per tile, digit counts -> hist[digit * tiles + tile]
//  scan:    exclusive scan of hist (digit-major): each (digit, tile) start
//  scatter: the tile is sorted by the digit in LDS with eight stable one-bit
//           splits, then each pair goes to its digit's start plus its rank.

__global__ __launch_bounds__(kScanBlock) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                        int64_t tiles, uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kScanBlock) {
    const int64_t i = base + k;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kScanBlock) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin, int64_t n, int shift,
                                                           int64_t tiles, const uint32_t* __restrict__ start,
                                                           uint32_t* __restrict__ kout,
                                                           uint32_t* __restrict__ vout) {
  __shared__ uint32_t sk[2][kScanTile];
  __shared__ uint32_t sv[2][kScanTile];
  __shared__ uint32_t lds[kScanBlock];
  __shared__ uint32_t dstart[256];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int cnt = (int)min((int64_t)kScanTile, n - base);
  // blocked arrangement: thread t owns tile positions t*8 .. t*8+7
  for (int k = t; k < kScanTile; k += kScanBlock) {
    const int64_t i = base + k;
    sk[0][k] = k < cnt ? kin[i] : 0xFFFFFFFFu;  // padding sorts last and is dropped
    sv[0][k] = k < cnt ? vin[i] : 0u;
  }
  __syncthreads();
  int cur = 0;
  for (int b = 0; b < 8; ++b) {
    uint32_t zeros = 0;
    uint32_t kk[kScanItems], vv[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      kk[j] = sk[cur][t * kScanItems + j];
      vv[j] = sv[cur][t * kScanItems + j];
      zeros += ((kk[j] >> (shift + b)) & 1u) ? 0u : 1u;
    }
    uint32_t total_zeros;
    uint32_t z = block_exscan(zeros, lds, &total_zeros);
    uint32_t o = (uint32_t)t * kScanItems - z;  // ones before this thread's items
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const bool one = (kk[j] >> (shift + b)) & 1u;
      const uint32_t pos = one ? total_zeros + o : z;
      sk[cur ^ 1][pos] = kk[j];
      sv[cur ^ 1][pos] = vv[j];
      if (one) ++o; else ++z;
    }
    cur ^= 1;
    __syncthreads();
  }
  // first local position of each digit, from the tile's sorted keys
  dstart[t] = 0xFFFFFFFFu;
  __syncthreads();
  for (int k = t; k < cnt; k += kScanBlock) {
    const uint32_t d = (sk[cur][k] >> shift) & 0xFFu;
    if (k == 0 || ((sk[cur][k - 1] >> shift) & 0xFFu) != d) dstart[d] = (uint32_t)k;
  }
  __syncthreads();
  for (int k = t; k < cnt; k += kScanBlock) {
    const uint32_t key = sk[cur][k];
    const uint32_t d = (key >> shift) & 0xFFu;
    const uint32_t pos = start[(int64_t)d * tiles + blockIdx.x] + ((uint32_t)k - dstart[d]);
    kout[pos] = key;
    vout[pos] = sv[cur][k];
  }
}

int64_t radix_hist_words(int64_t n) { return 256 * ((n + kScanTile - 1) / kScanTile); }

// Stable sort of n (key, value) pairs by the low `bits` bits of the keys.
// Sorted output ends in (k0, v0) if the number of passes is even, else in
// (k1, v1); *in_first tells which.  hist: radix_hist_words(n) words; tmp:
// scan_tmp_words(radix_hist_words(n)) words.
hipError_t launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n, int bits,
                             uint32_t* hist, uint32_t* tmp, bool* in_first, hipStream_t st) {
  *in_first = true;
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  uint32_t *ka = k0, *va = v0, *kb = k1, *vb = v1;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)tiles), dim3(kScanBlock), 0, st, ka, n, shift, tiles, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_exscan_u32(hist, hist, 256 * tiles, tmp, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)tiles), dim3(kScanBlock), 0, st, ka, va, n, shift, tiles, hist,
                       kb, vb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint32_t* tk = ka; ka = kb; kb = tk;
    uint32_t* tv = va; va = vb; vb = tv;
    *in_first = !*in_first;
  }
  return hipSuccess;
}

}  // namespace adr
