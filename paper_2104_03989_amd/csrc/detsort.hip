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
//  scatter: the tile's pairs in eight rounds of 256 (round r, thread t: tile
//           position 256 r + t); a pair goes to its digit's start in this
//           tile plus the number of pairs of that digit before it in the
//           tile: those of earlier rounds (a running count per digit), of
//           earlier waves in this round (per-wave digit counts) and of lower
//           lanes in its wave (the lanes whose digit matches, from eight
//           ballots).  Equal digits keep their order: the sort is stable.

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
  __shared__ uint32_t run[256];    // per digit: where its next pair goes
  __shared__ uint32_t wc[4][256];  // per wave: this round's pairs of each digit
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  run[t] = start[(int64_t)t * tiles + blockIdx.x];
  wc[0][t] = wc[1][t] = wc[2][t] = wc[3][t] = 0u;
  __syncthreads();
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t i = base + (int64_t)r * kScanBlock + t;
    const bool ok = i < n;
    const uint32_t key = ok ? kin[i] : 0u, val = ok ? vin[i] : 0u;
    const uint32_t d = (key >> shift) & 0xFFu;
    // the lanes of this wave holding a pair of the same digit
    unsigned long long m = __ballot(ok);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const unsigned long long bb = __ballot((d >> bit) & 1u);
      m &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const uint32_t before = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (ok && before == 0) wc[w][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (ok) {
      uint32_t pos = run[d] + before;
      for (int w2 = 0; w2 < w; ++w2) pos += wc[w2][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    // thread t advances digit t's running count and clears its wave counts
    run[t] += (wc[0][t] + wc[1][t]) + (wc[2][t] + wc[3][t]);
    wc[0][t] = wc[1][t] = wc[2][t] = wc[3][t] = 0u;
    __syncthreads();
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
