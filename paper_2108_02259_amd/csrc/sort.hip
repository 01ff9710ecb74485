// sort.hip -- device-wide exclusive scan, fills, and the stable LSD radix sort
// of 32-bit cell keys.  The sort is bit-exact: ties keep input order because
// each pass ranks equal digits by (round, wave, lane), which is input order.
#include "kernels.h"

namespace apic {

// ---------------------------------------------------------------------------
// wave / block scan helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_inclusive_scan(int x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread across a kScanThreads block; returns
// the block total in *total (all threads).
__device__ __forceinline__ int block_exclusive_scan(int x, int *lds, int *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kScanThreads / 64;
  int inc = wave_inclusive_scan(x);
  if (lane == 63) lds[wave] = inc;
  __syncthreads();
  int woff = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    int s = lds[w];
    if (w < wave) woff += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return woff + inc - x;
}

__device__ __forceinline__ int64_t dev_count(int64_t n_cap, const int64_t *n_dev) {
  if (!n_dev) return n_cap;
  int64_t n = *n_dev;
  return n < n_cap ? n : n_cap;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t *in, int64_t n_cap,
                                                              const int64_t *n_dev,
                                                              int32_t *partial) {
  __shared__ int lds[kScanThreads / 64];
  const int64_t n = dev_count(n_cap, n_dev);
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) s += in[i];
  }
  int tot;
  (void)block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Single workgroup: exclusive scan of the tile partials, total to *total.
__global__ __launch_bounds__(1024) void k_scan_partials(int32_t *partial, int ntiles,
                                                        int64_t *total) {
  __shared__ int lds[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t carry = 0;
  for (int base = 0; base < ntiles; base += 1024) {
    int i = base + threadIdx.x;
    int x = i < ntiles ? partial[i] : 0;
    int inc = wave_inclusive_scan(x);
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    int woff = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      int s = lds[w];
      if (w < wave) woff += s;
      tot += s;
    }
    if (i < ntiles) partial[i] = (int32_t)(carry + woff + inc - x);
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const int32_t *in, int32_t *out,
                                                            int64_t n_cap, const int64_t *n_dev,
                                                            const int32_t *partial, int mode) {
  __shared__ int lds[kScanThreads / 64];
  const int64_t n = dev_count(n_cap, n_dev);
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  int tot;
  int ex = block_exclusive_scan(s, lds, &tot) + partial[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = (mode == 1 && v[k] == 0) ? -1 : ex;
    ex += v[k];
  }
}

void scan_exclusive(const int32_t *in, int32_t *out, int64_t n_cap, const int64_t *n_dev,
                    int64_t *total, int32_t *partial, int mode, hipStream_t st) {
  int64_t ntiles = (n_cap + kScanTile - 1) / kScanTile;
  if (ntiles < 1) ntiles = 1;
  APIC_LAUNCH(k_scan_reduce, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, in, n_cap, n_dev, partial);
  APIC_LAUNCH(k_scan_partials, dim3(1), dim3(1024), 0, st, partial, (int)ntiles, total);
  APIC_LAUNCH(k_scan_down, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, in, out, n_cap, n_dev, partial, mode);
}

// ---------------------------------------------------------------------------
// fills (kernels, so that they can be captured in graphs)
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int32_t value, int64_t n_cap, const int64_t *n_dev,
                           int64_t scale) {
  int64_t n = dev_count(n_cap, n_dev) * scale;
  if (n > n_cap * scale) n = n_cap * scale;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

void fill_i32(int32_t *p, int32_t value, int64_t n_cap, const int64_t *n_dev, int64_t scale,
              hipStream_t st) {
  int64_t tot = n_cap * scale;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  APIC_LAUNCH(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, value, n_cap, n_dev, scale);
}

__global__ void k_zero_u32(uint32_t *p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

void fill_bytes_zero(void *p, int64_t bytes, hipStream_t st) {
  int64_t words = bytes / 4;
  int64_t blocks = (words + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  APIC_LAUNCH(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t *)p, words);
}

// Zero (count[0] * per) elements of `elem_bytes` bytes each, count on device.
__global__ void k_zero_counted(uint32_t *p, int64_t words_cap, const int32_t *count,
                               int64_t words_per) {
  int64_t words = (int64_t)(*count) * words_per;
  if (words > words_cap) words = words_cap;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

void fill_zero_f(void *p, int64_t elems_cap, const int32_t *n_dev, int64_t per, int elem_bytes,
                 hipStream_t st) {
  int64_t words_per = per * elem_bytes / 4;
  int64_t cap = elems_cap * words_per;
  int64_t blocks = (cap + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  APIC_LAUNCH(k_zero_counted, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t *)p, cap, n_dev, words_per);
}

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------
// Lanes of the wave whose 8-bit digit equals this lane's (restricted to `valid`).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid) {
  uint64_t m = valid;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    uint64_t bb = __ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? bb : ~bb;
  }
  return m;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *keys, int64_t n,
                                                             int shift, uint32_t *hist,
                                                             int ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
    bool ok = i < n;
    uint32_t d = ok ? (keys[i] >> shift) & 255u : 0u;
    uint64_t valid = __ballot(ok);
    uint64_t peers = match_digit(d, valid);
    if (ok && (peers & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, int64_t n,
    int shift, const int32_t *offs, int ntiles, int identity) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kSortThreads / 64][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  base[tid] = (uint32_t)offs[(int64_t)tid * ntiles + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const int64_t tbase = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = tbase + (int64_t)r * kSortThreads + tid;
    bool ok = i < n;
    uint32_t key = ok ? kin[i] : 0u;
    uint32_t val = ok ? (identity ? (uint32_t)i : vin[i]) : 0u;
    uint32_t d = (key >> shift) & 255u;
    uint64_t valid = __ballot(ok);
    uint64_t peers = match_digit(d, valid);
    int rank = __popcll(peers & lanemask_lt());
    if (ok && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (ok) {
      uint32_t pos = base[d] + (uint32_t)rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / 64; ++w) {
      add += wcnt[w][tid];
      wcnt[w][tid] = 0;
    }
    base[tid] += add;
    __syncthreads();
  }
  (void)lane;
}

int radix_sort(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, int64_t n, int bits,
               uint32_t *hist, int32_t *partial, int64_t *total, hipStream_t st) {
  const int64_t ntiles = sort_tiles(n);
  int passes = (bits + 7) / 8;
  if (passes < 1) passes = 1;
  uint32_t *ki = ka, *vi = va, *ko = kb, *vo = vb;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    APIC_LAUNCH(k_radix_hist, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, ki, n, shift, hist, (int)ntiles);
    scan_exclusive((const int32_t *)hist, (int32_t *)hist, 256 * ntiles, nullptr, total,
                   partial, 0, st);
    APIC_LAUNCH(k_radix_scatter, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, 
        ki, vi, ko, vo, n, shift, (const int32_t *)hist, (int)ntiles, p == 0 ? 1 : 0);
    uint32_t *tk = ki, *tv = vi;
    ki = ko;
    vi = vo;
    ko = tk;
    vo = tv;
  }
  return (passes & 1) ? 1 : 0;
}

}  // namespace apic
