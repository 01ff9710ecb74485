// sort.hip -- single-pass device-wide exclusive scans, fills, and the stable
// LSD radix sort of 32-bit cell keys.  The sort is bit-exact: ties keep input
// order because each pass ranks equal digits by (tile, round, wave, lane),
// which is input order.
#include "scan.h"

namespace apic {

// ---------------------------------------------------------------------------
// look-back state
// ---------------------------------------------------------------------------
__global__ void k_lookback_init(uint64_t *flags, int64_t cap, uint32_t *state) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap;
       i += (int64_t)gridDim.x * blockDim.x)
    flags[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    state[0] = 0;
    state[1] = 1;
  }
}

void lookback_init(const Lookback &lb, hipStream_t st) {
  int64_t blocks = (lb.capacity + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
  APIC_LAUNCH(k_lookback_init, dim3((unsigned)blocks), dim3(256), 0, st, lb.flags, lb.capacity,
              lb.state);
}

void scan_exclusive(const int32_t *in, int32_t *out, int64_t n_cap, const int64_t *n_dev,
                    int64_t *total, const Lookback &lb, int mode, hipStream_t st) {
  ArrayIn a{in};
  ArrayOut o{out, mode};
  APIC_LAUNCH((k_scan_onepass<ArrayIn, ArrayOut>), dim3(scan_tiles(n_cap)), dim3(kScanThreads), 0,
              st, a, o, n_cap, n_dev, total, lb.flags, lb.state);
}

void scan_exclusive_pair(const int32_t *in0, int32_t *out0, int64_t cap0, const int64_t *n0_dev,
                         int64_t *total0, const int32_t *in1, int32_t *out1, int64_t cap1,
                         const int64_t *n1_dev, int64_t *total1, const Lookback &lb, int mode,
                         hipStream_t st) {
  const unsigned tiles0 = scan_tiles(cap0), tiles1 = scan_tiles(cap1);
  APIC_LAUNCH((k_scan_pair<ArrayIn, ArrayOut>), dim3(tiles0 + tiles1), dim3(kScanThreads), 0, st,
              ArrayIn{in0}, ArrayOut{out0, mode}, cap0, n0_dev, total0, ArrayIn{in1},
              ArrayOut{out1, mode}, cap1, n1_dev, total1, (int)tiles0, lb.flags, lb.state);
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
// Digit counts per tile, digit-major (h[d * ntiles + t]).
__global__ __launch_bounds__(kSortThreads) void k_radix_tilehist(const uint32_t *keys, int64_t n,
                                                                 int ntiles, int shift,
                                                                 uint32_t *h0) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x, t = blockIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t tbase = (int64_t)t * kSortTile;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = tbase + (int64_t)r * kSortThreads + tid;
    const bool ok = i < n;
    count_digit(h, ok, ok ? (keys[i] >> shift) & 255u : 0u);
  }
  __syncthreads();
  h0[(int64_t)tid * ntiles + t] = h[tid];
}

// One stable pass: key i of tile t goes to offs[digit * ntiles + t] plus its
// rank among the tile's keys of that digit (round, wave, lane order = input
// order).
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, int64_t n,
    int shift, const int32_t *offs, int ntiles, int identity) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kSortThreads / 64][256];
  const int tid = threadIdx.x, wave = tid >> 6;
  const int t = blockIdx.x;
  base[tid] = (uint32_t)offs[(int64_t)tid * ntiles + t];
#pragma unroll
  for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const int64_t tbase = (int64_t)t * kSortTile;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = tbase + (int64_t)r * kSortThreads + tid;
    const bool ok = i < n;
    const uint32_t key = ok ? kin[i] : 0u;
    const uint32_t val = ok ? (identity ? (uint32_t)i : vin[i]) : 0u;
    const uint32_t d = (key >> shift) & 255u;
    const uint64_t peers = match_digit(d, __ballot(ok));
    const int rank = __popcll(peers & lanemask_lt());
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
}

int radix_sort(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, int64_t n, int lo,
               int bits, uint32_t *hist, const Lookback &lb, bool hist0_ready, hipStream_t st) {
  const int64_t ntiles = sort_tiles(n);
  const int64_t hw = 256 * ntiles;  // words of the digit-count table
  int passes = (bits - lo + 7) / 8;
  if (passes < 1) passes = 1;
  if (passes > 4) passes = 4;
  int32_t *offs = (int32_t *)(hist + hw);
  int64_t *total = (int64_t *)(hist + 2 * hw);  // 8-byte aligned scratch (hw is even)
  uint32_t *ki = ka, *vi = va, *ko = kb, *vo = vb;
  for (int p = 0; p < passes; ++p) {
    if (p > 0 || !hist0_ready)
      APIC_LAUNCH(k_radix_tilehist, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, ki, n,
                  (int)ntiles, lo + 8 * p, hist);
    scan_exclusive((const int32_t *)hist, offs, hw, nullptr, total, lb, 0, st);
    APIC_LAUNCH(k_radix_scatter, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, ki, vi, ko,
                vo, n, lo + 8 * p, (const int32_t *)offs, (int)ntiles, p == 0 ? 1 : 0);
    uint32_t *tk = ki, *tv = vi;
    ki = ko;
    vi = vo;
    ko = tk;
    vo = tv;
  }
  return (passes & 1) ? 1 : 0;
}

}  // namespace apic
