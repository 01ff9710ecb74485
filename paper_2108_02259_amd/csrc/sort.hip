// sort.hip -- single-pass device-wide exclusive scans, fills, and the stable
// LSD radix sort of 32-bit cell keys.  The sort is bit-exact: ties keep input
// order because each pass ranks equal digits by (tile, round, wave, lane),
// which is input order.
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

// ---------------------------------------------------------------------------
// decoupled look-back
// ---------------------------------------------------------------------------
// Tiles publish their partial sums in 64-bit flag words: the launch's epoch
// (30 bits), a status (aggregate of the tile alone, or inclusive prefix up to
// the tile) and a 32-bit value, written and read as single relaxed atomics at
// device scope (the value travels inside the word, so no fences are needed).
// A waiting tile polls a predecessor a bounded number of times; if the word
// has still not appeared it recomputes that predecessor's aggregate from the
// input, which no tile modifies (the scans are out of place), so every wait
// ends.  The last tile to finish advances the epoch for the next launch, so
// the flags never need clearing; no tile can read the advanced epoch before
// every tile of the launch has read its own.
constexpr uint64_t kLbAgg = 1, kLbIncl = 2;
constexpr int kLbSpin = 4096;

__device__ __forceinline__ uint64_t lb_pack(uint32_t epoch, uint64_t status, uint32_t value) {
  return ((uint64_t)(epoch & 0x3fffffffu) << 34) | (status << 32) | (uint64_t)value;
}
__device__ __forceinline__ bool lb_valid(uint64_t f, uint32_t epoch) {
  return (f >> 34) == (uint64_t)(epoch & 0x3fffffffu) && ((f >> 32) & 3u) != 0;
}
__device__ __forceinline__ uint64_t lb_load(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t lb_epoch(const uint32_t *state) {
  return __hip_atomic_load(&state[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Called once per taking-part tile after its last use of the flags; the
// last of `tiles` tiles to arrive advances the epoch.
__device__ __forceinline__ void lb_finish(uint32_t *state, uint32_t epoch, int tiles) {
  if (atomicAdd(&state[0], 1u) == (uint32_t)(tiles - 1)) {
    __hip_atomic_store(&state[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&state[1], epoch + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

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

// ---------------------------------------------------------------------------
// single-pass exclusive scan
// ---------------------------------------------------------------------------
struct ArrayIn {
  const int32_t *p;
  __device__ __forceinline__ int operator()(int64_t i) const { return p[i]; }
};
// 1 where a new 4x4x4-block segment starts in the sorted keys.
struct SegHeadIn {
  const uint32_t *keys;
  __device__ __forceinline__ int operator()(int64_t i) const {
    return (i == 0 || (keys[i] >> 6) != (keys[i - 1] >> 6)) ? 1 : 0;
  }
};

template <typename In>
__device__ uint32_t tile_sum(const In &in, int64_t n, int64_t tile) {
  uint32_t s = 0;
  const int64_t lo = tile * kScanTile, hi = lo + kScanTile < n ? lo + kScanTile : n;
  for (int64_t i = lo; i < hi; ++i) s += (uint32_t)in(i);
  return s;
}

// Exclusive prefix of tile t from the flags of tiles < t, read by the 64
// lanes of the calling wave one window of 64 predecessors at a time: lane k
// reads tile (top - k); the window's nearest inclusive prefix ends the walk.
// `fallback(j)` recomputes tile j's aggregate when its flag does not appear.
template <typename Fallback>
__device__ uint32_t wave_lookback(const uint64_t *flags, int64_t stride, int t, uint32_t epoch,
                                  const Fallback &fallback) {
  const int lane = threadIdx.x & 63;
  uint32_t excl = 0;
  for (int top = t - 1; top >= 0; top -= 64) {
    const int j = top - lane;
    uint64_t f = 0;
    if (j >= 0) {
      f = lb_load(&flags[(int64_t)j * stride]);
      for (int spin = 0; !lb_valid(f, epoch); ++spin) {
        if (spin >= kLbSpin) {
          f = lb_pack(epoch, kLbAgg, fallback(j));
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        f = lb_load(&flags[(int64_t)j * stride]);
      }
    }
    // tile 0 is always inclusive, so j < 0 never has to be summed
    const bool incl = j >= 0 && ((f >> 32) & 3u) == kLbIncl;
    const uint64_t im = __ballot(incl);
    const int stop = im ? __ffsll((unsigned long long)im) - 1 : 64;  // nearest inclusive lane
    uint32_t v = (j >= 0 && lane <= stop) ? (uint32_t)f : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    excl += v;
    if (im) break;
  }
  return excl;
}

template <typename In>
__global__ __launch_bounds__(kScanThreads) void k_scan_onepass(In in, int32_t *out, int64_t n_cap,
                                                               const int64_t *n_dev,
                                                               int64_t *total, uint64_t *flags,
                                                               uint32_t *state, int mode) {
  __shared__ int lds[kScanThreads / 64];
  __shared__ uint32_t s_excl;
  const int64_t n = dev_count(n_cap, n_dev);
  const int t = blockIdx.x;
  const uint32_t epoch = lb_epoch(state);
  const int last = n > 0 ? (int)((n - 1) / kScanTile) : 0;  // last tile holding data
  if (t > last) return;  // past the live count: takes no part
  const int64_t base = (int64_t)t * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? in(i) : 0;
    s += v[k];
  }
  int tot;
  const int ex = block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x < 64) {
    uint32_t excl = 0;
    if (t == 0) {
      if (threadIdx.x == 0) lb_store(&flags[0], lb_pack(epoch, kLbIncl, (uint32_t)tot));
    } else {
      if (threadIdx.x == 0) lb_store(&flags[t], lb_pack(epoch, kLbAgg, (uint32_t)tot));
      excl = wave_lookback(flags, 1, t, epoch, [&](int j) { return tile_sum(in, n, j); });
      if (threadIdx.x == 0) lb_store(&flags[t], lb_pack(epoch, kLbIncl, excl + (uint32_t)tot));
    }
    if (threadIdx.x == 0) {
      s_excl = excl;
      if (t == last) *total = (int64_t)excl + tot;
    }
  }
  __syncthreads();
  int run = (int)s_excl + ex;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = (mode == 1 && v[k] == 0) ? -1 : run;
    run += v[k];
  }
  if (threadIdx.x == 0) lb_finish(state, epoch, last + 1);
}

static unsigned scan_tiles(int64_t n_cap) {
  int64_t ntiles = (n_cap + kScanTile - 1) / kScanTile;
  return (unsigned)(ntiles < 1 ? 1 : ntiles);
}

void scan_exclusive(const int32_t *in, int32_t *out, int64_t n_cap, const int64_t *n_dev,
                    int64_t *total, const Lookback &lb, int mode, hipStream_t st) {
  ArrayIn a{in};
  APIC_LAUNCH(k_scan_onepass<ArrayIn>, dim3(scan_tiles(n_cap)), dim3(kScanThreads), 0, st, a, out,
              n_cap, n_dev, total, lb.flags, lb.state, mode);
}

void scan_segment_heads(const uint32_t *keys, int32_t *seg_id, int64_t n, int64_t *total,
                        const Lookback &lb, hipStream_t st) {
  SegHeadIn a{keys};
  APIC_LAUNCH(k_scan_onepass<SegHeadIn>, dim3(scan_tiles(n)), dim3(kScanThreads), 0, st, a,
              seg_id, n, (const int64_t *)nullptr, total, lb.flags, lb.state, 0);
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
    const uint32_t d = ok ? (keys[i] >> shift) & 255u : 0u;
    const uint64_t peers = match_digit(d, __ballot(ok));
    if (ok && (peers & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
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
               int bits, uint32_t *hist, const Lookback &lb, hipStream_t st) {
  const int64_t ntiles = sort_tiles(n);
  const int64_t hw = 256 * ntiles;  // words of the digit-count table
  int passes = (bits - lo + 7) / 8;
  if (passes < 1) passes = 1;
  if (passes > 4) passes = 4;
  int32_t *offs = (int32_t *)(hist + hw);
  int64_t *total = (int64_t *)(hist + 2 * hw);  // 8-byte aligned scratch (hw is even)
  uint32_t *ki = ka, *vi = va, *ko = kb, *vo = vb;
  for (int p = 0; p < passes; ++p) {
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
