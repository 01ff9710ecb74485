// scan.h -- the single-pass device-wide exclusive scan (decoupled look-back)
// and its wave/block helpers, shared by the sort, the segment tables and the
// node-block maps.  A scan is instantiated with an input functor in(i, n)
// and an output functor out(i, value, exclusive prefix, n).
#pragma once

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

// ---------------------------------------------------------------------------
// single-pass exclusive scan
// ---------------------------------------------------------------------------
// Inputs in(i, n) (pure: the look-back may evaluate a tile's inputs again)
// and outputs out(i, value, exclusive prefix, n) of the single-pass scan.
struct ArrayIn {
  const int32_t *p;
  __device__ __forceinline__ int operator()(int64_t i, int64_t) const { return p[i]; }
};
struct ArrayOut {
  int32_t *p;
  int mode;  // 1: -1 where the value is 0 (slot maps)
  __device__ __forceinline__ void operator()(int64_t i, int v, int run, int64_t) const {
    p[i] = (mode == 1 && v == 0) ? -1 : run;
  }
};

template <int ITEMS, typename In>
__device__ uint32_t tile_sum(const In &in, int64_t n, int64_t tile) {
  constexpr int64_t kTile = (int64_t)kScanThreads * ITEMS;
  uint32_t s = 0;
  const int64_t lo = tile * kTile, hi = lo + kTile < n ? lo + kTile : n;
  for (int64_t i = lo; i < hi; ++i) s += (uint32_t)in(i, n);
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

// Tile t (of tiles 0..last holding data) of one scan: reads its inputs,
// publishes its aggregate, looks back for its prefix in flags[0, t) and
// writes its outputs.  The caller signals lb_finish afterwards.
template <typename In, typename Out, int ITEMS>
__device__ __forceinline__ void scan_tile(const In &in, const Out &out, int64_t n, int t, int last,
                                          int64_t *total, uint64_t *flags, uint32_t epoch) {
  __shared__ int lds[kScanThreads / 64];
  __shared__ uint32_t s_excl;
  constexpr int64_t kTile = (int64_t)kScanThreads * ITEMS;
  const int64_t base = (int64_t)t * kTile + (int64_t)threadIdx.x * ITEMS;
  int v[ITEMS];
  int s = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? in(i, n) : 0;
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
      excl = wave_lookback(flags, 1, t, epoch, [&](int j) { return tile_sum<ITEMS>(in, n, j); });
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
  for (int k = 0; k < ITEMS; ++k) {
    const int64_t i = base + k;
    if (i < n) out(i, v[k], run, n);
    run += v[k];
  }
}

template <int ITEMS>
__device__ __forceinline__ int scan_last_tile(int64_t n) {
  constexpr int64_t kTile = (int64_t)kScanThreads * ITEMS;
  return n > 0 ? (int)((n - 1) / kTile) : 0;  // last tile holding data
}

// ITEMS consecutive elements per thread (kScanItems for long arrays; 1 for
// short tables whose per-element work is heavy, so that they spread over
// more workgroups).
template <typename In, typename Out, int ITEMS = kScanItems>
__global__ __launch_bounds__(kScanThreads) void k_scan_onepass(In in, Out out, int64_t n_cap,
                                                               const int64_t *n_dev,
                                                               int64_t *total, uint64_t *flags,
                                                               uint32_t *state) {
  const int64_t n = dev_count(n_cap, n_dev);
  const int t = blockIdx.x;
  const uint32_t epoch = lb_epoch(state);
  const int last = scan_last_tile<ITEMS>(n);
  if (t > last) return;  // past the live count: takes no part
  scan_tile<In, Out, ITEMS>(in, out, n, t, last, total, flags, epoch);
  if (threadIdx.x == 0) lb_finish(state, epoch, last + 1);
}

// Two independent scans in one launch: workgroups [0, tiles0) take the
// first (flags[0, tiles0)), the rest the second (flags from tiles0 on).
// Each scan's tile 0 starts its own look-back chain; one epoch covers both.
template <typename In, typename Out, int ITEMS = kScanItems>
__global__ __launch_bounds__(kScanThreads) void k_scan_pair(In in0, Out out0, int64_t cap0,
                                                            const int64_t *n0_dev, int64_t *total0,
                                                            In in1, Out out1, int64_t cap1,
                                                            const int64_t *n1_dev, int64_t *total1,
                                                            int tiles0, uint64_t *flags,
                                                            uint32_t *state) {
  const int64_t n0 = dev_count(cap0, n0_dev), n1 = dev_count(cap1, n1_dev);
  const int last0 = scan_last_tile<ITEMS>(n0), last1 = scan_last_tile<ITEMS>(n1);
  const uint32_t epoch = lb_epoch(state);
  const int b = blockIdx.x;  // workgroup-uniform branches
  if (b < tiles0) {
    if (b > last0) return;
    scan_tile<In, Out, ITEMS>(in0, out0, n0, b, last0, total0, flags, epoch);
  } else {
    const int t = b - tiles0;
    if (t > last1) return;
    scan_tile<In, Out, ITEMS>(in1, out1, n1, t, last1, total1, flags + tiles0, epoch);
  }
  if (threadIdx.x == 0) lb_finish(state, epoch, last0 + last1 + 2);
}

inline unsigned scan_tiles(int64_t n_cap, int items = kScanItems) {
  const int64_t tile = (int64_t)kScanThreads * items;
  int64_t ntiles = (n_cap + tile - 1) / tile;
  return (unsigned)(ntiles < 1 ? 1 : ntiles);
}

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

// Count this lane's 8-bit digit d (if ok) into the LDS histogram h: the
// lowest lane of each group of equal digits adds the group's size.
__device__ __forceinline__ void count_digit(uint32_t *h, bool ok, uint32_t d) {
  const uint64_t peers = match_digit(d, __ballot(ok));
  if (ok && (peers & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
}

}  // namespace apic
