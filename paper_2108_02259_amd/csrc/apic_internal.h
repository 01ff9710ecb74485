// apic_internal.h -- internal types shared by the HIP translation units of the
// contact library.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apic_contact.h"

namespace apic {

// Optional timing of every launch: when a timer is installed (eager profiled
// steps), kernels are launched with HIP's extended launch, which records a
// start/stop event pair with the dispatch itself on the launch stream.
struct LaunchTimer {
  virtual void events(hipEvent_t *start, hipEvent_t *stop) = 0;
  virtual ~LaunchTimer() = default;
};
extern thread_local LaunchTimer *g_launch_timer;

// ---------------------------------------------------------------------------
// Layout constants
// ---------------------------------------------------------------------------
// A "block" is 4x4x4 grid cells.  A particle in cell c (per axis) touches the
// quadratic-spline nodes c-1 .. c+2 (Appendix B).  Node blocks are shifted by
// one node: node block k holds nodes 4k-1 .. 4k+2, so every particle of cell
// block B touches only node blocks B and B+1 per axis (8 node blocks).  The
// LDS tile of a cell block is the 8x8x8 node cube of those 8 node blocks;
// local node l = (cell in block) + stencil offset, 0 <= l < 7 per axis.
constexpr int kBlock = 4;
constexpr int kNodesPerBlock = 64;
constexpr int kTileX = 8;               // tile row length
constexpr int kTileY = 8;               // rows per slab
constexpr int kTileZStride = 8 * 8 + 4; // padded slab stride (LDS banks)
// Elements per component of a tile: the 8 * kTileZStride = 544 used, padded
// to 576 = 9 * 64 so that the components lie a multiple of 256 bytes apart
// and one LDS instruction can address two of them (the read2st64 /
// write2st64 forms).
constexpr int kTileSize = 576;
static_assert(kTileSize >= 8 * kTileZStride, "tile");
constexpr int kItem = 64;                // particles per work item (one wave)
constexpr int kMaxKeyBlocks = 1 << 26;   // 26 block bits + 6 cell bits = 32

// Error bits accumulated on the device.
enum : int32_t {
  kErrOutOfGrid = 1,
  kErrKeyOverflow = 2,
  kErrCapacity = 4,
  kErrBody = 8,
  kErrNonFinite = 16,
  kErrResize = 32,      // key space or map exceeded a resident plan's capacity
  kErrTable = 64,       // a device scene table does not match its plan
};

// ---------------------------------------------------------------------------
// Tables (device memory)
// ---------------------------------------------------------------------------
struct SceneDev {
  double origin[3];
  double h;
  double mu;
  double dt;             // drift step of the resident driver (0 in a single call)
  double accel[3];       // mechanical acceleration (Vbar = V + dt a; dt = 0 in a single call)
  double x_ref[3];       // reference point of the reported angular momentum
  int64_t offset, count;
  int32_t dims[3];
  int32_t n_iter;
  int32_t body_base;  // capacity index of this scene's body 0
  int32_t n_bodies;   // body ids must be < n_bodies
  int32_t flags;      // APIC_PIC | APIC_RULE_SEPARATE
  int32_t pad;
};

// Accumulated with atomics while cells are computed.
struct SceneAcc {
  int32_t bmin[3], bmax[3];  // cell-block box
  int32_t max_body;
  int32_t pad;
};

struct BodyAcc {
  int32_t bmin[3], bmax[3];
};

// Derived once per step from the boxes.
struct SceneLay {
  int64_t smap_off;      // offset of this scene's node-block map
  int32_t smin[3];       // node-block map origin (= cell-block box min)
  int32_t sext[3];       // node-block map extent (= box extent + 1)
};

// A body's key range numbers its blocks super block by super block (2x2x2
// blocks each, over the body's super-block box, x fastest), so that the
// blocks of one super block of one body are consecutive in key order.
struct BodyLay {
  int64_t bmap_off;      // offset of this body's node-block map
  int32_t bmin[3];       // cell-block box min
  int32_t ext[3];        // cell-block box extent (0 if empty)
  int32_t kmin[3];       // super-block box min (floor(bmin / 2))
  int32_t kext[3];       // super-block box extent (0 if empty)
  int32_t key_off;       // first key block of this body
  int32_t scene;
};

// One segment = the particles of one (body, cell block).  16-byte aligned
// (96 bytes) so that it moves in 16-byte loads and stores.
struct alignas(16) Segment {
  int32_t start, count;
  int32_t body;          // capacity body index
  int32_t scene;
  int32_t B[3];          // cell-block coordinates
  int32_t sslot[8];      // shared-grid node-block slots, j = jx + 2 jy + 4 jz
  int32_t bslot[8];      // body-grid node-block slots
};

// A work item: up to kItem particles of one segment.  The items of one
// (body, super block) run are consecutive and padded with empty items
// (count 0) to a multiple of the step's group size, so that aligned groups
// of 1, 4 or 8 items never straddle two runs.
struct Item {
  int32_t seg, start, count;
  int32_t full_y;  // 1 if one of its particles has no contact normal (set with the normals)
};

// Counters written by the device, read back by the host when it sizes
// buffers, and checked for errors after a step.
struct Counters {
  int32_t err;
  int32_t key_blocks;
  int32_t n_seg;
  int32_t n_items;
  int32_t n_sblocks;     // active shared-grid node blocks
  int32_t n_bblocks;     // active body-grid node blocks
  int32_t max_gb;        // largest capacity body index holding a particle (-1: none)
  int32_t pad1;
  int64_t smap_total;
  int64_t bmap_total;
};

// Per-scene FP64 reductions: P(3) L(3) E Pscale Lscale count uncon.
constexpr int kRed = 11;

// Partial results of one wavefront (or work item), reduced by a second kernel
// instead of many same-address atomics (those serialise at ~10 ns each).
struct RedRec {
  int32_t key;  // scene, or -1 if empty
  int32_t pad;
  double v[kRed];
};

struct BoxRec {
  int32_t key;  // capacity body index, or -1 if empty
  int32_t mn[3];
  int32_t mx[3];
  int32_t pad;
};

// Compiler memory barrier: keeps the LDS read-add-write of one stencil node
// ahead of the next node's (LDS instructions of a wave complete in order).
#define LDS_ORDER() asm volatile("" ::: "memory")

// Pin a value at this point of the instruction stream (and order memory
// around it): arithmetic producing it cannot sink below, arithmetic using it
// cannot rise above.  Keeps the unrolled stencil loops from holding all 64
// nodes' operands in registers at once.
template <typename T>
__device__ __forceinline__ void pin(T &v) {
  asm volatile("" : "+v"(v) : : "memory");
}

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tile_index(int lx, int ly, int lz) {
  return lx + kTileX * ly + kTileZStride * lz;
}

// Node n (0..63, x fastest) of node block j (0..7) in the 8x8x8 tile.
__device__ __forceinline__ int tile_index_block(int j, int n) {
  int lx = 4 * (j & 1) + (n & 3);
  int ly = 4 * ((j >> 1) & 1) + ((n >> 2) & 3);
  int lz = 4 * (j >> 2) + (n >> 4);
  return tile_index(lx, ly, lz);
}

__device__ __forceinline__ int floor_div4(int c) { return c >> 2; }  // arithmetic shift

// One DPP step on a double: lane i receives the value of the lane that
// `CTRL` selects (0 where it selects none, or in rows outside ROW_MASK).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK,
                                                            0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL,
                                                            ROW_MASK, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One halving exchange of wave_sum_spread: slots (2u, 2u+1) differ in bit b
// of their value index; each lane keeps the slot whose bit equals bit b of
// its lane (`bit`) and adds the partner lane's other slot, which holds the
// same value index for the partner's lanes.
template <int CTRL, int M>
__device__ __forceinline__ void halve_f64(const double (&in)[2 * M], double (&out)[M], bool bit) {
#pragma unroll
  for (int u = 0; u < M; ++u) {
    const double a = in[2 * u], b = in[2 * u + 1];
    const double keep = bit ? b : a, send = bit ? a : b;
    out[u] = keep + dpp_f64<CTRL, 0xf>(send);
  }
}

// Sums over the 64 lanes of K values at once, spread out: lane j (j < K,
// in every row) returns the total of value j.  Four halving exchanges within
// each row of 16 (partners lane ^ 1, lane ^ 2, and the rotations by 4 and 8,
// which pair lanes that agree in their low bits and differ in the next)
// leave lane l with value (l mod 16) summed over its row; two cross-row
// exchanges add the other rows.  About 90 instructions for K = 11, where 11
// separate six-step reductions take about 220.  Every lane of the wave must
// be active.
template <int K>
__device__ __forceinline__ double wave_sum_spread(const double (&q)[K]) {
  static_assert(K >= 1 && K <= 16, "at most 16 values");
  const int lane = threadIdx.x & 63;
  double s0[16], s1[8], s2[4], s3[2], s4[1];
#pragma unroll
  for (int t = 0; t < 16; ++t) s0[t] = t < K ? q[t] : 0.0;
  halve_f64<0xB1, 8>(s0, s1, lane & 1);         // quad_perm [1,0,3,2]: lane ^ 1
  halve_f64<0x4E, 4>(s1, s2, (lane >> 1) & 1);  // quad_perm [2,3,0,1]: lane ^ 2
  halve_f64<0x124, 2>(s2, s3, (lane >> 2) & 1); // row_ror:4
  halve_f64<0x128, 1>(s3, s4, (lane >> 3) & 1); // row_ror:8
  double v = s4[0];
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// P(3), L(3) about the scene's reference point with the affine spin, E, P
// scale, L scale, particle count, unconstrained count (filled elsewhere).
__device__ __forceinline__ void momentum_terms(const double r[3], const double v[3],
                                               const double C[9], double m, double h,
                                               double q[kRed]) {
  const double k = 0.5 * h * h;
  q[0] = m * v[0];
  q[1] = m * v[1];
  q[2] = m * v[2];
  q[3] = m * (r[1] * v[2] - r[2] * v[1] + k * (C[7] - C[5]));
  q[4] = m * (r[2] * v[0] - r[0] * v[2] + k * (C[2] - C[6]));
  q[5] = m * (r[0] * v[1] - r[1] * v[0] + k * (C[3] - C[1]));
  double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  double c2 = 0.0;
#pragma unroll
  for (int a = 0; a < 9; ++a) c2 += C[a] * C[a];
  q[6] = 0.5 * m * (v2 + k * c2);
  q[7] = m * sqrt(v2);
  q[8] = m * (sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) * sqrt(v2) + k * sqrt(c2));
  q[9] = 1.0;
  q[10] = 0.0;
}

// Records [base, base + 256) of [0, count) reduced by one 256-thread
// workgroup into out[key * kRed + c]: one set of atomics when all of them
// name one scene, per record otherwise.  Every thread of the workgroup must
// call it (it synchronises the workgroup).
__device__ __forceinline__ void reduce_rec_block(const RedRec *rec, int64_t base, int64_t count,
                                                 double *out) {
  __shared__ double part[kRed][4];
  __shared__ int32_t key0;
  const int64_t i = base + threadIdx.x;
  int key = -1;
  if (i < count) key = rec[i].key;
  if (threadIdx.x == 0) key0 = -2;
  __syncthreads();
  if (key >= 0) atomicCAS(&key0, -2, key);
  __syncthreads();
  const int k0 = key0;
  const bool uniform = __syncthreads_and(key < 0 || key == k0);
  if (k0 >= 0) {  // workgroup-uniform
    if (uniform) {
      const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
      double q[kRed];
#pragma unroll
      for (int c = 0; c < kRed; ++c) q[c] = key >= 0 ? rec[i].v[c] : 0.0;
      const double v = wave_sum_spread(q);
      if (lane < kRed) part[lane][wave] = v;
      __syncthreads();
      if (threadIdx.x < kRed)
        atomicAdd(&out[(int64_t)k0 * kRed + threadIdx.x],
                  part[threadIdx.x][0] + part[threadIdx.x][1] + part[threadIdx.x][2] +
                      part[threadIdx.x][3]);
    } else if (key >= 0) {
      for (int c = 0; c < kRed; ++c) atomicAdd(&out[(int64_t)key * kRed + c], rec[i].v[c]);
    }
  }
  __syncthreads();
}

// Binary search: the scene whose [offset, offset+count) holds particle p.
__device__ __forceinline__ int scene_of(const SceneDev *sc, int ns, int64_t p) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sc[mid].offset <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace apic

#define APIC_LAUNCH(kernel, grid, block, shmem, stream, ...)                              \
  do {                                                                                    \
    if (apic::g_launch_timer) {                                                           \
      hipEvent_t start_, stop_;                                                           \
      apic::g_launch_timer->events(&start_, &stop_);                                      \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, start_, stop_, 0,         \
                            __VA_ARGS__);                                                 \
    } else {                                                                              \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                \
    }                                                                                     \
  } while (0)
