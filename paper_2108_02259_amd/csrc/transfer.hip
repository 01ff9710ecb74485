// transfer.hip -- the grid transfers of the APIC operator H (Section 2.1.2)
// and the augury-iteration series with the Coulomb rule (Sections 2.3-2.4).
//
// Work decomposition: particles are sorted by (body, 4x4x4 cell block, cell);
// a work item is up to 64 particles of one (body, cell block) segment and is
// processed by one 64-lane wavefront.  Every node such a particle touches lies
// in an 8x8x8 node cube made of 8 node blocks, which is staged in LDS:
//  - P2G accumulates into the LDS cube (plain read-add-write, see p2g), then
//    flushes the cube to HBM with one global atomic per touched node and
//    component;
//  - G2P loads the cube's grid values with coalesced 256-byte rows and
//    gathers the 64 stencil nodes of each particle from LDS.
// The quadratic spline weights are separable, so P2G and G2P use per-axis
// partial sums (about 580 FMA each per particle instead of 1000+).
//
// One step runs: k_mass (grid mass and per-body mass), k_p2g0 (contact
// normals and Vbar to grid), then for k = 1..N the fused round k_iter (G2P
// of the previous field, the rule, P2G of the next series field), and the
// final G2P.  Grid velocities q/m are formed as the rounds load their tiles.
//
// Precision: T = float for the mixed path (weights, P2G/G2P accumulation,
// grid masses and momenta, body masses), T = double for the plain FP64 path.
// Grid velocity q/m, the normals' gradient and the friction rule use double
// in both.
#include "kernels.h"

// Occupancy targets (waves per SIMD) handed to the register allocator; the
// FP64 kernels need twice the registers for the same state.
#define APIC_ROUND_WAVES (sizeof(T) == 4 ? 5 : 2)
#define APIC_P2G_WAVES (sizeof(T) == 4 ? 5 : 3)

namespace apic {

template <typename T>
struct Stencil {
  T w[3][4];  // N per axis (Appendix B basis, 1/4 middle coefficients)
  T ht[3];    // h t per axis
  T h;
  // x_i - x_p along axis d for stencil offset a (nodes c-1..c+2)
  __device__ __forceinline__ T dx(int d, int a) const { return h * T(a - 1) - ht[d]; }
  __device__ __forceinline__ T wdx(int d, int a) const { return w[d][a] * dx(d, a); }
};

// Index of the calling wave in its workgroup, as a wave-uniform value (so
// that what is derived from it -- work items, segments, slots -- lives in
// scalar registers and is read with scalar loads).
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Lane access to a wave-uniform array through a buffer resource: the base
// address stays in scalar registers and each lane supplies only a 32-bit
// byte offset, so no per-lane 64-bit address occupies vector registers (the
// compiler otherwise keeps one such pair per array live across the item loop).
// p must be wave-uniform; offsets are below 4 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t lane_rsrc(const void *p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, -1, 0x00020000);
}
__device__ __forceinline__ float lane_ld(const float *p, uint32_t li) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(lane_rsrc(p), li * 4u, 0, 0));
}
__device__ __forceinline__ double lane_ld(const double *p, uint32_t li) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(lane_rsrc(p), li * 8u, 0, 0));
}
__device__ __forceinline__ uint32_t lane_ld(const uint32_t *p, uint32_t li) {
  return __builtin_amdgcn_raw_buffer_load_b32(lane_rsrc(p), li * 4u, 0, 0);
}
__device__ __forceinline__ void lane_st(float *p, uint32_t li, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), lane_rsrc(p), li * 4u, 0, 0);
}
__device__ __forceinline__ void lane_st(double *p, uint32_t li, double v) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(lane_rsrc(p), 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), lane_rsrc(p), li * 8u, 0, 0);
}

// Lane index formed afresh at the point of use: lane-dependent offsets
// derived from it are recomputed where needed (a few integer operations)
// instead of being hoisted out of the item loop and held in registers.
__device__ __forceinline__ int fresh_lane() {
  int l = (int)(threadIdx.x & 63);
  pin(l);
  return l;
}

// The series state Y of a particle, in two row arrays: values 0..3 (the
// velocity part and the first affine value) in Yv = Y[n][4], values 4..11 in
// YC = (Y + 4n)[n][8].  For a particle with a contact normal the Coulomb
// rule's W takes all of D's affine part, so Y's affine values are exactly
// zero.  `full` is decided per work item (the same particles in every round
// of a step; Item::full_y, set where the normals are computed, or the scene's
// Section 2.3 rule, which keeps the affine change where dv.n <= 0): an item
// none of whose particles lacks a normal reads and writes Yv only.
template <typename T>
__device__ __forceinline__ void load_y(const T *Y, int64_t n, int64_t i0, uint32_t li, bool full,
                                       T v[12]) {
  constexpr int kPer = 16 / sizeof(T);
  const __amdgpu_buffer_rsrc_t rv = lane_rsrc(Y + 4 * i0);
#pragma unroll
  for (int k = 0; k < 4 / kPer; ++k) {
    const auto q = __builtin_amdgcn_raw_buffer_load_b128(rv, li * (4 * sizeof(T)), 16 * k, 0);
    __builtin_memcpy(&v[k * kPer], &q, 16);
  }
  if (full) {
    const __amdgpu_buffer_rsrc_t rc = lane_rsrc(Y + 4 * n + 8 * i0);
#pragma unroll
    for (int k = 0; k < 8 / kPer; ++k) {
      const auto q = __builtin_amdgcn_raw_buffer_load_b128(rc, li * (8 * sizeof(T)), 16 * k, 0);
      __builtin_memcpy(&v[4 + k * kPer], &q, 16);
    }
  } else {
#pragma unroll
    for (int c = 4; c < 12; ++c) v[c] = T(0);
  }
}
template <typename T>
__device__ __forceinline__ void store_y(T *Y, int64_t n, int64_t i0, uint32_t li, bool full,
                                        const T v[12]) {
  constexpr int kPer = 16 / sizeof(T);
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b128(lane_rsrc(Y), 0, 0, 0));
  const __amdgpu_buffer_rsrc_t rv = lane_rsrc(Y + 4 * i0);
#pragma unroll
  for (int k = 0; k < 4 / kPer; ++k) {
    V q;
    __builtin_memcpy(&q, &v[k * kPer], 16);
    __builtin_amdgcn_raw_buffer_store_b128(q, rv, li * (4 * sizeof(T)), 16 * k, 0);
  }
  if (full) {
    const __amdgpu_buffer_rsrc_t rc = lane_rsrc(Y + 4 * n + 8 * i0);
#pragma unroll
    for (int k = 0; k < 8 / kPer; ++k) {
      V q;
      __builtin_memcpy(&q, &v[4 + k * kPer], 16);
      __builtin_amdgcn_raw_buffer_store_b128(q, rc, li * (8 * sizeof(T)), 16 * k, 0);
    }
  }
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Per-axis basis of Appendix B at cell-relative coordinate t in [0, 1):
// nodes c-1..c+2 carry (1-t)^2/4, (2-t^2)/4, (1+2t-t^2)/4, t^2/4.
template <typename T>
__device__ __forceinline__ void make_stencil(const T t[3], T h, Stencil<T> &S) {
  S.h = h;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T tt = t[d], u = T(1) - tt, t2 = tt * tt;
    S.w[d][0] = T(0.25) * u * u;
    S.w[d][1] = T(0.25) * (T(2) - t2);
    S.w[d][2] = T(0.25) * (T(1) + T(2) * tt - t2);
    S.w[d][3] = T(0.25) * t2;
    S.ht[d] = h * tt;
  }
}

__device__ __forceinline__ int particle_base(uint32_t key) {
  const int cx = key & 3, cy = (key >> 2) & 3, cz = (key >> 4) & 3;
  return tile_index(cx, cy, cz);
}

// G2P (eqs. gridToParticle, scaledVelGrad): vel = sum N v_i,
// B = sum N v_i (x) (x_i - x_p); returns C = B D^{-1} = (2/h^2) B.
template <typename T>
__device__ __forceinline__ void g2p(const T (*tv)[kTileSize], int base, const Stencil<T> &S,
                                    T inv_D, T vel[3], T C[9]) {
  T Bm[3][3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    vel[q] = T(0);
    Bm[q][0] = Bm[q][1] = Bm[q][2] = T(0);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    T r[3] = {0, 0, 0}, ry[3] = {0, 0, 0}, rz[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T s[3] = {0, 0, 0}, sz[3] = {0, 0, 0};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int idx = base + a + kTileX * b + kTileZStride * c;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const T v = tv[q][idx];
          s[q] += S.w[2][c] * v;
          sz[q] += S.wdx(2, c) * v;
        }
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        r[q] += S.w[1][b] * s[q];
        ry[q] += S.wdx(1, b) * s[q];
        rz[q] += S.w[1][b] * sz[q];
        pin(r[q]);  // one row of 4 nodes in flight at a time
        pin(ry[q]);
        pin(rz[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      vel[q] += S.w[0][a] * r[q];
      Bm[q][0] += S.wdx(0, a) * r[q];
      Bm[q][1] += S.w[0][a] * ry[q];
      Bm[q][2] += S.w[0][a] * rz[q];
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int b = 0; b < 3; ++b) C[3 * q + b] = Bm[q][b] * inv_D;
}

// P2G of a generalized velocity (u, E) with E = B D^{-1} (eq. particleToGrid):
// adds N m (u + E (x_i - x_p)) to each of the 64 stencil nodes of the tile.
//
// LDS accumulation is a plain read-add-write per node (float LDS atomics are
// an order of magnitude slower on this part).  It is race-free because (1)
// the lanes taking part in one pass hold particles of distinct cells, so in
// any one instruction their 64 addresses are distinct, and (2) LDS_ORDER keeps
// each node's read-add-write ahead of the next node's, and LDS instructions
// of a wave complete in order.
template <typename T>
__device__ __forceinline__ void p2g(T (*tq)[kTileSize], int base, const Stencil<T> &S, T m,
                                    const T u[3], const T E[9]) {
  // Pinned at entry: what is derived from the inputs is formed here, row by
  // row, not hoisted out of the caller's pass loop (which would keep every
  // row's operands live at once).
  T mu[3], mE[3][3];
  pin(m);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    mu[q] = m * u[q];
#pragma unroll
    for (int b = 0; b < 3; ++b) mE[q][b] = m * E[3 * q + b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    T A[3], Ay[3], Az[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      A[q] = S.w[0][a] * (mu[q] + mE[q][0] * S.dx(0, a));
      Ay[q] = S.w[0][a] * mE[q][1];
      Az[q] = S.w[0][a] * mE[q][2];
      pin(A[q]);
      pin(Ay[q]);
      pin(Az[q]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T P[3], Q[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        P[q] = S.w[1][b] * (A[q] + Ay[q] * S.dx(1, b));
        Q[q] = S.w[1][b] * Az[q];
        pin(P[q]);  // this row's operands are formed here, not hoisted
        pin(Q[q]);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int idx = base + a + kTileX * b + kTileZStride * c;
#pragma unroll
        for (int q = 0; q < 3; ++q)
          tq[q][idx] = fma_t(S.w[2][c], P[q], fma_t(S.wdx(2, c), Q[q], tq[q][idx]));
        LDS_ORDER();
      }
    }
  }
}

// Mass P2G (eq. massToGrid): N m to the mass tile, with the same
// race-freedom argument as p2g.
template <typename T>
__device__ __forceinline__ void p2g_mass(T *tm, int base, const Stencil<T> &S, T m) {
  pin(m);  // as in p2g
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T wab = S.w[0][a] * S.w[1][b] * m;
      pin(wab);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int idx = base + a + kTileX * b + kTileZStride * c;
        tm[idx] += wab * S.w[2][c];
        LDS_ORDER();
      }
    }
}

// Pass structure of one work item: lanes are ranked among the lanes holding a
// particle of the same cell (6-bit cell-in-block key), and pass r scatters the
// lanes of rank r.  With one particle per cell this is a single pass.
__device__ __forceinline__ int cell_rank(bool active, uint32_t cell6, int *passes) {
  const uint64_t act = __ballot(active);
  uint64_t peers = act;
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    const uint64_t bb = __ballot((cell6 >> b) & 1u);
    peers &= ((cell6 >> b) & 1u) ? bb : ~bb;
  }
  // set bits of peers below this lane (mbcnt: no lane mask kept in registers)
  const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
  int rank = active ? below : 0;
  // one particle per cell (the common case): a single pass, no reduction
  if (__ballot(rank > 0) == 0) {
    *passes = act ? 1 : 0;
    return rank;
  }
  int mx = rank;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
  *passes = mx + 1;
  return rank;
}

// The value the next lane holds (lane + 1; zero for lane 63), moved by a DPP
// wavefront shift, which exchanges registers between lanes without the LDS.
// What a lane outside the current execution mask holds is not defined: the
// callers select such values away.
__device__ __forceinline__ float from_next_lane(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_next_lane(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x130, 0xf,
                                                            0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0x130,
                                                            0xf, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Paired scatter of crowded work items.  Where cells hold several particles,
// pass r of cell_rank costs a whole read-add-write of the stencil for the few
// lanes of rank r.  The layout orders particles by cell within each block run
// of a 64-particle gather wave, so the lanes holding one cell are mostly
// consecutive (a block that straddles two gather waves gives its items two
// ordered runs, and a cell may then appear in both).  Here each run of
// consecutive lanes holding one cell is cut into pairs (its lanes 0-1, 2-3,
// ...): the first lane of a pair, a unit, scatters the sum of both particles'
// terms, which it receives from the second by lane exchange; an odd run's last
// lane is a unit of its own.  Units of one cell, from any run, are ranked as
// lanes are in cell_rank, and pass r scatters the units of rank r (with their
// partners taking part in forming the terms), so one pass writes each node at
// most once per instruction, as before.  `rank` is the pass a lane takes part
// in (-1: none).
struct Pairing {
  int rank;
  bool unit;     // writes the tile in its pass
  bool partner;  // the next lane's particle is this unit's pair
};

__device__ __forceinline__ Pairing pair_lanes(bool active, uint32_t cell6, int *passes) {
  const int lane = (int)(threadIdx.x & 63);
  // active lanes are a prefix of the wave, so an active lane's predecessor is active
  const int prev = __shfl_up((int)cell6, 1, 64);
  const uint64_t same = __ballot(active && lane > 0 && prev == (int)cell6);
  Pairing p;
  if (same == 0) {  // no two consecutive lanes share a cell: every lane is a unit
    p.unit = active;
    p.partner = false;
    p.rank = cell_rank(active, cell6, passes);
    if (!active) p.rank = -1;
    return p;
  }
  // position in the run of equal cells: distance to the run's first lane
  const uint64_t heads = __ballot(active && !((same >> lane) & 1ull));
  const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1);  // lanes <= this one
  const uint64_t hb = heads & le;
  const int start = hb ? 63 - __clzll((unsigned long long)hb) : lane;
  p.unit = active && ((lane - start) & 1) == 0;
  p.partner = p.unit && lane < 63 && ((same >> (lane + 1)) & 1ull) != 0;
  const int urank = cell_rank(p.unit, cell6, passes);
  const int pair_rank = __shfl_up(urank, 1, 64);  // a second lane joins its unit's pass
  p.rank = p.unit ? urank : (active ? pair_rank : -1);
  return p;
}

// p2g for the lanes of one pass of the paired scatter (see pair_lanes): every
// taking part lane forms its particle's row terms; a unit adds its partner's
// (moved from the next lane, zero without a partner) to its own and writes the
// sum.  The partner's z weights come along once.
template <typename T>
__device__ __forceinline__ void p2g_pair(T (*tq)[kTileSize], int base, const Stencil<T> &S, T m,
                                         const T u[3], const T E[9], bool unit, bool partner) {
  T wn[4], wdn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const T a = from_next_lane(S.w[2][c]), b = from_next_lane(S.wdx(2, c));
    wn[c] = partner ? a : T(0);
    wdn[c] = partner ? b : T(0);
  }
  T mu[3], mE[3][3];
  pin(m);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    mu[q] = m * u[q];
#pragma unroll
    for (int b = 0; b < 3; ++b) mE[q][b] = m * E[3 * q + b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    T A[3], Ay[3], Az[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      A[q] = S.w[0][a] * (mu[q] + mE[q][0] * S.dx(0, a));
      Ay[q] = S.w[0][a] * mE[q][1];
      Az[q] = S.w[0][a] * mE[q][2];
      pin(A[q]);
      pin(Ay[q]);
      pin(Az[q]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T P[3], Q[3], Pn[3], Qn[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        P[q] = S.w[1][b] * (A[q] + Ay[q] * S.dx(1, b));
        Q[q] = S.w[1][b] * Az[q];
        pin(P[q]);
        pin(Q[q]);
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const T pn = from_next_lane(P[q]), qn = from_next_lane(Q[q]);
        Pn[q] = partner ? pn : T(0);
        Qn[q] = partner ? qn : T(0);
        pin(Pn[q]);
        pin(Qn[q]);
      }
      if (unit) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int idx = base + a + kTileX * b + kTileZStride * c;
#pragma unroll
          for (int q = 0; q < 3; ++q)
            tq[q][idx] = fma_t(S.w[2][c], P[q],
                               fma_t(S.wdx(2, c), Q[q],
                                     fma_t(wn[c], Pn[q], fma_t(wdn[c], Qn[q], tq[q][idx]))));
          LDS_ORDER();
        }
      }
    }
  }
}

// The scatter passes of a work item: with PAIRS the paired scatter, else one
// pass per cell rank with every lane a unit of its own.
template <bool PAIRS>
__device__ __forceinline__ Pairing scatter_lanes(bool active, uint32_t cell6, int *passes) {
  if constexpr (PAIRS) {
    return pair_lanes(active, cell6, passes);
  } else {
    Pairing p;
    p.unit = active;
    p.partner = false;
    p.rank = cell_rank(active, cell6, passes);
    return p;
  }
}

// One item's scatter passes.  With PAIRS: plain p2g where a pass has no pairs
// (every pass of an item with one particle per cell), p2g_pair otherwise.
template <typename T, bool PAIRS>
__device__ __forceinline__ void p2g_passes(T (*tq)[kTileSize], int base, const Stencil<T> &S,
                                           T m, const T u[3], const T E[9], const Pairing &pl,
                                           int passes) {
  for (int pass = 0; pass < passes; ++pass) {
    const bool unit = pl.unit && pl.rank == pass;
    if constexpr (PAIRS) {
      if (__ballot(unit && pl.partner) != 0) {
        if (pl.rank == pass) p2g_pair(tq, base, S, m, u, E, unit, pl.partner);
      } else if (unit) {
        p2g(tq, base, S, m, u, E);
      }
    } else {
      if (unit) p2g(tq, base, S, m, u, E);
    }
    LDS_ORDER();
  }
}

// Mass P2G for one pass of the paired scatter (as p2g_pair).
template <typename T>
__device__ __forceinline__ void p2g_mass_pair(T *tm, int base, const Stencil<T> &S, T m,
                                              bool unit, bool partner) {
  T wn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const T a = from_next_lane(S.w[2][c]);
    wn[c] = partner ? a : T(0);
  }
  pin(m);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T wab = S.w[0][a] * S.w[1][b] * m;
      pin(wab);
      const T nb = from_next_lane(wab);
      T wabn = partner ? nb : T(0);
      pin(wabn);
      if (unit) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int idx = base + a + kTileX * b + kTileZStride * c;
          tm[idx] = fma_t(wab, S.w[2][c], fma_t(wabn, wn[c], tm[idx]));
          LDS_ORDER();
        }
      }
    }
}

template <typename T, bool PAIRS>
__device__ __forceinline__ void p2g_mass_passes(T *tm, int base, const Stencil<T> &S, T m,
                                                const Pairing &pl, int passes) {
  for (int pass = 0; pass < passes; ++pass) {
    const bool unit = pl.unit && pl.rank == pass;
    if constexpr (PAIRS) {
      if (__ballot(unit && pl.partner) != 0) {
        if (pl.rank == pass) p2g_mass_pair(tm, base, S, m, unit, pl.partner);
      } else if (unit) {
        p2g_mass(tm, base, S, m);
      }
    } else {
      if (unit) p2g_mass(tm, base, S, m);
    }
    LDS_ORDER();
  }
}


// Outward normal from the particle's own-body grid mass: n = -grad m^b / |.|;
// zero when the gradient vanishes (the particle is then unconstrained).
template <typename U>
__device__ __forceinline__ void body_normal(const U *tb, int base, const double t[3], double h,
                                            double n[3]) {
  double w[3][4], g[3][4];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double tt = t[d], u = 1.0 - tt, t2 = tt * tt;
    w[d][0] = 0.25 * u * u;
    w[d][1] = 0.25 * (2.0 - t2);
    w[d][2] = 0.25 * (1.0 + 2.0 * tt - t2);
    w[d][3] = 0.25 * t2;
    g[d][0] = -0.5 * u / h;
    g[d][1] = -0.5 * tt / h;
    g[d][2] = 0.5 * u / h;
    g[d][3] = 0.5 * tt / h;
  }
  double gx = 0, gy = 0, gz = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double r = 0, ry = 0, rz = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double s = 0, sz = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double mi = (double)tb[base + a + kTileX * b + kTileZStride * c];
        s += w[2][c] * mi;
        sz += g[2][c] * mi;
      }
      r += w[1][b] * s;
      ry += g[1][b] * s;
      rz += w[1][b] * sz;
      pin(r);
      pin(ry);
      pin(rz);
    }
    gx += g[0][a] * r;
    gy += w[0][a] * ry;
    gz += w[0][a] * rz;
  }
  const double len = sqrt(gx * gx + gy * gy + gz * gz);
  if (len > 0.0) {
    n[0] = -gx / len;
    n[1] = -gy / len;
    n[2] = -gz / len;
  } else {
    n[0] = n[1] = n[2] = 0.0;
  }
}

// Section 2.4: undesirable part of the velocity change d at normal n.
__device__ __forceinline__ void undesirable(const double d[3], const double n[3], double mu,
                                            double w[3]) {
  const double dn = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
  if (dn > 0.0) {
    w[0] = d[0];
    w[1] = d[1];
    w[2] = d[2];
    return;
  }
  double dt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) dt[a] = d[a] - dn * n[a];
  const double tau = sqrt(dt[0] * dt[0] + dt[1] * dt[1] + dt[2] * dt[2]);
  const double s = fmin(tau, -mu * dn);
  // w = d_t (1 - s / |d_t|): one division per particle; exactly 0 when the
  // change lies in the cone (s = |d_t|)
  const double f = tau > 0.0 ? (tau - s) / tau : 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) w[a] = f * dt[a];
}

// Tile of NC components from a [slot][comps_in_buf][64] buffer: slots
// first, then every block's loads together (absent blocks read block 0 and
// are masked).
template <typename T, int NC>
__device__ __forceinline__ void load_tile(T (*tile)[kTileSize], const T *buf, const int32_t *slot,
                                          int comps_in_buf) {
  const uint32_t lane = (uint32_t)fresh_lane();
  int s[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) s[j] = __builtin_amdgcn_readfirstlane(slot[j]);
  T v[8][NC];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t sj = s[j] >= 0 ? s[j] : 0;
#pragma unroll
    for (int q = 0; q < NC; ++q)
      v[j][q] = lane_ld(buf + (sj * comps_in_buf + q) * kNodesPerBlock, lane);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int li = tile_index_block(j, lane);
#pragma unroll
    for (int q = 0; q < NC; ++q) tile[q][li] = s[j] >= 0 ? v[j][q] : T(0);
  }
}

// The 8x8x8 node velocities of a tile from grid momenta: v = q / m, formed as
// q * (1/m) in FP64 (0 where the mass is 0), then stored in T.  All eight
// slots are read first and then every block's loads are issued together
// (absent blocks read block 0 and are masked), so the tile costs two memory
// round trips rather than two per block.
template <typename T>
__device__ __forceinline__ void load_vel_tile(T (*tile)[kTileSize], const T *q, const double *invm,
                                              const int32_t *slot) {
  const uint32_t lane = (uint32_t)fresh_lane();
  int s[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) s[j] = __builtin_amdgcn_readfirstlane(slot[j]);
  T v[8][3];
  double inv[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t sj = s[j] >= 0 ? s[j] : 0;
    inv[j] = lane_ld(invm + sj * kNodesPerBlock, lane);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[j][c] = lane_ld(q + (sj * 3 + c) * kNodesPerBlock, lane);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int li = tile_index_block(j, lane);
#pragma unroll
    for (int c = 0; c < 3; ++c) tile[c][li] = s[j] >= 0 ? (T)((double)v[j][c] * inv[j]) : T(0);
  }
}

template <typename T, int NC, bool ZERO = true>
__device__ __forceinline__ void flush_tile(T (*tile)[kTileSize], T *buf, const int32_t *slot,
                                           int comps_in_buf) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int s = slot[j];
    const int li = tile_index_block(j, lane);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const T v = tile[q][li];
      if (ZERO) tile[q][li] = T(0);
      if (v != T(0) && s >= 0)
        unsafeAtomicAdd(&buf[((int64_t)s * comps_in_buf + q) * kNodesPerBlock + lane], v);
    }
  }
}

template <typename T, int NC>
__device__ __forceinline__ void zero_tile(T (*tile)[kTileSize]) {
  const int lane = fresh_lane();
  for (int i = lane; i < kTileSize; i += 64)
#pragma unroll
    for (int q = 0; q < NC; ++q) tile[q][i] = T(0);
}

// Ordering within one wavefront: each wave's LDS tile is written and read
// only by that wave, and a wave's LDS instructions complete in issue order,
// so a compiler ordering point suffices between a wave's own phases (it does
// not wait for the flush atomics).  It orders nothing across waves: every
// exchange between the waves of a workgroup (the grouped flushes and their
// tables) goes through group_barrier.
__device__ __forceinline__ void wave_sync() { LDS_ORDER(); }

// Workgroup barrier for LDS data only: the fences are restricted to LDS, so
// the waves do not wait here for their global atomics (nothing the
// workgroup reads later depends on them within the kernel).
__device__ __forceinline__ void group_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int item_count(const StepArgs &a) {
  return a.cnt->err ? 0 : a.cnt->n_items;
}

// Work-item schedule of the particle kernels.  Workgroups are dispatched to
// the eight XCDs in turn (workgroup b runs on XCD b mod 8), each XCD with its
// own L2.  With xcd_split the item list (sorted, so neighbouring items share
// node blocks) is cut into eight contiguous ranges and the workgroups of XCD x
// walk range x, which keeps a node block's tile loads and flush atomics in one
// L2; otherwise every workgroup strides over the whole list.
struct ItemLoop {
  int w, end, step;
};

// Units of `unit` consecutive items (a multiple of the run padding
// divides every run, so a unit never straddles two runs).
__device__ __forceinline__ ItemLoop item_loop(const StepArgs &a, int unit = 1) {
  const int nitems = item_count(a) / unit;
  ItemLoop L;
  if (a.xcd_split) {  // the host keeps gridDim.x a multiple of 8 in this mode
    const int per = gridDim.x >> 3;
    const int chunk = (nitems + 7) >> 3;
    const int lo = (blockIdx.x & 7) * chunk;
    L.w = lo + (blockIdx.x >> 3);
    L.end = min(nitems, lo + chunk);
    L.step = per;
  } else {
    L.w = blockIdx.x;
    L.end = nitems;
    L.step = gridDim.x;
  }
  return L;
}

// ---------------------------------------------------------------------------
// Work-item groups
// ---------------------------------------------------------------------------
// The items of one (body, super block) run are consecutive -- the cell key
// numbers a body's blocks super block by super block -- and padded with
// empty items to a multiple of 8.  A group is the G aligned items g*G ..
// g*G + G - 1, all of one run; empty items have no particles.  The G waves
// of a workgroup take one item each and scatter into their own
// LDS tiles; the workgroup then merges the tiles node by node over the 3x3x3
// node blocks of the super block, so a node leaves the workgroup in one
// global atomic instead of one per item.  With G = 1 each wave flushes its
// own tile.
template <int G>
struct GroupLds {
  int32_t slot[27];   // shared-grid slot of super node block J (-1: none)
  int32_t bslot[27];  // body-grid slot of J (mass kernel; the group is one body)
  uint32_t mask[27];  // waves whose tile covers J
  int32_t sbi[G];     // wave's block within the super block, x + 2y + 4z
  int32_t seg[G];     // wave's segment, -1 if it has nothing to flush
};

__device__ __forceinline__ int block_in_super(const Segment &sg) {
  return (sg.B[0] & 1) | ((sg.B[1] & 1) << 1) | ((sg.B[2] & 1) << 2);
}

// Cover masks and slots of the 27 node blocks (after every wave has filled
// its sbi/seg entry and a barrier).
template <int G, bool BODY = false>
__device__ __forceinline__ void group_tables(const StepArgs &a, GroupLds<G> &gl) {
  const int t = threadIdx.x;
  if (t < 27) {
    const int Jx = t % 3, Jy = (t / 3) % 3, Jz = t / 9;
    uint32_t mask = 0;
    int32_t slot = -1, bslot = -1;
    for (int w = 0; w < G; ++w) {
      const int sgi = gl.seg[w];
      if (sgi < 0) continue;
      const int sb = gl.sbi[w];
      const int jx = Jx - (sb & 1), jy = Jy - ((sb >> 1) & 1), jz = Jz - (sb >> 2);
      if (jx < 0 || jx > 1 || jy < 0 || jy > 1 || jz < 0 || jz > 1) continue;
      mask |= 1u << w;
      slot = a.seg[sgi].sslot[jx + 2 * jy + 4 * jz];
      if (BODY) bslot = a.seg[sgi].bslot[jx + 2 * jy + 4 * jz];
    }
    gl.mask[t] = mask;
    gl.slot[t] = slot;
    if (BODY) gl.bslot[t] = bslot;
  }
}

// Sum the covering waves' tiles per node (wave order) and add each nonzero
// sum once to the global buffer; with ZERO the tiles read are left zero.  Wave v of
// the workgroup takes node blocks J = v, v + G, ..., one node per lane, so
// everything about J is wave-uniform.
template <typename T, int G, int NC, bool ZERO = true>
__device__ __forceinline__ void group_flush(T (*tiles)[NC][kTileSize], const GroupLds<G> &gl,
                                            T *buf, int comps_in_buf) {
  const int lane = fresh_lane();
  const int loff = tile_index_block(0, lane);
  for (int J = wave_id(); J < 27; J += G) {
    const uint32_t mask = __builtin_amdgcn_readfirstlane(gl.mask[J]);
    if (!mask) continue;
    const int Jx = J % 3, Jy = (J / 3) % 3, Jz = J / 9;
    T sum[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) sum[q] = T(0);
#pragma unroll
    for (int w = 0; w < G; ++w) {
      if (!((mask >> w) & 1u)) continue;
      const int sb = __builtin_amdgcn_readfirstlane(gl.sbi[w]);
      const int j = (Jx - (sb & 1)) + 2 * (Jy - ((sb >> 1) & 1)) + 4 * (Jz - (sb >> 2));
      const int li = tile_index_block(j, 0) + loff;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        sum[q] += tiles[w][q][li];
        if (ZERO) tiles[w][q][li] = T(0);
      }
    }
    const int s = __builtin_amdgcn_readfirstlane(gl.slot[J]);
    if (s < 0) continue;
    T *dst = buf + (int64_t)s * comps_in_buf * kNodesPerBlock;
#pragma unroll
    for (int q = 0; q < NC; ++q)
      if (sum[q] != T(0)) unsafeAtomicAdd(&dst[q * kNodesPerBlock + lane], sum[q]);
  }
}

// Flush of a group's shared-grid tiles: each wave's own tile when G = 1,
// else the merged tiles (all threads of the workgroup take part).
// ZERO: leave the tiles read zero (for kernels that accumulate the next item
// into them); the rounds reload every tile entry G2P reads, so they skip it.
template <typename T, int G, int NC, bool ZERO = true>
__device__ __forceinline__ void flush_group(const StepArgs &a, T (*tiles)[NC][kTileSize],
                                            GroupLds<G> &gl, bool flushes, int seg_index,
                                            T *buf, int comps_in_buf) {
  if (G == 1) {
    wave_sync();
    if (flushes) flush_tile<T, NC, ZERO>(tiles[0], buf, a.seg[seg_index].sslot, comps_in_buf);
    wave_sync();
  } else {
    const int wave = wave_id();
    const int sgi = flushes ? seg_index : -1;  // wave-uniform
    const int sbi = flushes ? block_in_super(a.seg[seg_index]) : 0;
    if ((threadIdx.x & 63) == 0) {
      int wv = wave;
      pin(wv);  // its LDS address formed here, not held across the item loop
      gl.seg[wv] = sgi;
      gl.sbi[wv] = sbi;
    }
    group_barrier();
    group_tables<G>(a, gl);
    group_barrier();
    group_flush<T, G, NC, ZERO>(tiles, gl, buf, comps_in_buf);
    group_barrier();
  }
}

// Flush of a group's mass tiles into both the shared grid mass (by sslot)
// and the body grid mass (by bslot).  An item's contribution to its body's
// grid equals its contribution to the shared grid, and a group is one body,
// so one tile per wave and one sum per node serve both.  The tiles read are
// left zero.
template <typename T, int G>
__device__ __forceinline__ void flush_group_mass(const StepArgs &a, T (*tiles)[1][kTileSize],
                                                 GroupLds<G> &gl, bool flushes, int seg_index,
                                                 T *mass, T *bmass) {
  const int lane = threadIdx.x & 63;
  if (G == 1) {
    wave_sync();
    if (flushes) {
      const Segment &sg = a.seg[seg_index];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int s = __builtin_amdgcn_readfirstlane(sg.sslot[j]);
        const int b = __builtin_amdgcn_readfirstlane(sg.bslot[j]);
        const int li = tile_index_block(j, lane);
        const T v = tiles[0][0][li];
        tiles[0][0][li] = T(0);
        if (v != T(0)) {
          if (s >= 0) unsafeAtomicAdd(&mass[(int64_t)s * kNodesPerBlock + lane], v);
          if (b >= 0) unsafeAtomicAdd(&bmass[(int64_t)b * kNodesPerBlock + lane], v);
        }
      }
    }
    wave_sync();
    return;
  }
  const int wave = wave_id();
  const int sgi = flushes ? seg_index : -1;
  const int sbi = flushes ? block_in_super(a.seg[seg_index]) : 0;
  if (lane == 0) {
    gl.seg[wave] = sgi;
    gl.sbi[wave] = sbi;
  }
  group_barrier();
  group_tables<G, true>(a, gl);
  group_barrier();
  const int loff = tile_index_block(0, lane);
  for (int J = wave; J < 27; J += G) {
    const uint32_t mask = __builtin_amdgcn_readfirstlane(gl.mask[J]);
    if (!mask) continue;
    const int Jx = J % 3, Jy = (J / 3) % 3, Jz = J / 9;
    T sum = T(0);
#pragma unroll
    for (int w = 0; w < G; ++w) {
      if (!((mask >> w) & 1u)) continue;
      const int sb = __builtin_amdgcn_readfirstlane(gl.sbi[w]);
      const int j = (Jx - (sb & 1)) + 2 * (Jy - ((sb >> 1) & 1)) + 4 * (Jz - (sb >> 2));
      const int li = tile_index_block(j, 0) + loff;
      sum += tiles[w][0][li];
      tiles[w][0][li] = T(0);
    }
    if (sum == T(0)) continue;
    const int s = __builtin_amdgcn_readfirstlane(gl.slot[J]);
    const int b = __builtin_amdgcn_readfirstlane(gl.bslot[J]);
    if (s >= 0) unsafeAtomicAdd(&mass[(int64_t)s * kNodesPerBlock + lane], sum);
    if (b >= 0) unsafeAtomicAdd(&bmass[(int64_t)b * kNodesPerBlock + lane], sum);
  }
  group_barrier();
}

// ---------------------------------------------------------------------------
// grid mass and per-body mass
// ---------------------------------------------------------------------------
template <typename T, int G, bool PAIRS>
__global__ __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu(APIC_P2G_WAVES)))
void k_mass(StepArgs a, const T *t, const T *m, GridPtrs g) {
  __shared__ T tm[G][1][kTileSize];  // one item's mass (shared grid and its body's grid)
  __shared__ GroupLds<G> gl;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  zero_tile<T, 1>(tm[wave]);
  wave_sync();
  const int64_t n = a.n;
  for (ItemLoop L = item_loop(a, G); L.w < L.end; L.w += L.step) {
    const int w0 = L.w * G;
    if (a.items[w0].count == 0) continue;  // padding only (uniform over the workgroup)
    const Item mine = a.items[w0 + wave];
    const bool member = mine.count > 0;
    const Item it = member ? mine : a.items[w0];
    const Segment &sg = a.seg[it.seg];
    const bool active = member && lane < it.count;
    const uint32_t li = active ? lane : 0u;
    const int64_t i0 = it.start;
    const uint32_t key = lane_ld(a.keys + i0, li);
    int passes;
    const Pairing pl = scatter_lanes<PAIRS>(active, key & 63u, &passes);
    if (active) {
      T tt[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) tt[c] = lane_ld(t + c * n + i0, li);
      Stencil<T> S;
      make_stencil(tt, (T)a.sc[sg.scene].h, S);
      const T mp = lane_ld(m + i0, li);
      const int base = particle_base(key);
      p2g_mass_passes<T, PAIRS>(&tm[wave][0][0], base, S, mp, pl, passes);
    }
    flush_group_mass<T, G>(a, tm, gl, member, it.seg, (T *)g.mass, (T *)g.bmass);
  }
}

// ---------------------------------------------------------------------------
// Contact normals (from the per-body mass grid) and P2G of Vbar into buffer 0
// ---------------------------------------------------------------------------
// Both need the complete mass grids and nothing else of each other, so one
// pass over the items does both: a wave first stages its item's body-mass
// tile (FP64) in the space of its P2G tile, computes the normals of its
// particles, clears that space and then scatters Vbar.  Normals are skipped
// for scenes without series rounds (unused there).
template <typename T, int G, bool PAIRS>
__global__ __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu(APIC_P2G_WAVES)))
void k_p2g0(StepArgs a, const T *t, const T *m, const T *vbar, T *nrm, Item *items, GridPtrs g) {
  __shared__ T tq[G][3][kTileSize];
  __shared__ GroupLds<G> gl;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  zero_tile<T, 3>(tq[wave]);
  wave_sync();
  const int64_t n = a.n;
  for (ItemLoop L = item_loop(a, G); L.w < L.end; L.w += L.step) {
    const int w0 = L.w * G;
    if (a.items[w0].count == 0) continue;  // padding only (uniform over the workgroup)
    const Item mine = a.items[w0 + wave];
    const bool member = mine.count > 0;
    const Item it = member ? mine : a.items[w0];
    const Segment &sg = a.seg[it.seg];
    const bool active = member && lane < it.count;
    const uint32_t li = active ? lane : 0u;
    const int64_t i0 = it.start;
    const uint32_t key = lane_ld(a.keys + i0, li);
    const int base = particle_base(key);
    const SceneDev &sd = a.sc[sg.scene];
    T tt[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) tt[c] = lane_ld(t + c * n + i0, li);
    if (member && sd.n_iter > 0 && a.given_normals) {  // wave-uniform
      // the caller's normals, already in sorted order
      bool no_nrm = false;
      if (active)
        no_nrm = lane_ld(nrm + i0, li) == T(0) && lane_ld(nrm + n + i0, li) == T(0) &&
                 lane_ld(nrm + 2 * n + i0, li) == T(0);
      const uint64_t any = __ballot(no_nrm);
      if (lane == 0) items[w0 + wave].full_y = any != 0 ? 1 : 0;
    } else if (member && sd.n_iter > 0) {  // wave-uniform
      // the body-mass tile in the first component of this wave's P2G tile
      load_tile<T, 1>(tq[wave], (const T *)g.bmass, sg.bslot, 1);
      wave_sync();
      bool no_nrm = false;
      if (active) {
        const double td[3] = {(double)tt[0], (double)tt[1], (double)tt[2]};
        double nd[3];
        body_normal(&tq[wave][0][0], base, td, sd.h, nd);
        T nt[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          nt[c] = (T)nd[c];
          lane_st(nrm + c * n + i0, li, nt[c]);
        }
        no_nrm = nt[0] == T(0) && nt[1] == T(0) && nt[2] == T(0);
      }
      // the item's flag for the rounds: full Y rows if a particle has no normal
      const uint64_t any = __ballot(no_nrm);
      if (lane == 0) items[w0 + wave].full_y = any != 0 ? 1 : 0;
      wave_sync();
      zero_tile<T, 1>(tq[wave]);
      wave_sync();
    }
    int passes;
    const Pairing pl = scatter_lanes<PAIRS>(active, key & 63u, &passes);
    if (active) {
      Stencil<T> S;
      make_stencil(tt, (T)sd.h, S);
      T u[3], E[9];
#pragma unroll
      for (int q = 0; q < 3; ++q) u[q] = lane_ld(vbar + q * n + i0, li);
      // PIC (Section 2.1.1): the momentum sum has no affine term
      const bool pic = (sd.flags & APIC_PIC) != 0;
#pragma unroll
      for (int q = 0; q < 9; ++q) E[q] = pic ? T(0) : lane_ld(vbar + (3 + q) * n + i0, li);
      const T mp = lane_ld(m + i0, li);
      p2g_passes<T, PAIRS>(tq[wave], base, S, mp, u, E, pl, passes);
    }
    flush_group<T, G, 3>(a, tq, gl, member, it.seg, (T *)g.buf[0], 3);
  }
  // side job for the rounds (the mass grid is complete since the mass kernel):
  // 1 / m per active node in FP64, 0 where m = 0
  const T *mass = (const T *)g.mass;
  const int64_t nodes = (int64_t)a.cnt->n_sblocks * kNodesPerBlock;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nodes;
       q += (int64_t)gridDim.x * blockDim.x) {
    const double mi = (double)mass[q];
    g.invm[q] = mi > 0.0 ? 1.0 / mi : 0.0;
  }
}

// ---------------------------------------------------------------------------
// One round k of the series (fused G2P + rule + P2G)
// ---------------------------------------------------------------------------
// Stored per particle between rounds: Y = D_{k-1} - W_k, so that after the
// next G2P (of W_k) the accumulated change is D_k = Y + H W_k, and the final
// answer is Vhat = Vbar + D_N.  Round 1 starts from D_0 = H Vbar - Vbar.
// Y is laid out by particle in two row arrays (see load_y).
// Scenes with n_iter == k-1 finish in round k: they write Vhat and scatter
// nothing.  Round max n_iter + 1 only finishes (k_final).
// VAR: scenes may carry flags (PIC transfers, the Section 2.3 rule); without
// it the flags are ignored and none of their code is compiled in (the batch
// has none), which keeps the common kernel's register budget.
template <typename T, bool FIRST, int G, bool VAR, bool PAIRS>
__global__ __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu(APIC_ROUND_WAVES)))
void k_iter(StepArgs a, int k, const T *t, const T *m, const T *vbar, const T *nrm, T *Y,
            GridPtrs g, const uint32_t *perm, T *v_out, T *C_out) {
  // One tile per wave: the gathered grid velocities, then (cleared) the
  // scatter target.
  __shared__ T tile[G][3][kTileSize];
  __shared__ GroupLds<G> gl;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int64_t n = a.n;
  const T *gcur = (const T *)g.buf[(k - 1) % 3];
  T *gnext = (T *)g.buf[k % 3];
  {  // the buffer round k+1 scatters into (last read by round k-1)
    T *gclear = (T *)g.buf[(k + 1) % 3];
    const int64_t words = (int64_t)a.cnt->n_sblocks * 3 * kNodesPerBlock;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < words;
         q += (int64_t)gridDim.x * blockDim.x)
      gclear[q] = T(0);
  }
  for (ItemLoop L = item_loop(a, G); L.w < L.end; L.w += L.step) {
    const int w0 = L.w * G;
    if (a.items[w0].count == 0) continue;  // padding only (uniform over the workgroup)
    const Item mine = a.items[w0 + wave];
    const bool member = mine.count > 0;
    const Item it = member ? mine : a.items[w0];
    const Segment &sg = a.seg[it.seg];
    const SceneDev &sd = a.sc[sg.scene];
    if (sd.n_iter < k - 1) continue;  // scene already finished (uniform per group)
    const bool finishing = sd.n_iter == k - 1;
    if (member) load_vel_tile<T>(tile[wave], gcur, g.invm, sg.sslot);
    wave_sync();
    const bool active = member && lane < it.count;
    // per-particle arrays: wave-uniform base it.start (+ c n), lane offset li
    const uint32_t li = active ? lane : 0u;
    const int64_t i0 = it.start;
    const uint32_t key = lane_ld(a.keys + i0, li);
    const int base = particle_base(key);
    const T h = (T)sd.h;
    Stencil<T> S;
    T W[12];
    if (active) {
      T tt[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) tt[c] = lane_ld(t + c * n + i0, li);
      make_stencil(tt, h, S);
      T hv[3], hC[9];
      g2p(tile[wave], base, S, T(2) / (h * h), hv, hC);
      const T *vbi = vbar + i0;
      // full series rows: some particle of the item has no normal, or the
      // Section 2.3 rule may leave a constrained particle's affine change in Y
      const int flags = VAR ? sd.flags : 0;  // wave-uniform
      const bool full = it.full_y != 0 || (flags & APIC_RULE_SEPARATE) != 0;
      // PIC: C is not part of the transferred state; H passes the affine
      // part through (H Vbar keeps Vbar's C, H W keeps W's zero C), so the
      // series never moves it.  keepC = 0 zeroes G's affine part.
      const bool pic = (flags & APIC_PIC) != 0;
      const T keepC = pic ? T(0) : T(1);  // applied where hC is used
      if (finishing) {
        const int64_t dst = perm ? (int64_t)lane_ld(perm + i0, li) : i0 + li;
        if (FIRST) {  // N = 0: Vhat = H Vbar exactly as gathered
#pragma unroll
          for (int c = 0; c < 3; ++c) v_out[c * n + dst] = hv[c];
#pragma unroll
          for (int c = 0; c < 9; ++c)
            C_out[c * n + dst] = pic ? lane_ld(vbi + (3 + c) * n, li) : hC[c];
        } else {
          T yr[12];
          load_y(Y, n, i0, li, full, yr);
#pragma unroll
          for (int c = 0; c < 3; ++c) v_out[c * n + dst] = lane_ld(vbi + c * n, li) + (yr[c] + hv[c]);
#pragma unroll
          for (int c = 0; c < 9; ++c)
            C_out[c * n + dst] = lane_ld(vbi + (3 + c) * n, li) + (yr[3 + c] + keepC * hC[c]);
        }
      } else {
        T D[12];
        if (FIRST) {
#pragma unroll
          for (int c = 0; c < 3; ++c) D[c] = hv[c] - lane_ld(vbi + c * n, li);
#pragma unroll
          for (int c = 0; c < 9; ++c) D[3 + c] = keepC * (hC[c] - lane_ld(vbi + (3 + c) * n, li));
        } else {
          T yr[12];
          load_y(Y, n, i0, li, full, yr);
#pragma unroll
          for (int c = 0; c < 3; ++c) D[c] = yr[c] + hv[c];
#pragma unroll
          for (int c = 0; c < 9; ++c) D[3 + c] = yr[3 + c] + keepC * hC[c];
        }
        const T *ni = nrm + i0;
        const double nd[3] = {(double)lane_ld(ni, li), (double)lane_ld(ni + n, li),
                              (double)lane_ld(ni + 2 * n, li)};
        if (nd[0] == 0.0 && nd[1] == 0.0 && nd[2] == 0.0) {  // unconstrained
#pragma unroll
          for (int c = 0; c < 12; ++c) W[c] = T(0);
        } else {
          const double dd[3] = {(double)D[0], (double)D[1], (double)D[2]};
          double wv[3];
          undesirable(dd, nd, sd.mu, wv);
#pragma unroll
          for (int c = 0; c < 3; ++c) W[c] = (T)wv[c];
#pragma unroll
          for (int c = 0; c < 9; ++c) W[3 + c] = D[3 + c];
          if (flags & APIC_RULE_SEPARATE) {
            // Section 2.3: the whole change (Coulomb's W where d.n > 0, which
            // is d and all of dC), nothing where the change does not pull the
            // particle away from its surface
            const double dn = dd[0] * nd[0] + dd[1] * nd[1] + dd[2] * nd[2];
            if (!(dn > 0.0))
#pragma unroll
              for (int c = 0; c < 12; ++c) W[c] = T(0);
          }
        }
        T yr[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) yr[c] = D[c] - W[c];
        store_y(Y, n, i0, li, full, yr);
      }
    }
    if (!finishing) {
      // every lane has gathered: reuse the tile as the scatter target
      int passes = 0;
      const Pairing pl = scatter_lanes<PAIRS>(active, key & 63u, &passes);
      wave_sync();
      if (member) zero_tile<T, 3>(tile[wave]);
      wave_sync();
      if (active) {
        const T mp = lane_ld(m + i0, li);
        p2g_passes<T, PAIRS>(tile[wave], base, S, mp, W, W + 3, pl, passes);
      }
      flush_group<T, G, 3, false>(a, tile, gl, member, it.seg, gnext, 3);
    }
    wave_sync();
  }
}


// The last round (k = max n_iter + 1): G2P of the last field for the scenes
// finishing now, Vhat to (v_out, C_out) at perm[i] (or i), then for every
// particle -- including those of scenes that finished in earlier rounds,
// whose Vhat is read back -- the FP64 momentum after the step (positions
// before the drift, the stored T values of Vhat), the resident driver's
// drift x += dt v when `drift` is set, and one per-scene record per work item
// (a work item is one scene; padding items write key -1).
template <typename T, bool FIRST>
__global__ __launch_bounds__(64) void k_final(StepArgs a, int k, const T *t, const T *m,
                                              const T *vbar, const T *nrm, const T *Y, GridPtrs g,
                                              const uint32_t *perm, T *v_out, T *C_out, T *x,
                                              int drift, RedRec *rec) {
  __shared__ T tile[1][3][kTileSize];
  const uint32_t lane = threadIdx.x;
  const int64_t n = a.n;
  const T *gcur = (const T *)g.buf[(k - 1) % 3];
  const bool direct = perm == nullptr;  // outputs at the sorted index (resident state)
  for (ItemLoop L = item_loop(a); L.w < L.end; L.w += L.step) {
    const int w = L.w;
    const Item it = a.items[w];
    if (it.count == 0) {  // run padding
      if (lane == 0) rec[w].key = -1;
      continue;
    }
    const Segment &sg = a.seg[it.seg];
    const int s = sg.scene;
    const SceneDev &sd = a.sc[s];
    const bool now = sd.n_iter == k - 1;  // wave-uniform
    if (now) load_vel_tile<T>(tile[0], gcur, g.invm, sg.sslot);
    wave_sync();
    const bool active = (int)lane < it.count;
    const uint32_t li = active ? lane : 0u;
    const int64_t i0 = it.start;
    double q[kRed];
#pragma unroll
    for (int c = 0; c < kRed; ++c) q[c] = 0.0;
    if (active) {
      const int64_t dst = perm ? (int64_t)lane_ld(perm + i0, li) : i0 + li;
      T out[12];
      if (now) {
        const T h = (T)sd.h;
        T tt[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) tt[c] = lane_ld(t + c * n + i0, li);
        Stencil<T> S;
        make_stencil(tt, h, S);
        T hv[3], hC[9];
        g2p(tile[0], particle_base(lane_ld(a.keys + i0, li)), S, T(2) / (h * h), hv, hC);
        const bool pic = (sd.flags & APIC_PIC) != 0;  // PIC: C passes through (see k_iter)
#pragma unroll
        for (int c = 0; c < 9; ++c) hC[c] *= pic ? T(0) : T(1);
        if (FIRST) {  // N = 0: Vhat = H Vbar exactly as gathered
#pragma unroll
          for (int c = 0; c < 3; ++c) out[c] = hv[c];
#pragma unroll
          for (int c = 0; c < 9; ++c)
            out[3 + c] = pic ? lane_ld(vbar + (3 + c) * n + i0, li) : hC[c];
        } else {
          T yr[12];
          load_y(Y, n, i0, li, it.full_y != 0 || (sd.flags & APIC_RULE_SEPARATE) != 0, yr);
#pragma unroll
          for (int c = 0; c < 3; ++c) out[c] = lane_ld(vbar + c * n + i0, li) + (yr[c] + hv[c]);
#pragma unroll
          for (int c = 0; c < 9; ++c)
            out[3 + c] = lane_ld(vbar + (3 + c) * n + i0, li) + (yr[3 + c] + hC[c]);
        }
        if (direct) {
#pragma unroll
          for (int c = 0; c < 3; ++c) lane_st(v_out + c * n + i0, li, out[c]);
#pragma unroll
          for (int c = 0; c < 9; ++c) lane_st(C_out + c * n + i0, li, out[3 + c]);
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) v_out[c * n + dst] = out[c];
#pragma unroll
          for (int c = 0; c < 9; ++c) C_out[c * n + dst] = out[3 + c];
        }
      } else {  // finished in an earlier round
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = v_out[c * n + dst];
#pragma unroll
        for (int c = 0; c < 9; ++c) out[3 + c] = C_out[c * n + dst];
      }
      double r[3], vv[3], CC[9];
      T xp[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        xp[d] = direct ? lane_ld(x + d * n + i0, li) : x[d * n + dst];
        vv[d] = (double)out[d];
        r[d] = (double)xp[d] - sd.x_ref[d];
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) CC[c] = (double)out[3 + c];
      momentum_terms(r, vv, CC, (double)lane_ld(m + i0, li), sd.h, q);
      if (sd.n_iter > 0) {
        const T *ni = nrm + i0;
        q[10] = (lane_ld(ni, li) == T(0) && lane_ld(ni + n, li) == T(0) &&
                 lane_ld(ni + 2 * n, li) == T(0)) ? 1.0 : 0.0;
      }
      if (drift) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const T xn = xp[d] + (T)(sd.dt * vv[d]);
          if (direct)
            lane_st(x + d * n + i0, li, xn);
          else
            x[d * n + dst] = xn;
        }
      }
    }
    const double v = wave_sum_spread(q);
    if ((int)lane < kRed) rec[w].v[lane] = v;
    if (lane == 0) rec[w].key = s;
    wave_sync();
  }
}

// Workgroup shape of the grouped kernels: a.group waves (1, 4 or 8), and the
// paired scatter (FP32 only) when a.pairs is set.
#define APIC_GROUP_DISPATCH_P(KERNEL_G, P, ...)     \
  do {                                              \
    if (a.group >= 8 && sizeof(T) == 4) {          \
      constexpr int G_ = 8;                         \
      constexpr bool P_ = P;                        \
      KERNEL_G(__VA_ARGS__);                        \
    } else if (a.group >= 4) {                      \
      constexpr int G_ = 4;                         \
      constexpr bool P_ = P;                        \
      KERNEL_G(__VA_ARGS__);                        \
    } else {                                        \
      constexpr int G_ = 1;                         \
      constexpr bool P_ = P;                        \
      KERNEL_G(__VA_ARGS__);                        \
    }                                               \
  } while (0)
#define APIC_GROUP_DISPATCH(KERNEL_G, ...)                    \
  do {                                                        \
    if constexpr (sizeof(T) == 4) {                           \
      if (a.pairs) {                                          \
        APIC_GROUP_DISPATCH_P(KERNEL_G, true, __VA_ARGS__);   \
        break;                                                \
      }                                                       \
    }                                                         \
    APIC_GROUP_DISPATCH_P(KERNEL_G, false, __VA_ARGS__);      \
  } while (0)

// The launch's arguments with the XCD-split schedule (item_loop) on, where
// the grid allows it (a multiple of 8 workgroups).
static StepArgs xcd_split_args(const StepArgs &a, int grid) {
  StepArgs b = a;
  b.xcd_split = (grid % 8) == 0 ? 1 : 0;
  return b;
}

template <typename T>
void launch_mass(const StepArgs &a, const T *t, const T *m, GridPtrs g, hipStream_t st) {
#define L_MASS() APIC_LAUNCH((k_mass<T, G_, P_>), dim3(a.grid_wg), dim3(64 * G_), 0, st, a, t, m, g)
  APIC_GROUP_DISPATCH(L_MASS);
#undef L_MASS
}

template <typename T>
void launch_p2g0(const StepArgs &a, const T *t, const T *m, const T *vbar, T *nrm, Item *items,
                 GridPtrs g, hipStream_t st) {
#define L_P2G0() \
  APIC_LAUNCH((k_p2g0<T, G_, P_>), dim3(a.grid_wg), dim3(64 * G_), 0, st, a, t, m, vbar, nrm, \
              items, g)
  APIC_GROUP_DISPATCH(L_P2G0);
#undef L_P2G0
}

template <typename T>
void launch_round(const StepArgs &a, int k, const T *t, const T *m, const T *vbar, const T *nrm,
                  T *Y, GridPtrs g, const uint32_t *perm, T *v_out, T *C_out, hipStream_t st) {
#define L_ITER(FIRST_, VAR_) \
  APIC_LAUNCH((k_iter<T, FIRST_, G_, VAR_, P_>), dim3(a.grid_wg), dim3(64 * G_), 0, st, a, k, t, m, \
              vbar, nrm, Y, g, perm, v_out, C_out)
  if (k == 1 && a.variants)
    APIC_GROUP_DISPATCH(L_ITER, true, true);
  else if (k == 1)
    APIC_GROUP_DISPATCH(L_ITER, true, false);
  else if (a.variants)
    APIC_GROUP_DISPATCH(L_ITER, false, true);
  else
    APIC_GROUP_DISPATCH(L_ITER, false, false);
#undef L_ITER
}

template <typename T>
void launch_final(const StepArgs &a, int k, const T *t, const T *m, const T *vbar, const T *nrm,
                  const T *Y, GridPtrs g, const uint32_t *perm, T *v_out, T *C_out, T *x,
                  int drift, RedRec *rec, hipStream_t st) {
  // always the XCD-split schedule: each XCD's L2 then holds the velocity
  // tiles its neighbouring items share (the last round is bound by those
  // reloads; 59 -> 50 us on the benchmark scene)
  const StepArgs b = xcd_split_args(a, a.item_wg);
  if (k == 1)
    APIC_LAUNCH((k_final<T, true>), dim3(a.item_wg), dim3(64), 0, st, b, k, t, m, vbar, nrm, Y,
                g, perm, v_out, C_out, x, drift, rec);
  else
    APIC_LAUNCH((k_final<T, false>), dim3(a.item_wg), dim3(64), 0, st, b, k, t, m, vbar, nrm, Y,
                g, perm, v_out, C_out, x, drift, rec);
}

#define INST(T)                                                                                 \
  template void launch_mass<T>(const StepArgs &, const T *, const T *, GridPtrs, hipStream_t);  \
  template void launch_p2g0<T>(const StepArgs &, const T *, const T *, const T *, T *, Item *, \
                               GridPtrs, hipStream_t);                                          \
  template void launch_round<T>(const StepArgs &, int, const T *, const T *, const T *,          \
                                const T *, T *, GridPtrs, const uint32_t *, T *, T *,           \
                                hipStream_t);                                                   \
  template void launch_final<T>(const StepArgs &, int, const T *, const T *, const T *,          \
                                const T *, const T *, GridPtrs, const uint32_t *, T *, T *, T *, \
                                int, RedRec *, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace apic
