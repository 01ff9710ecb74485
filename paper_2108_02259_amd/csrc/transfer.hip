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
// One step runs: k_mass (grid mass and per-body mass), k_normals (contact
// normals), k_p2g0 (Vbar to grid), then for k = 1..N the fused round k_iter
// (G2P of the previous field, the rule, P2G of the next series field), and
// the final G2P.  The grid velocity q/m is formed in between by k_gridvel.
//
// Precision: T = float for the mixed path (weights, P2G/G2P accumulation,
// grid momenta), T = double for the plain FP64 path.  Grid velocity q/m,
// normals, body masses and the friction rule use double in both.
#include "kernels.h"

// Occupancy targets (waves per SIMD) handed to the register allocator; the
// FP64 kernels need twice the registers for the same state.
#define APIC_ROUND_WAVES (sizeof(T) == 4 ? 4 : 2)
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
  T mu[3], mE[3][3];
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
        for (int q = 0; q < 3; ++q) tq[q][idx] += S.w[2][c] * P[q] + S.wdx(2, c) * Q[q];
        LDS_ORDER();
      }
    }
  }
}

// Mass P2G (eq. massToGrid): N m to the shared mass tile (T) and the body's
// mass tile (double), with the same race-freedom argument as p2g.
template <typename T>
__device__ __forceinline__ void p2g_mass(T *tm, T *tb, int base, const Stencil<T> &S, T m) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T wab = S.w[0][a] * S.w[1][b] * m;
      pin(wab);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int idx = base + a + kTileX * b + kTileZStride * c;
        const T wm = wab * S.w[2][c];
        tm[idx] += wm;
        tb[idx] += wm;
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
  const int lane = threadIdx.x & 63;
  const uint64_t lower = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int rank = active ? __popcll(peers & lower) : 0;
  int mx = active ? rank : 0;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
  *passes = act ? mx + 1 : 0;
  return rank;
}

// Outward normal from the particle's own-body grid mass: n = -grad m^b / |.|;
// zero when the gradient vanishes (the particle is then unconstrained).
__device__ __forceinline__ void body_normal(const double *tb, int base, const double t[3],
                                            double h, double n[3]) {
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
        const double mi = tb[base + a + kTileX * b + kTileZStride * c];
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
#pragma unroll
  for (int a = 0; a < 3; ++a) w[a] = tau > 0.0 ? dt[a] - s * dt[a] / tau : 0.0;
}

template <typename T, int NC>
__device__ __forceinline__ void load_tile(T (*tile)[kTileSize], const T *buf, const int32_t *slot,
                                          int comps_in_buf) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int s = slot[j];
    const int li = tile_index_block(j, lane);
#pragma unroll
    for (int q = 0; q < NC; ++q)
      tile[q][li] = s >= 0 ? buf[((int64_t)s * comps_in_buf + q) * kNodesPerBlock + lane] : T(0);
  }
}

template <typename T, int NC>
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
      tile[q][li] = T(0);
      if (v != T(0) && s >= 0)
        unsafeAtomicAdd(&buf[((int64_t)s * comps_in_buf + q) * kNodesPerBlock + lane], v);
    }
  }
}

// One-component flush into a buffer of a wider type (body mass: T -> double).
template <typename T, typename U>
__device__ __forceinline__ void flush_tile_to(T (*tile)[kTileSize], U *buf, const int32_t *slot) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int s = slot[j];
    const int li = tile_index_block(j, lane);
    const T v = tile[0][li];
    tile[0][li] = T(0);
    if (v != T(0) && s >= 0) unsafeAtomicAdd(&buf[(int64_t)s * kNodesPerBlock + lane], (U)v);
  }
}

template <typename T, int NC>
__device__ __forceinline__ void zero_tile(T (*tile)[kTileSize]) {
  const int lane = threadIdx.x & 63;
  for (int i = lane; i < kTileSize; i += 64)
#pragma unroll
    for (int q = 0; q < NC; ++q) tile[q][i] = T(0);
}

// The transfer kernels run one 64-lane wavefront per workgroup.  Lanes
// exchange data only through LDS, whose instructions complete in issue order
// within a wavefront, so a compiler ordering point replaces the workgroup
// barrier -- and, unlike a barrier, does not wait for the flush atomics.
__device__ __forceinline__ void wave_sync() { LDS_ORDER(); }

template <typename T>
__device__ __forceinline__ void load_t(const T *t, int64_t n, int64_t i, T tt[3]) {
  tt[0] = t[i];
  tt[1] = t[n + i];
  tt[2] = t[2 * n + i];
}

__device__ __forceinline__ int item_count(const StepArgs &a) {
  return a.cnt->err ? 0 : a.cnt->n_items;
}

// ---------------------------------------------------------------------------
// grid mass and per-body mass
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(APIC_P2G_WAVES)))
void k_mass(StepArgs a, const T *t, const T *m, GridPtrs g) {
  __shared__ T tm[1][kTileSize];
  __shared__ T tb[1][kTileSize];  // one item's body mass; flushed into FP64
  zero_tile<T, 1>(tm);
  zero_tile<T, 1>(tb);
  wave_sync();
  const int lane = threadIdx.x;
  const int nitems = item_count(a);
  const int64_t n = a.n;
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const Item it = a.items[w];
    const Segment &sg = a.seg[it.seg];
    const bool active = lane < it.count;
    const int64_t i = it.start + (active ? lane : 0);
    const uint32_t key = a.keys[i];
    int passes;
    const int rank = cell_rank(active, key & 63u, &passes);
    if (active) {
      T tt[3];
      load_t(t, n, i, tt);
      Stencil<T> S;
      make_stencil(tt, (T)a.sc[sg.scene].h, S);
      const T mp = m[i];
      const int base = particle_base(key);
      for (int pass = 0; pass < passes; ++pass) {
        if (rank == pass) p2g_mass(&tm[0][0], &tb[0][0], base, S, mp);
        LDS_ORDER();
      }
    }
    wave_sync();
    flush_tile<T, 1>(tm, (T *)g.mass, sg.sslot, 1);
    flush_tile_to<T, double>(tb, g.bmass, sg.bslot);
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// contact normals from the per-body mass grid
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_normals(StepArgs a, const T *t, T *nrm, GridPtrs g) {
  __shared__ double tb[1][kTileSize];
  const int lane = threadIdx.x;
  const int nitems = item_count(a);
  const int64_t n = a.n;
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const Item it = a.items[w];
    const Segment &sg = a.seg[it.seg];
    const SceneDev &sd = a.sc[sg.scene];
    if (sd.n_iter == 0) continue;  // no series, normals unused
    load_tile<double, 1>(tb, g.bmass, sg.bslot, 1);
    wave_sync();
    if (lane < it.count) {
      const int64_t i = it.start + lane;
      T tt[3];
      load_t(t, n, i, tt);
      const double td[3] = {(double)tt[0], (double)tt[1], (double)tt[2]};
      double nd[3];
      body_normal(&tb[0][0], particle_base(a.keys[i]), td, sd.h, nd);
#pragma unroll
      for (int c = 0; c < 3; ++c) nrm[c * n + i] = (T)nd[c];
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// P2G of Vbar into buffer 0
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(APIC_P2G_WAVES)))
void k_p2g0(StepArgs a, const T *t, const T *m, const T *vbar, GridPtrs g) {
  __shared__ T tq[3][kTileSize];
  zero_tile<T, 3>(tq);
  wave_sync();
  const int lane = threadIdx.x;
  const int nitems = item_count(a);
  const int64_t n = a.n;
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const Item it = a.items[w];
    const Segment &sg = a.seg[it.seg];
    const bool active = lane < it.count;
    const int64_t i = it.start + (active ? lane : 0);
    const uint32_t key = a.keys[i];
    int passes;
    const int rank = cell_rank(active, key & 63u, &passes);
    if (active) {
      T tt[3];
      load_t(t, n, i, tt);
      Stencil<T> S;
      make_stencil(tt, (T)a.sc[sg.scene].h, S);
      T u[3], E[9];
#pragma unroll
      for (int q = 0; q < 3; ++q) u[q] = vbar[q * n + i];
#pragma unroll
      for (int q = 0; q < 9; ++q) E[q] = vbar[(3 + q) * n + i];
      const T mp = m[i];
      const int base = particle_base(key);
      for (int pass = 0; pass < passes; ++pass) {
        if (rank == pass) p2g(tq, base, S, mp, u, E);
        LDS_ORDER();
      }
    }
    wave_sync();
    flush_tile<T, 3>(tq, (T *)g.buf[0], sg.sslot, 3);
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// grid velocity v_i = (m_i v_i) / m_i in FP64 (0 where m_i = 0), in place;
// the other buffer is cleared for the next scatter.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gridvel(const Counters *cnt, const T *mass, T *cur,
                                                 T *other) {
  const int64_t total = (int64_t)cnt->n_sblocks * kNodesPerBlock;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t slot = q >> 6, node = q & 63;
    const double mi = (double)mass[q];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t idx = (slot * 3 + c) * kNodesPerBlock + node;
      const double p = (double)cur[idx];
      cur[idx] = mi > 0.0 ? (T)(p / mi) : T(0);
      other[idx] = T(0);
    }
  }
}

// ---------------------------------------------------------------------------
// One round k of the series (fused G2P + rule + P2G)
// ---------------------------------------------------------------------------
// Stored per particle between rounds: Y = D_{k-1} - W_k, so that after the
// next G2P (of W_k) the accumulated change is D_k = Y + H W_k, and the final
// answer is Vhat = Vbar + D_N.  Round 1 starts from D_0 = H Vbar - Vbar.
// Scenes with n_iter == k-1 finish in round k: they write Vhat and scatter
// nothing.  FINAL rounds only finish.
template <typename T, bool FIRST, bool FINAL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(APIC_ROUND_WAVES)))
void k_iter(StepArgs a, int k, const T *t, const T *m, const T *vbar, const T *nrm, T *Y,
            GridPtrs g, int cur, const uint32_t *perm, T *v_out, T *C_out) {
  // One tile: the gathered grid velocities, then (cleared) the scatter target.
  __shared__ T tile[3][kTileSize];
  const int lane = threadIdx.x;
  const int nitems = item_count(a);
  const int64_t n = a.n;
  const T *gcur = (const T *)g.buf[cur];
  T *gnext = (T *)g.buf[1 - cur];
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const Item it = a.items[w];
    const Segment &sg = a.seg[it.seg];
    const SceneDev &sd = a.sc[sg.scene];
    if (sd.n_iter < k - 1) continue;  // scene already finished (uniform per item)
    const bool finishing = FINAL || sd.n_iter == k - 1;
    load_tile<T, 3>(tile, gcur, sg.sslot, 3);
    wave_sync();
    const bool active = lane < it.count;
    const int64_t i = it.start + (active ? lane : 0);
    const uint32_t key = a.keys[i];
    const int base = particle_base(key);
    const T h = (T)sd.h;
    Stencil<T> S;
    T W[12];
    if (active) {
      T tt[3];
      load_t(t, n, i, tt);
      make_stencil(tt, h, S);
      T hv[3], hC[9];
      g2p(tile, base, S, T(2) / (h * h), hv, hC);
      if (finishing) {
        const int64_t dst = perm ? (int64_t)perm[i] : i;
        if (FIRST) {  // N = 0: Vhat = H Vbar exactly as gathered
#pragma unroll
          for (int c = 0; c < 3; ++c) v_out[c * n + dst] = hv[c];
#pragma unroll
          for (int c = 0; c < 9; ++c) C_out[c * n + dst] = hC[c];
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) v_out[c * n + dst] = vbar[c * n + i] + (Y[c * n + i] + hv[c]);
#pragma unroll
          for (int c = 0; c < 9; ++c)
            C_out[c * n + dst] = vbar[(3 + c) * n + i] + (Y[(3 + c) * n + i] + hC[c]);
        }
      } else if (!FINAL) {
        T D[12];
        if (FIRST) {
#pragma unroll
          for (int c = 0; c < 3; ++c) D[c] = hv[c] - vbar[c * n + i];
#pragma unroll
          for (int c = 0; c < 9; ++c) D[3 + c] = hC[c] - vbar[(3 + c) * n + i];
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) D[c] = Y[c * n + i] + hv[c];
#pragma unroll
          for (int c = 0; c < 9; ++c) D[3 + c] = Y[(3 + c) * n + i] + hC[c];
        }
        const double nd[3] = {(double)nrm[i], (double)nrm[n + i], (double)nrm[2 * n + i]};
        if (nd[0] == 0.0 && nd[1] == 0.0 && nd[2] == 0.0) {
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
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) Y[c * n + i] = D[c] - W[c];
      }
    }
    if (!FINAL && !finishing) {
      // every lane has gathered: reuse the tile as the scatter target
      int passes = 0;
      const int rank = cell_rank(active, key & 63u, &passes);
      wave_sync();
      zero_tile<T, 3>(tile);
      wave_sync();
      if (active) {
        const T mp = m[i];
        for (int pass = 0; pass < passes; ++pass) {
          if (rank == pass) p2g(tile, base, S, mp, W, W + 3);
          LDS_ORDER();
        }
      }
      wave_sync();
      flush_tile<T, 3>(tile, gnext, sg.sslot, 3);
    }
    wave_sync();
  }
}

template <typename T>
void launch_mass(const StepArgs &a, const T *t, const T *m, GridPtrs g, hipStream_t st) {
  APIC_LAUNCH((k_mass<T>), dim3(a.grid_wg), dim3(64), 0, st, a, t, m, g);
}

template <typename T>
void launch_normals(const StepArgs &a, const T *t, T *nrm, GridPtrs g, hipStream_t st) {
  APIC_LAUNCH((k_normals<T>), dim3(a.grid_wg), dim3(64), 0, st, a, t, nrm, g);
}

template <typename T>
void launch_p2g0(const StepArgs &a, const T *t, const T *m, const T *vbar, GridPtrs g,
                 hipStream_t st) {
  APIC_LAUNCH((k_p2g0<T>), dim3(a.grid_wg), dim3(64), 0, st, a, t, m, vbar, g);
}

template <typename T>
void launch_gridvel(const StepArgs &a, GridPtrs g, int cur, hipStream_t st) {
  APIC_LAUNCH((k_gridvel<T>), dim3(a.grid_wg * 2), dim3(256), 0, st, a.cnt, (const T *)g.mass, (T *)g.buf[cur],
                                               (T *)g.buf[1 - cur]);
}

template <typename T>
void launch_iter(const StepArgs &a, int k, bool final, const T *t, const T *m, const T *vbar,
                 const T *nrm, T *Y, GridPtrs g, int cur, const uint32_t *perm, T *v_out,
                 T *C_out, hipStream_t st) {
  if (k == 1 && final)
    APIC_LAUNCH((k_iter<T, true, true>), dim3(a.grid_wg), dim3(64), 0, st, a, k, t, m, vbar, nrm, Y, g, cur, perm, v_out,
                                                     C_out);
  else if (k == 1)
    APIC_LAUNCH((k_iter<T, true, false>), dim3(a.grid_wg), dim3(64), 0, st, a, k, t, m, vbar, nrm, Y, g, cur, perm,
                                                      v_out, C_out);
  else if (final)
    APIC_LAUNCH((k_iter<T, false, true>), dim3(a.grid_wg), dim3(64), 0, st, a, k, t, m, vbar, nrm, Y, g, cur, perm,
                                                      v_out, C_out);
  else
    APIC_LAUNCH((k_iter<T, false, false>), dim3(a.grid_wg), dim3(64), 0, st, a, k, t, m, vbar, nrm, Y, g, cur, perm,
                                                       v_out, C_out);
}

#define INST(T)                                                                                 \
  template void launch_mass<T>(const StepArgs &, const T *, const T *, GridPtrs, hipStream_t);  \
  template void launch_normals<T>(const StepArgs &, const T *, T *, GridPtrs, hipStream_t);     \
  template void launch_p2g0<T>(const StepArgs &, const T *, const T *, const T *, GridPtrs,     \
                               hipStream_t);                                                    \
  template void launch_gridvel<T>(const StepArgs &, GridPtrs, int, hipStream_t);                \
  template void launch_iter<T>(const StepArgs &, int, bool, const T *, const T *, const T *,     \
                               const T *, T *, GridPtrs, int, const uint32_t *, T *, T *,       \
                               hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace apic
