// transfer.hip -- the grid transfers of the APIC operator H (Section 2.1.2)
// and the augury-iteration series with the Coulomb rule (Sections 2.3-2.4).
//
// Work decomposition: particles are sorted by (body, 4x4x4 cell block, cell);
// a work item is up to 64 particles of one (body, cell block) segment and is
// processed by one 64-lane wavefront.  Every node such a particle touches lies
// in an 8x8x8 node cube made of 8 node blocks, which is staged in LDS:
//  - P2G accumulates into the LDS cube with LDS float atomics, then flushes
//    the cube to HBM with one global atomic per node and component;
//  - G2P loads the cube's grid velocities with coalesced 256-byte rows and
//    gathers the 64 stencil nodes of each particle from LDS.
// The quadratic spline weights are separable, so P2G and G2P use per-axis
// partial sums (about 580 FMA each per particle instead of 1000+).
//
// Precision: T = float for the mixed path (weights, P2G/G2P accumulation,
// grid momenta), T = double for the plain FP64 path.  Grid velocity q/m,
// normals, the friction rule and all reductions use double in both.
#include "kernels.h"

namespace apic {

template <typename T>
struct Stencil {
  T w[3][4];    // N per axis (Appendix B basis, 1/4 middle coefficients)
  T wdx[3][4];  // N * (x_i - x_p) per axis
  T dx[3][4];   // x_i - x_p per axis
};

// Per-axis basis of Appendix B at cell-relative coordinate t in [0, 1):
// nodes c-1..c+2 carry (1-t)^2/4, (2-t^2)/4, (1+2t-t^2)/4, t^2/4.
template <typename T>
__device__ __forceinline__ void make_stencil(const T t[3], T h, Stencil<T> &S) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T tt = t[d], u = T(1) - tt, t2 = tt * tt;
    S.w[d][0] = T(0.25) * u * u;
    S.w[d][1] = T(0.25) * (T(2) - t2);
    S.w[d][2] = T(0.25) * (T(1) + T(2) * tt - t2);
    S.w[d][3] = T(0.25) * t2;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      S.dx[d][a] = h * (T(a - 1) - tt);
      S.wdx[d][a] = S.w[d][a] * S.dx[d][a];
    }
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
          sz[q] += S.wdx[2][c] * v;
        }
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        r[q] += S.w[1][b] * s[q];
        ry[q] += S.wdx[1][b] * s[q];
        rz[q] += S.w[1][b] * sz[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      vel[q] += S.w[0][a] * r[q];
      Bm[q][0] += S.wdx[0][a] * r[q];
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
      A[q] = S.w[0][a] * (mu[q] + mE[q][0] * S.dx[0][a]);
      Ay[q] = S.w[0][a] * mE[q][1];
      Az[q] = S.w[0][a] * mE[q][2];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T P[3], Q[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        P[q] = S.w[1][b] * (A[q] + Ay[q] * S.dx[1][b]);
        Q[q] = S.w[1][b] * Az[q];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int idx = base + a + kTileX * b + kTileZStride * c;
#pragma unroll
        for (int q = 0; q < 3; ++q) atomicAdd(&tq[q][idx], S.w[2][c] * P[q] + S.wdx[2][c] * Q[q]);
      }
    }
  }
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

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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

template <typename T, int NC>
__device__ __forceinline__ void zero_tile(T (*tile)[kTileSize]) {
  const int lane = threadIdx.x & 63;
  for (int i = lane; i < kTileSize; i += 64)
#pragma unroll
    for (int q = 0; q < NC; ++q) tile[q][i] = T(0);
}

// ---------------------------------------------------------------------------
// P2G of mass (shared and per body) and of Vbar into buffer 0
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_p2g0(StepArgs a, const T *t, const T *m, const T *vbar,
                                             GridPtrs g) {
  __shared__ T tq[3][kTileSize];
  __shared__ T tm[1][kTileSize];
  __shared__ double tb[1][kTileSize];
  zero_tile<T, 3>(tq);
  zero_tile<T, 1>(tm);
  zero_tile<double, 1>(tb);
  __syncthreads();
  const int lane = threadIdx.x;
  const int nitems = (a.cnt->err & kErrCapacity) ? 0 : a.cnt->n_items;
  const int64_t n = a.n;
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const Item it = a.items[w];
    const Segment &sg = a.seg[it.seg];
    const SceneDev &sd = a.sc[sg.scene];
    if (lane < it.count) {
      const int64_t i = it.start + lane;
      const uint32_t key = a.keys[i];
      const int base = particle_base(key);
      T tt[3] = {t[i], t[n + i], t[2 * n + i]};
      Stencil<T> S;
      make_stencil(tt, (T)sd.h, S);
      const T mp = m[i];
      T u[3], E[9];
#pragma unroll
      for (int q = 0; q < 3; ++q) u[q] = vbar[q * n + i];
#pragma unroll
      for (int q = 0; q < 9; ++q) E[q] = vbar[(3 + q) * n + i];
      p2g(tq, base, S, mp, u, E);
#pragma unroll
      for (int aa = 0; aa < 4; ++aa)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const T wab = S.w[0][aa] * S.w[1][b] * mp;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int idx = base + aa + kTileX * b + kTileZStride * c;
            const T wm = wab * S.w[2][c];
            atomicAdd(&tm[0][idx], wm);
            atomicAdd(&tb[0][idx], (double)wm);
          }
        }
    }
    __syncthreads();
    flush_tile<T, 3>(tq, (T *)g.buf[0], sg.sslot, 3);
    flush_tile<T, 1>(tm, (T *)g.mass, sg.sslot, 1);
    flush_tile<double, 1>(tb, g.bmass, sg.bslot, 1);
    __syncthreads();
  }
}

template <typename T>
void launch_p2g0(const StepArgs &a, const T *t, const T *m, const T *vbar, GridPtrs g,
                 hipStream_t st) {
  k_p2g0<T><<<a.grid_wg, 64, 0, st>>>(a, t, m, vbar, g);
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

template <typename T>
void launch_gridvel(const StepArgs &a, GridPtrs g, int cur, hipStream_t st) {
  k_gridvel<T><<<a.grid_wg * 2, 256, 0, st>>>(a.cnt, (const T *)g.mass, (T *)g.buf[cur],
                                               (T *)g.buf[1 - cur]);
}

// ---------------------------------------------------------------------------
// One round k of the series (fused G2P + rule + P2G)
// ---------------------------------------------------------------------------
// Stored per particle between rounds: Y = D_{k-1} - W_k, so that after the
// next G2P (of W_k) the accumulated change is D_k = Y + H W_k, and the final
// answer is Vhat = Vbar + D_N.  Round 1 starts from D_0 = H Vbar - Vbar.
template <typename T, bool FIRST>
__global__ __launch_bounds__(64) void k_iter(StepArgs a, int k, const T *t, const T *m,
                                             const T *vbar, T *nrm, T *Y, GridPtrs g, int cur,
                                             const uint32_t *perm, T *v_out, T *C_out, T *x_io,
                                             double dt, double *red) {
  __shared__ T tv[3][kTileSize];
  __shared__ T tq[3][kTileSize];
  __shared__ double tb[FIRST ? 1 : 1][FIRST ? kTileSize : 1];
  zero_tile<T, 3>(tq);
  __syncthreads();
  const int lane = threadIdx.x;
  const int nitems = (a.cnt->err & kErrCapacity) ? 0 : a.cnt->n_items;
  const bool write_ok = a.cnt->err == 0;
  const int64_t n = a.n;
  const T *gcur = (const T *)g.buf[cur];
  T *gnext = (T *)g.buf[1 - cur];
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const Item it = a.items[w];
    const Segment &sg = a.seg[it.seg];
    const SceneDev &sd = a.sc[sg.scene];
    if (sd.n_iter < k - 1) continue;  // scene already finished (uniform per item)
    const bool finishing = sd.n_iter == k - 1;
    load_tile<T, 3>(tv, gcur, sg.sslot, 3);
    if (FIRST && !finishing) load_tile<double, 1>((double(*)[kTileSize])tb, g.bmass, sg.bslot, 1);
    __syncthreads();
    double q[kRed];
    bool have_red = false;
    if (lane < it.count) {
      const int64_t i = it.start + lane;
      const uint32_t key = a.keys[i];
      const int base = particle_base(key);
      const T h = (T)sd.h;
      T tt[3] = {t[i], t[n + i], t[2 * n + i]};
      Stencil<T> S;
      make_stencil(tt, h, S);
      T hv[3], hC[9];
      g2p(tv, base, S, T(2) / (h * h), hv, hC);
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
      if (finishing) {
        T out[12];
        if (FIRST) {  // N = 0: Vhat = H Vbar exactly as gathered
#pragma unroll
          for (int c = 0; c < 3; ++c) out[c] = hv[c];
#pragma unroll
          for (int c = 0; c < 9; ++c) out[3 + c] = hC[c];
        } else {
#pragma unroll
          for (int c = 0; c < 12; ++c) out[c] = vbar[c * n + i] + D[c];
        }
        const int64_t dst = perm ? (int64_t)perm[i] : i;
        if (write_ok) {
#pragma unroll
          for (int c = 0; c < 3; ++c) v_out[c * n + dst] = out[c];
#pragma unroll
          for (int c = 0; c < 9; ++c) C_out[c * n + dst] = out[3 + c];
        }
        double r[3], vv[3], CC[9];
        const int cl[3] = {(int)(key & 3), (int)((key >> 2) & 3), (int)((key >> 4) & 3)};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          r[c] = sd.h * ((double)(4 * sg.B[c] + cl[c]) + (double)tt[c]);
          vv[c] = (double)out[c];
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) CC[c] = (double)out[3 + c];
        if (x_io && write_ok)
#pragma unroll
          for (int c = 0; c < 3; ++c) x_io[c * n + i] = x_io[c * n + i] + (T)(dt * vv[c]);
        if (red) {
          const double h2 = 0.5 * sd.h * sd.h, mp = (double)m[i];
          q[0] = mp * vv[0];
          q[1] = mp * vv[1];
          q[2] = mp * vv[2];
          q[3] = mp * (r[1] * vv[2] - r[2] * vv[1] + h2 * (CC[7] - CC[5]));
          q[4] = mp * (r[2] * vv[0] - r[0] * vv[2] + h2 * (CC[2] - CC[6]));
          q[5] = mp * (r[0] * vv[1] - r[1] * vv[0] + h2 * (CC[3] - CC[1]));
          double v2 = vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2], c2 = 0;
#pragma unroll
          for (int c = 0; c < 9; ++c) c2 += CC[c] * CC[c];
          q[6] = 0.5 * mp * (v2 + h2 * c2);
          q[7] = mp * sqrt(v2);
          q[8] = mp * (sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) * sqrt(v2) + h2 * sqrt(c2));
          q[9] = 1.0;
          const T *nn = nrm;
          q[10] = (sd.n_iter == 0) ? 0.0
                  : (nn[i] == T(0) && nn[n + i] == T(0) && nn[2 * n + i] == T(0)) ? 1.0 : 0.0;
          have_red = true;
        }
      } else {
        double nd[3];
        if (FIRST) {
          const double td[3] = {(double)tt[0], (double)tt[1], (double)tt[2]};
          body_normal(&tb[0][0], base, td, sd.h, nd);
#pragma unroll
          for (int c = 0; c < 3; ++c) nrm[c * n + i] = (T)nd[c];
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) nd[c] = (double)nrm[c * n + i];
        }
        T W[12];
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
        p2g(tq, base, S, m[i], W, W + 3);
      }
    }
    if (red && finishing) {
      // reduce over the wave (items are single-scene)
      const uint64_t any = __ballot(have_red);
      if (any) {
#pragma unroll
        for (int c = 0; c < kRed; ++c) {
          double v = wave_sum_d(have_red ? q[c] : 0.0);
          if (lane == 0) atomicAdd(&red[(int64_t)sg.scene * kRed + c], v);
        }
      }
    }
    __syncthreads();
    if (!finishing) flush_tile<T, 3>(tq, gnext, sg.sslot, 3);
    __syncthreads();
  }
}

template <typename T>
void launch_iter(const StepArgs &a, int k, const T *t, const T *m, const T *vbar, T *nrm, T *Y,
                 GridPtrs g, int cur, const uint32_t *perm, T *v_out, T *C_out, T *x_io,
                 double dt, double *red, hipStream_t st) {
  if (k == 1)
    k_iter<T, true><<<a.grid_wg, 64, 0, st>>>(a, k, t, m, vbar, nrm, Y, g, cur, perm, v_out,
                                               C_out, x_io, dt, red);
  else
    k_iter<T, false><<<a.grid_wg, 64, 0, st>>>(a, k, t, m, vbar, nrm, Y, g, cur, perm, v_out,
                                                C_out, x_io, dt, red);
}

template <typename T>
void launch_final(const StepArgs &a, int k, const T *t, const T *m, const T *vbar, const T *Y,
                  GridPtrs g, int cur, const uint32_t *perm, T *v_out, T *C_out, T *x_io,
                  double dt, double *red, hipStream_t st) {
  launch_iter<T>(a, k, t, m, vbar, nullptr, (T *)Y, g, cur, perm, v_out, C_out, x_io, dt, red,
                 st);
}

#define INST(T)                                                                              \
  template void launch_p2g0<T>(const StepArgs &, const T *, const T *, const T *, GridPtrs,  \
                               hipStream_t);                                                 \
  template void launch_gridvel<T>(const StepArgs &, GridPtrs, int, hipStream_t);             \
  template void launch_iter<T>(const StepArgs &, int, const T *, const T *, const T *, T *,  \
                               T *, GridPtrs, int, const uint32_t *, T *, T *, T *, double,  \
                               double *, hipStream_t);                                       \
  template void launch_final<T>(const StepArgs &, int, const T *, const T *, const T *,      \
                                const T *, GridPtrs, int, const uint32_t *, T *, T *, T *,   \
                                double, double *, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace apic
