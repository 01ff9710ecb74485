// layout.hip -- cell keys, the sorted particle layout, segments, work items and
// the sparse node-block maps of the shared and per-body grids.
//
// Cells follow Appendix B: the base node of a particle is floor((x - o)/h),
// computed in FP64 so that every precision path (and the CPU reference) agrees
// bit for bit on the cell, hence on keys and order.
#include <climits>

#include <algorithm>

#include "scan.h"

namespace apic {

// ---------------------------------------------------------------------------
// cells and boxes
// ---------------------------------------------------------------------------
struct CellInfo {
  int32_t c[3];
  double t[3];
  bool ok;
  int err;
};

template <typename T>
__device__ __forceinline__ CellInfo cell_of(const T *x, int64_t n, int64_t p, const SceneDev &s) {
  CellInfo ci;
  ci.ok = true;
  ci.err = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double xi = ((double)x[d * n + p] - s.origin[d]) / s.h;
    double f = floor(xi);
    if (!(f >= -1073741824.0 && f <= 1073741823.0)) {  // NaN fails too
      ci.ok = false;
      ci.err |= (xi != xi) ? kErrNonFinite : kErrOutOfGrid;
      f = 0.0;
    }
    ci.c[d] = (int32_t)f;
    ci.t[d] = xi - f;
    if (s.dims[d] > 0 && (ci.c[d] < 1 || ci.c[d] > s.dims[d] - 3)) {
      ci.ok = false;
      ci.err |= kErrOutOfGrid;
    }
  }
  return ci;
}

__device__ __forceinline__ void wave_minmax3(int32_t mn[3], int32_t mx[3]) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      mn[d] = min(mn[d], __shfl_xor(mn[d], o, 64));
      mx[d] = max(mx[d], __shfl_xor(mx[d], o, 64));
    }
}

// Start of a step's layout: empty scene and body boxes, zero counters (the
// error word taken from `sticky` when given), and the per-scene reduction
// sums cleared (red_n doubles).
__global__ void k_layout_init(SceneAcc *sacc, int ns, BodyAcc *bacc, int nb_cap, Counters *cnt,
                              const int32_t *sticky, double *red, int64_t red_n,
                              int32_t *scene_err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) {
    scene_err[i] = 0;
    for (int d = 0; d < 3; ++d) {
      sacc[i].bmin[d] = INT_MAX;
      sacc[i].bmax[d] = INT_MIN;
    }
    sacc[i].max_body = -1;
  }
  if (i < nb_cap)
    for (int d = 0; d < 3; ++d) {
      bacc[i].bmin[d] = INT_MAX;
      bacc[i].bmax[d] = INT_MIN;
    }
  if (i < red_n) red[i] = 0.0;
  if (i == 0) {
    Counters z = {};
    if (sticky) z.err = *sticky;
    z.max_gb = -1;
    *cnt = z;
  }
}

void launch_layout_init(SceneAcc *sacc, int ns, BodyAcc *bacc, int nb_cap, Counters *cnt,
                        const int32_t *sticky, double *red, int64_t red_n, int32_t *scene_err,
                        hipStream_t st) {
  int64_t m = std::max<int64_t>({(int64_t)ns, (int64_t)nb_cap, red_n, (int64_t)1});
  APIC_LAUNCH(k_layout_init, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, sacc, ns, bacc,
              nb_cap, cnt, sticky, red, red_n, scene_err);
}

// Cells of every particle; each wavefront emits one record with the block box
// of its body (if all its valid lanes share one body), else falls back to
// per-lane atomics.
template <typename T>
__global__ __launch_bounds__(256) void k_cells(const T *x, const uint16_t *body, int64_t n,
                                               const SceneDev *sc, int ns, BodyAcc *bacc,
                                               BoxRec *rec, Counters *cnt, int32_t *scene_err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int64_t wave = p >> 6;
  bool ok = p < n;
  int gb = 0, err = 0, s = 0;
  int32_t B[3] = {0, 0, 0};
  if (ok) {
    s = scene_of(sc, ns, p);
    const SceneDev sd = sc[s];
    CellInfo ci = cell_of(x, n, p, sd);
    err |= ci.err;
    const int b = body[p];
    if (b >= sd.n_bodies) {
      err |= kErrBody;
      ci.ok = false;
    }
    gb = sd.body_base + b;
    ok = ci.ok;
#pragma unroll
    for (int d = 0; d < 3; ++d) B[d] = floor_div4(ci.c[d]);
  }
  if (err) {
    atomicOr(&cnt->err, err);
    atomicOr(&scene_err[s], err);  // which scene's particles are at fault
  }
  const uint64_t valid = __ballot(ok);
  BoxRec r;
  r.key = -1;
  r.pad = 0;
  if (valid) {
    const int first = __ffsll((unsigned long long)valid) - 1;
    const int gb0 = __shfl(gb, first, 64);
    const bool uniform = __ballot(ok && gb != gb0) == 0;
    if (uniform) {
      int32_t mn[3], mx[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        mn[d] = ok ? B[d] : INT_MAX;
        mx[d] = ok ? B[d] : INT_MIN;
      }
      wave_minmax3(mn, mx);
      r.key = gb0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        r.mn[d] = mn[d];
        r.mx[d] = mx[d];
      }
    } else if (ok) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        atomicMin(&bacc[gb].bmin[d], B[d]);
        atomicMax(&bacc[gb].bmax[d], B[d]);
      }
      atomicMax(&cnt->max_gb, gb);
    }
  }
  if (lane == 0) rec[wave] = r;
}

template <typename T>
void launch_cells(const T *x, const uint16_t *body, int64_t n, const SceneDev *sc, int ns,
                  BodyAcc *bacc, BoxRec *rec, Counters *cnt, int32_t *scene_err, hipStream_t st) {
  if (n <= 0) return;
  APIC_LAUNCH((k_cells<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, body, n, sc,
              ns, bacc, rec, cnt, scene_err);
}

// Block-wide reduction of 256 box records: one set of atomics per block when
// all its records name one body, per record otherwise; and one atomic max of
// the block's largest body index into cnt->max_gb.
__global__ __launch_bounds__(256) void k_reduce_box(const BoxRec *rec, int64_t count,
                                                    BodyAcc *bacc, Counters *cnt) {
  __shared__ int32_t smn[3][4], smx[3][4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  BoxRec r;
  r.key = -1;
  if (i < count) r = rec[i];
  __shared__ int32_t key0, kmax;
  if (threadIdx.x == 0) key0 = -2, kmax = -1;
  __syncthreads();
  if (r.key >= 0) {
    atomicCAS(&key0, -2, r.key);
    atomicMax(&kmax, r.key);
  }
  __syncthreads();
  if (threadIdx.x == 0 && kmax >= 0) atomicMax(&cnt->max_gb, kmax);
  const int k0 = key0;
  const bool uniform = __syncthreads_and(r.key < 0 || r.key == k0);
  if (k0 < 0) return;  // no valid record in this block
  if (uniform) {
    int32_t mn[3], mx[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      mn[d] = r.key >= 0 ? r.mn[d] : INT_MAX;
      mx[d] = r.key >= 0 ? r.mx[d] : INT_MIN;
    }
    wave_minmax3(mn, mx);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
      for (int d = 0; d < 3; ++d) {
        smn[d][wave] = mn[d];
        smx[d][wave] = mx[d];
      }
    __syncthreads();
    if (threadIdx.x == 0)
      for (int d = 0; d < 3; ++d) {
        int32_t a = smn[d][0], b = smx[d][0];
        for (int w = 1; w < 4; ++w) {
          a = min(a, smn[d][w]);
          b = max(b, smx[d][w]);
        }
        atomicMin(&bacc[k0].bmin[d], a);
        atomicMax(&bacc[k0].bmax[d], b);
      }
  } else if (r.key >= 0) {
    for (int d = 0; d < 3; ++d) {
      atomicMin(&bacc[r.key].bmin[d], r.mn[d]);
      atomicMax(&bacc[r.key].bmax[d], r.mx[d]);
    }
  }
}

void launch_reduce_box(const BoxRec *rec, int64_t count, BodyAcc *bacc, Counters *cnt,
                       hipStream_t st) {
  if (count <= 0) return;
  APIC_LAUNCH(k_reduce_box, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, rec, count,
              bacc, cnt);
}

// ---------------------------------------------------------------------------
// domains: body key offsets and node-block maps (one workgroup)
// ---------------------------------------------------------------------------
// Exclusive scan of one int64 per thread across the 1024-thread block.
__device__ __forceinline__ int64_t block_excl_scan64(int64_t x, int64_t *lds, int64_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int64_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) lds[wave] = inc;
  __syncthreads();
  int64_t woff = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    int64_t v = lds[w];
    if (w < wave) woff += v;
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return woff + inc - x;
}

__device__ __forceinline__ int scene_of_body(const SceneDev *sc, int ns, int gb) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sc[mid].body_base <= gb) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Bodies in capacity order (scene-major, so empty bodies take no key space):
// key and body-map offsets by a block scan; scene boxes as the union of their
// bodies' boxes; then scene-map offsets.
__global__ __launch_bounds__(1024) void k_domains(const SceneDev *sc, int ns, int nb_cap,
                                                  SceneAcc *sacc, const BodyAcc *bacc,
                                                  SceneLay *slay, BodyLay *blay, Counters *cnt,
                                                  int key_bits, int64_t smap_cap,
                                                  int64_t bmap_cap) {
  __shared__ int64_t lds[16];
  int64_t carry_key = 0, carry_bmap = 0, carry_smap = 0;
  // bodies past the last one holding a particle are empty and never looked up
  const int nb_used = min(nb_cap, cnt->max_gb + 1);
  for (int base = 0; base < nb_used; base += 1024) {
    const int gb = base + threadIdx.x;
    int64_t kv = 0, mv = 0;
    BodyAcc ba;
    bool ne = false;
    if (gb < nb_used) {
      ba = bacc[gb];
      ne = ba.bmin[0] <= ba.bmax[0];
      if (ne) {
        kv = 8;
        mv = 1;
        for (int d = 0; d < 3; ++d) {
          int64_t e = (int64_t)(ba.bmax[d] - ba.bmin[d] + 1);
          kv *= (int64_t)((ba.bmax[d] >> 1) - (ba.bmin[d] >> 1) + 1);
          mv *= e + 1;
        }
      }
    }
    int64_t tk, tb;
    const int64_t koff = block_excl_scan64(kv, lds, &tk) + carry_key;
    const int64_t boff = block_excl_scan64(mv, lds, &tb) + carry_bmap;
    if (gb < nb_used) {
      const int s = scene_of_body(sc, ns, gb);
      BodyLay bl;
      bl.scene = s;
      bl.key_off = (int32_t)(koff < kMaxKeyBlocks ? koff : kMaxKeyBlocks);
      bl.bmap_off = boff;
      for (int d = 0; d < 3; ++d) {
        bl.bmin[d] = ne ? ba.bmin[d] : 0;
        bl.ext[d] = ne ? ba.bmax[d] - ba.bmin[d] + 1 : 0;
        bl.kmin[d] = ne ? ba.bmin[d] >> 1 : 0;
        bl.kext[d] = ne ? (ba.bmax[d] >> 1) - (ba.bmin[d] >> 1) + 1 : 0;
      }
      blay[gb] = bl;
      if (ne)
        for (int d = 0; d < 3; ++d) {
          atomicMin(&sacc[s].bmin[d], ba.bmin[d]);
          atomicMax(&sacc[s].bmax[d], ba.bmax[d]);
        }
    }
    carry_key += tk;
    carry_bmap += tb;
  }
  __syncthreads();
  for (int base = 0; base < ns; base += 1024) {
    const int s = base + threadIdx.x;
    int64_t vol = 0;
    SceneAcc a;
    if (s < ns) {
      a = sacc[s];
      if (a.bmin[0] <= a.bmax[0]) {
        vol = 1;
        for (int d = 0; d < 3; ++d) vol *= (int64_t)(a.bmax[d] - a.bmin[d] + 2);
      }
    }
    int64_t ts;
    const int64_t soff = block_excl_scan64(vol, lds, &ts) + carry_smap;
    if (s < ns) {
      SceneLay L;
      L.smap_off = soff;
      const bool ne = a.bmin[0] <= a.bmax[0];
      for (int d = 0; d < 3; ++d) {
        L.smin[d] = ne ? a.bmin[d] : 0;
        L.sext[d] = ne ? a.bmax[d] - a.bmin[d] + 2 : 0;
      }
      slay[s] = L;
    }
    carry_smap += ts;
  }
  if (threadIdx.x == 0) {
    if (carry_key > kMaxKeyBlocks) atomicOr(&cnt->err, kErrKeyOverflow);
    if (key_bits > 0 && key_bits < 32 && carry_key * 64 > ((int64_t)1 << key_bits))
      atomicOr(&cnt->err, kErrResize);
    if ((smap_cap > 0 && carry_smap > smap_cap) || (bmap_cap > 0 && carry_bmap > bmap_cap))
      atomicOr(&cnt->err, kErrResize);
    cnt->key_blocks = (int32_t)(carry_key < kMaxKeyBlocks ? carry_key : kMaxKeyBlocks);
    cnt->smap_total = carry_smap;
    cnt->bmap_total = carry_bmap;
  }
}

void launch_domains(const SceneDev *sc, int ns, int nb_cap, SceneAcc *sacc, const BodyAcc *bacc,
                    SceneLay *slay, BodyLay *blay, Counters *cnt, int key_bits, int64_t smap_cap,
                    int64_t bmap_cap, hipStream_t st) {
  APIC_LAUNCH(k_domains, dim3(1), dim3(1024), 0, st, sc, ns, nb_cap, sacc, bacc, slay, blay, cnt, key_bits, smap_cap,
                                bmap_cap);
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ uint32_t cell_key(const T *x, const uint16_t *body, int64_t n,
                                            int64_t p, const SceneDev *sc, int ns,
                                            const BodyLay *blay) {
  const int s = scene_of(sc, ns, p);
  const SceneDev sd = sc[s];
  CellInfo ci = cell_of(x, n, p, sd);
  const int b = body[p];
  uint32_t key = 0;
  if (ci.ok && b < sd.n_bodies) {
    const BodyLay bl = blay[sd.body_base + b];
    int32_t L[3], sub = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int32_t B = floor_div4(ci.c[d]);
      L[d] = (B >> 1) - bl.kmin[d];
      sub |= (B & 1) << d;
    }
    int64_t lin = (int64_t)bl.key_off +
                  8 * (L[0] + (int64_t)bl.kext[0] * (L[1] + (int64_t)bl.kext[1] * L[2])) + sub;
    int cib = (ci.c[0] & 3) | ((ci.c[1] & 3) << 2) | ((ci.c[2] & 3) << 4);
    if (lin < kMaxKeyBlocks) key = (uint32_t)(lin * 64 + cib);
  }
  return key;
}

// Keys in the radix sort's tile geometry (kSortItems keys per thread), with
// the first pass's per-tile digit counts (digit-major, as the sort lays them
// out), so that the sort starts at its first scan.
template <typename T>
__global__ __launch_bounds__(kSortThreads) void k_keys(const T *x, const uint16_t *body, int64_t n,
                                                       const SceneDev *sc, int ns,
                                                       const BodyLay *blay, uint32_t *keys,
                                                       int ntiles, int shift, uint32_t *hist) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x, t = blockIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t tbase = (int64_t)t * kSortTile;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t p = tbase + (int64_t)r * kSortThreads + tid;
    const bool ok = p < n;
    uint32_t key = 0;
    if (ok) {
      key = cell_key(x, body, n, p, sc, ns, blay);
      keys[p] = key;
    }
    count_digit(h, ok, (key >> shift) & 255u);
  }
  __syncthreads();
  hist[(int64_t)tid * ntiles + t] = h[tid];
}

template <typename T>
void launch_keys(const T *x, const uint16_t *body, int64_t n, const SceneDev *sc, int ns,
                 const BodyLay *blay, uint32_t *keys, int shift, uint32_t *hist, hipStream_t st) {
  if (n <= 0) return;
  const int64_t ntiles = sort_tiles(n);
  APIC_LAUNCH((k_keys<T>), dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, x, body, n, sc, ns,
              blay, keys, (int)ntiles, shift, hist);
}

// ---------------------------------------------------------------------------
// gather into sorted order (+ momentum before)
// ---------------------------------------------------------------------------
// One record per wavefront of per-scene sums (when the wave is uniform in
// scene; per-lane atomics into `direct` otherwise).
__device__ __forceinline__ void reduce_scene(bool ok, int s, const double q[kRed], RedRec *rec,
                                             int64_t wave, double *direct) {
  const int lane = threadIdx.x & 63;
  const uint64_t valid = __ballot(ok);
  int key = -1;
  if (valid) {
    const int first = __ffsll((unsigned long long)valid) - 1;
    const int s0 = __shfl(s, first, 64);
    const bool uniform = __ballot(ok && s != s0) == 0;
    if (uniform) {
      key = s0;
      double qq[kRed];
#pragma unroll
      for (int k = 0; k < kRed; ++k) qq[k] = ok ? q[k] : 0.0;
      const double v = wave_sum_spread(qq);
      if (lane < kRed) rec[wave].v[lane] = v;
    } else if (ok) {
#pragma unroll
      for (int k = 0; k < kRed; ++k) atomicAdd(&direct[(int64_t)s * kRed + k], q[k]);
    }
  }
  if (lane == 0) rec[wave].key = key;
}

// Position of this lane's particle once the 64 sorted particles of its wave
// are also ordered by cell within each block: the sort orders by block only,
// so each block's particles form a run of lanes; a particle's new lane is its
// run's first lane plus its stable rank by 6-bit cell key within the run.
// (Lanes holding cells in x-fastest order keep the LDS tile accesses of the
// transfer kernels free of bank conflicts.)
__device__ __forceinline__ int64_t cell_order_slot(int64_t i, bool ok, uint32_t key) {
  const int lane = (int)(threadIdx.x & 63);
  const uint32_t blk = key >> 6;
  const uint32_t pblk = __shfl_up(blk, 1, 64);
  const int pok = __shfl_up(ok ? 1 : 0, 1, 64);
  const bool head = lane == 0 || pblk != blk || pok != (ok ? 1 : 0);
  const uint64_t heads = __ballot(head);
  const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1);  // lanes <= this one
  const int start = 63 - __clzll((unsigned long long)(heads & le));
  const uint64_t later = heads & ~le;
  const int end = later ? __ffsll((unsigned long long)later) - 1 : 64;
  uint64_t eq = (end == 64 ? ~0ull : ((1ull << end) - 1)) & ~((1ull << start) - 1);
  const uint32_t cell = key & 63u;
  int less = 0;
#pragma unroll
  for (int b = 5; b >= 0; --b) {
    const bool bit = (cell >> b) & 1u;
    const uint64_t m1 = __ballot(bit);
    if (bit) less += __popcll(eq & ~m1);
    eq &= bit ? m1 : ~m1;
  }
  const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(eq >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)eq, 0u));
  return i - lane + start + less + below;
}

// Also forms the step's input Vbar = V + dt {a, 0} (the resident driver's
// prediction; dt = 0 in a stateless call), copies the caller's normals into
// sorted order when given, and flags non-finite velocities, affine matrices
// or normals and non-positive or non-finite masses.
template <typename T>
__global__ __launch_bounds__(256) void k_gather(const uint32_t *perm, const uint32_t *keys,
                                                int64_t n, const T *x,
                                                const T *v, const T *C, const T *m,
                                                const uint16_t *body, const SceneDev *sc, int ns,
                                                T *t_out, T *vbar_out, T *m_out,
                                                int32_t *sbody_out, T *x_out, uint16_t *body_out,
                                                const uint32_t *orig_in, uint32_t *orig_out,
                                                uint32_t *keys_out, uint32_t *perm_out,
                                                RedRec *rec, double *direct, const T *nrm_in,
                                                T *nrm_out, Counters *cnt, int32_t *scene_err) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i0 < n;
  const uint32_t key = ok ? keys[i0] : 0u;
  const int64_t i = cell_order_slot(i0, ok, key);
  int s = 0;
  double q[kRed];
  bool bad = false;
  if (ok) {
    const int64_t p = perm[i0];
    keys_out[i] = key;
    perm_out[i] = (uint32_t)p;
    s = scene_of(sc, ns, p);
    const SceneDev sd = sc[s];
    CellInfo ci = cell_of(x, n, p, sd);
#pragma unroll
    for (int d = 0; d < 3; ++d) t_out[d * n + i] = (T)ci.t[d];
    const bool accel = sd.dt != 0.0 && (sd.accel[0] != 0.0 || sd.accel[1] != 0.0 ||
                                        sd.accel[2] != 0.0);
    double vv[3], CC[9], r[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T val = v[d * n + p];
      if (accel) val = (T)((double)val + sd.dt * sd.accel[d]);
      bad |= !isfinite((double)val);
      vbar_out[d * n + i] = val;
      vv[d] = (double)val;
      T xv = x[d * n + p];
      r[d] = (double)xv - sd.x_ref[d];
      if (x_out) x_out[d * n + i] = xv;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      T val = C[k * n + p];
      bad |= !isfinite((double)val);
      vbar_out[(3 + k) * n + i] = val;
      CC[k] = (double)val;
    }
    const T mv = m[p];
    bad |= !(mv > T(0)) || !isfinite((double)mv);
    m_out[i] = mv;
    if (nrm_in)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T nv = nrm_in[d * n + p];
        bad |= !isfinite((double)nv);
        nrm_out[d * n + i] = nv;
      }
    const int b = body[p];
    sbody_out[i] = sd.body_base + (b < sd.n_bodies ? b : 0);
    if (body_out) body_out[i] = (uint16_t)b;
    if (orig_out) orig_out[i] = orig_in ? orig_in[p] : (uint32_t)p;
    if (rec) momentum_terms(r, vv, CC, (double)mv, sd.h, q);
    if (bad) atomicOr(&scene_err[s], kErrNonFinite);
  }
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&cnt->err, kErrNonFinite);
  if (rec) reduce_scene(ok, s, q, rec, i0 >> 6, direct);
}

template <typename T>
void launch_gather(const uint32_t *perm, const uint32_t *keys, int64_t n, const T *x, const T *v,
                   const T *C, const T *m, const uint16_t *body, const SceneDev *sc, int ns,
                   T *t_out, T *vbar_out, T *m_out, int32_t *sbody_out, T *x_out,
                   uint16_t *body_out, const uint32_t *orig_in, uint32_t *orig_out,
                   uint32_t *keys_out, uint32_t *perm_out, RedRec *rec, double *direct,
                   const T *nrm_in, T *nrm_out, Counters *cnt, int32_t *scene_err,
                   hipStream_t st) {
  if (n <= 0) return;
  APIC_LAUNCH((k_gather<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, perm, keys, n,
              x, v, C, m, body, sc, ns, t_out, vbar_out, m_out, sbody_out, x_out, body_out,
              orig_in, orig_out, keys_out, perm_out, rec, direct, nrm_in, nrm_out, cnt,
              scene_err);
}

// ---------------------------------------------------------------------------
// segments and work items
// ---------------------------------------------------------------------------

// The segment tables come from two single-pass scans.  The first runs over
// the sorted particles: a particle whose block key differs from its
// predecessor's starts a segment, and the scan's output step stores that
// segment's start.  The second runs over the segments, one per thread: each
// contributes its work items (one per 64 particles, plus the run padding on
// the last segment of a run), and the output step fills in the segment
// (count, body, scene, block), marks the 8 shared and 8 body node blocks it
// touches, and writes its items.  Runs are recognised from the keys: a
// body's first block key is a multiple of 8, so key >> 9 names the (body,
// super block) pair.

__device__ __forceinline__ int64_t smap_index(const SceneLay &L, int bx, int by, int bz) {
  int rx = bx - L.smin[0], ry = by - L.smin[1], rz = bz - L.smin[2];
  return L.smap_off + rx + (int64_t)L.sext[0] * (ry + (int64_t)L.sext[1] * rz);
}

__device__ __forceinline__ int64_t bmap_index(const BodyLay &L, int bx, int by, int bz) {
  int rx = bx - L.bmin[0], ry = by - L.bmin[1], rz = bz - L.bmin[2];
  int64_t ex = L.ext[0] + 1, ey = L.ext[1] + 1;
  return L.bmap_off + rx + ex * (ry + ey * rz);
}

// 1 where a new (body, 4x4x4 block) segment starts in the sorted keys.
struct SegHeadIn {
  const uint32_t *keys;
  __device__ __forceinline__ int operator()(int64_t i, int64_t) const {
    return (i == 0 || (keys[i] >> 6) != (keys[i - 1] >> 6)) ? 1 : 0;
  }
};

struct SegHeadOut {
  Segment *seg;
  int64_t seg_cap;
  Counters *cnt;
  __device__ __forceinline__ void operator()(int64_t i, int head, int k, int64_t) const {
    if (!head) return;
    if (k >= seg_cap)
      atomicOr(&cnt->err, kErrCapacity);
    else
      seg[k].start = (int32_t)i;
  }
};

__device__ __forceinline__ int32_t seg_start(const Segment *seg, int64_t k, int64_t ns,
                                             int64_t np) {
  return k < ns ? seg[k].start : (int32_t)np;
}

// Work items of segment k: one per 64 particles; the last segment of a run
// also takes the run's padding to a multiple of `align`.  Reads only the
// starts the first scan wrote.
struct SegItemsIn {
  const Segment *seg;
  const uint32_t *keys;
  int64_t np;
  int align;
  __device__ int operator()(int64_t k, int64_t ns) const {
    const int32_t st = seg[k].start, en = seg_start(seg, k + 1, ns, np);
    int32_t items = (en - st + kItem - 1) / kItem;
    if (align > 1) {
      const uint32_t run = keys[st] >> 9;
      if (k + 1 == ns || (keys[en] >> 9) != run) {  // last segment of its run
        int32_t total = items;
        int32_t hi = st;
        for (int64_t h = k - 1; h >= 0 && k - h < 8; --h) {
          const int32_t lo = seg[h].start;
          if ((keys[lo] >> 9) != run) break;
          total += (hi - lo + kItem - 1) / kItem;
          hi = lo;
        }
        items += (align - total % align) % align;
      }
    }
    return items;
  }
};

struct ItemsOut {
  Segment *seg;
  const uint32_t *keys;
  const int32_t *sbody;
  const BodyLay *blay;
  const SceneLay *slay;
  int32_t *smark, *bmark;
  int64_t smap_cap, bmap_cap;
  Item *items;
  int64_t item_cap;
  Counters *cnt;
  int64_t *tot;
  int64_t np;
  __device__ void operator()(int64_t k, int n_items, int off, int64_t ns) const {
    if (k == 0) {  // slot-map extents for the map scans
      tot[5] = cnt->smap_total;
      tot[6] = cnt->bmap_total;
    }
    Segment &sg = seg[k];
    const int32_t start = sg.start;
    const int32_t count = seg_start(seg, k + 1, ns, np) - start;
    const uint32_t key = keys[start];
    const int gb = sbody[start];
    const BodyLay bl = blay[gb];
    const int64_t local = (int64_t)(key >> 6) - bl.key_off;
    const int sub = (int)(local & 7);
    const int64_t sl = local >> 3;
    const int ex = bl.kext[0] > 0 ? bl.kext[0] : 1, ey = bl.kext[1] > 0 ? bl.kext[1] : 1;
    int32_t B[3];
    B[0] = 2 * (bl.kmin[0] + (int)(sl % ex)) + (sub & 1);
    B[1] = 2 * (bl.kmin[1] + (int)((sl / ex) % ey)) + ((sub >> 1) & 1);
    B[2] = 2 * (bl.kmin[2] + (int)(sl / ((int64_t)ex * ey))) + ((sub >> 2) & 1);
    sg.count = count;
    sg.body = gb;
    sg.scene = bl.scene;
#pragma unroll
    for (int d = 0; d < 3; ++d) sg.B[d] = B[d];
    const SceneLay sl_ = slay[bl.scene];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      sg.sslot[j] = -1;
      sg.bslot[j] = -1;
      const int bx = B[0] + (j & 1), by = B[1] + ((j >> 1) & 1), bz = B[2] + (j >> 2);
      const int64_t si = smap_index(sl_, bx, by, bz);
      const int64_t bi = bmap_index(bl, bx, by, bz);
      if (si >= 0 && si < smap_cap) smark[si] = 1;
      if (bi >= 0 && bi < bmap_cap) bmark[bi] = 1;
    }
    // real items, then (last segment of a run) empty padding items
    for (int64_t w = off; w < (int64_t)off + n_items; ++w) {
      if (w >= item_cap) {
        atomicOr(&cnt->err, kErrCapacity);
        break;
      }
      const int32_t s = (int32_t)(w - off) * kItem;
      Item it;
      it.seg = (int32_t)k;
      it.start = start + (s < count ? s : 0);
      it.count = s < count ? min(kItem, count - s) : 0;
      it.full_y = 0;
      items[w] = it;
    }
  }
};

void launch_segments(const uint32_t *keys, int64_t n, const Lookback &lb, int64_t *tot,
                     const int32_t *sbody, const BodyLay *blay, const SceneLay *slay,
                     Segment *seg, int64_t seg_cap, Item *items, int64_t item_cap, int32_t *smark,
                     int64_t smap_cap, int32_t *bmark, int64_t bmap_cap, int align, Counters *cnt,
                     hipStream_t st) {
  if (n <= 0) return;
  SegHeadIn hin{keys};
  SegHeadOut hout{seg, seg_cap, cnt};
  APIC_LAUNCH((k_scan_onepass<SegHeadIn, SegHeadOut>), dim3(scan_tiles(n)), dim3(kScanThreads),
              0, st, hin, hout, n, (const int64_t *)nullptr, &tot[0], lb.flags, lb.state);
  SegItemsIn iin{seg, keys, n, align};
  ItemsOut iout{seg, keys, sbody, blay, slay, smark, bmark, smap_cap, bmap_cap, items, item_cap,
                cnt, tot, n};
  APIC_LAUNCH((k_scan_onepass<SegItemsIn, ItemsOut, 1>), dim3(scan_tiles(seg_cap, 1)),
              dim3(kScanThreads), 0, st, iin, iout, seg_cap, (const int64_t *)&tot[0], &tot[1],
              lb.flags, lb.state);
}

// ---------------------------------------------------------------------------
// node-block maps
// ---------------------------------------------------------------------------
// Each segment's 8 slots; the marks are cleared for the next step, and the
// first thread turns the slot totals into block counts (with capacity checks).
// Also clears the step's accumulation targets over the active blocks (grid
// mass, momentum buffers 0 and 1, body mass; `words` 32-bit words per node
// value), which the previous step no longer reads, and reduces the gather's
// momentum records into gred.
__global__ void k_seg_slots(Segment *seg, Counters *cnt, int64_t seg_cap, const SceneLay *slay,
                            const BodyLay *blay, int32_t *smark, const int32_t *smap,
                            int64_t smap_cap, int32_t *bmark, const int32_t *bmap,
                            int64_t bmap_cap, const int64_t *tot, int64_t sblk_cap,
                            int64_t bblk_cap, int64_t item_cap, uint32_t *mass, uint32_t *q0,
                            uint32_t *q1, uint32_t *bmass, int words, const RedRec *grec,
                            int64_t grec_count, double *gred, int32_t *b2s) {
  // the gather's per-wave momentum records (workgroup-uniform loop)
  for (int64_t rb = blockIdx.x; rb * 256 < grec_count; rb += gridDim.x)
    reduce_rec_block(grec, rb * 256, grec_count, gred);
  {
    const int64_t sn = (tot[2] < sblk_cap ? tot[2] : sblk_cap) * kNodesPerBlock * words;
    const int64_t bn = (tot[3] < bblk_cap ? tot[3] : bblk_cap) * kNodesPerBlock * words;
    const int64_t top = 3 * sn > bn ? 3 * sn : bn;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < top;
         q += (int64_t)gridDim.x * blockDim.x) {
      if (q < 3 * sn) {
        q0[q] = 0u;
        q1[q] = 0u;
      }
      if (q < sn) mass[q] = 0u;
      if (q < bn) bmass[q] = 0u;
    }
  }
  int64_t ns = tot[0];
  if (ns > seg_cap) ns = seg_cap;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < ns * 8;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = q >> 3;
    const int j = (int)(q & 7);
    Segment &sg = seg[k];
    const int bx = sg.B[0] + (j & 1), by = sg.B[1] + ((j >> 1) & 1), bz = sg.B[2] + (j >> 2);
    int64_t si = smap_index(slay[sg.scene], bx, by, bz);
    int64_t bi = bmap_index(blay[sg.body], bx, by, bz);
    const bool sok = si >= 0 && si < smap_cap, bok = bi >= 0 && bi < bmap_cap;
    const int32_t ss = sok ? smap[si] : -1, bs = bok ? bmap[bi] : -1;
    sg.sslot[j] = ss;
    sg.bslot[j] = bs;
    if (b2s && bs >= 0 && bs < bblk_cap) b2s[bs] = ss;  // the same node block on the shared grid
    if (sok) smark[si] = 0;
    if (bok) bmark[bi] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t s = tot[2], b = tot[3];
    int err = 0;
    if (s > sblk_cap || b > bblk_cap) err |= kErrCapacity;
    if (cnt->smap_total > smap_cap || cnt->bmap_total > bmap_cap) err |= kErrCapacity;
    if (err) atomicOr(&cnt->err, err);
    cnt->n_sblocks = (int32_t)(s < sblk_cap ? s : sblk_cap);
    cnt->n_bblocks = (int32_t)(b < bblk_cap ? b : bblk_cap);
    cnt->n_seg = (int32_t)ns;
    const int64_t w = tot[1];
    cnt->n_items = (int32_t)(w < item_cap ? w : item_cap);
  }
}

void launch_maps(Segment *seg, int64_t seg_cap, const SceneLay *slay, const BodyLay *blay,
                 int32_t *smark, int32_t *smap, int64_t smap_cap, int32_t *bmark, int32_t *bmap,
                 int64_t bmap_cap, const Lookback &lb, int64_t *tot, Counters *cnt,
                 int64_t sblk_cap, int64_t bblk_cap, int64_t item_cap, GridPtrs g, int tbytes,
                 int node_wg, const RedRec *grec, int64_t grec_count, double *gred,
                 int32_t *b2s, hipStream_t st) {
  int64_t blocks = std::max<int64_t>((seg_cap * 8 + 255) / 256, node_wg);
  if (blocks > 8192) blocks = 8192;
  scan_exclusive_pair(smark, smap, smap_cap, &tot[5], &tot[2], bmark, bmap, bmap_cap, &tot[6],
                      &tot[3], lb, 1, st);
  APIC_LAUNCH(k_seg_slots, dim3((unsigned)blocks), dim3(256), 0, st, seg, cnt, seg_cap, slay,
              blay, smark, smap, smap_cap, bmark, bmap, bmap_cap, tot, sblk_cap, bblk_cap,
              item_cap, (uint32_t *)g.mass, (uint32_t *)g.buf[0], (uint32_t *)g.buf[1],
              (uint32_t *)g.bmass, tbytes / 4, grec, grec_count, gred, b2s);
}

// One workgroup per 256 records (skipped when the step has an error).
__global__ __launch_bounds__(256) void k_reduce_red(const RedRec *rec, int64_t count_cap,
                                                    const int32_t *count_dev,
                                                    const Counters *cnt, double *out) {
  if (cnt && cnt->err) return;  // workgroup-uniform
  int64_t count = count_dev ? (int64_t)*count_dev : count_cap;
  if (count > count_cap) count = count_cap;
  reduce_rec_block(rec, (int64_t)blockIdx.x * blockDim.x, count, out);
}

void launch_reduce_red(const RedRec *rec, int64_t count_cap, const int32_t *count_dev,
                       const Counters *cnt, double *out, hipStream_t st) {
  if (count_cap <= 0) return;
  APIC_LAUNCH(k_reduce_red, dim3((unsigned)((count_cap + 255) / 256)), dim3(256), 0, st, rec, count_cap, count_dev,
                                                                     cnt, out);
}

// explicit instantiations
template void launch_cells<float>(const float *, const uint16_t *, int64_t, const SceneDev *, int,
                                  BodyAcc *, BoxRec *, Counters *, int32_t *, hipStream_t);
template void launch_cells<double>(const double *, const uint16_t *, int64_t, const SceneDev *,
                                   int, BodyAcc *, BoxRec *, Counters *, int32_t *, hipStream_t);
template void launch_keys<float>(const float *, const uint16_t *, int64_t, const SceneDev *, int,
                                 const BodyLay *, uint32_t *, int, uint32_t *, hipStream_t);
template void launch_keys<double>(const double *, const uint16_t *, int64_t, const SceneDev *, int,
                                 const BodyLay *, uint32_t *, int, uint32_t *, hipStream_t);
template void launch_gather<float>(const uint32_t *, const uint32_t *, int64_t, const float *,
    const float *, const float *, const float *, const uint16_t *, const SceneDev *, int, float *,
    float *, float *, int32_t *, float *, uint16_t *, const uint32_t *, uint32_t *, uint32_t *,
    uint32_t *, RedRec *, double *, const float *, float *, Counters *, int32_t *, hipStream_t);
template void launch_gather<double>(const uint32_t *, const uint32_t *, int64_t, const double *,
    const double *, const double *, const double *, const uint16_t *, const SceneDev *, int, double *,
    double *, double *, int32_t *, double *, uint16_t *, const uint32_t *, uint32_t *, uint32_t *,
    uint32_t *, RedRec *, double *, const double *, double *, Counters *, int32_t *, hipStream_t);

}  // namespace apic
