// misc.hip -- small kernels of the resident driver: error bookkeeping,
// per-step momentum drift, and the final unpermute to the caller's order.
#include "apic_api_internal.h"

namespace apic {

__global__ void k_clear_sticky(SimDev *dev) { dev->sticky = 0; }

void launch_clear_sticky(SimDev *dev, hipStream_t st) { APIC_LAUNCH(k_clear_sticky, dim3(1), dim3(1), 0, st, dev); }

// One thread per scene: largest relative drift of P and L so far; thread 0
// records the step's errors and counts completed steps.
__global__ void k_step_end(const Counters *cnt, const double *red, int ns, SimDev *dev,
                           double *drift) {
  const int err = cnt->err;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += gridDim.x * blockDim.x) {
    if (err) break;
    const double *b = red + kRed * s, *a = red + kRed * (ns + s);
    double dP = 0.0, dL = 0.0;
    for (int d = 0; d < 3; ++d) {
      dP = fmax(dP, fabs(a[d] - b[d]));
      dL = fmax(dL, fabs(a[3 + d] - b[3 + d]));
    }
    dP = b[7] > 0.0 ? dP / b[7] : 0.0;
    dL = b[8] > 0.0 ? dL / b[8] : 0.0;
    drift[2 * s] = fmax(drift[2 * s], dP);
    drift[2 * s + 1] = fmax(drift[2 * s + 1], dL);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    dev->sticky |= err;
    if (!err) dev->steps_done += 1;
  }
}

void launch_step_end(const Counters *cnt, const double *red, int ns, SimDev *dev, double *drift,
                     hipStream_t st) {
  unsigned g = (unsigned)((ns + 255) / 256);
  if (g < 1) g = 1;
  APIC_LAUNCH(k_step_end, dim3(g), dim3(256), 0, st, cnt, red, ns, dev, drift);
}

__global__ void k_store_scene(SceneDev *dst, SceneDev s) { *dst = s; }

void launch_store_scene(SceneDev *dst, const SceneDev &s, hipStream_t st) {
  APIC_LAUNCH(k_store_scene, dim3(1), dim3(1), 0, st, dst, s);
}

__global__ void k_iota(uint32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (uint32_t)i;
}

void launch_iota(uint32_t *p, int64_t n, hipStream_t st) {
  unsigned g = (unsigned)std::min<int64_t>(8192, (n + 255) / 256);
  APIC_LAUNCH(k_iota, dim3(g ? g : 1), dim3(256), 0, st, p, n);
}

template <typename T>
__global__ void k_unpermute(const uint32_t *orig, int64_t n, const T *xs, const T *vcs, T *x,
                            T *v, T *C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = orig[i];
    if (x)
      for (int d = 0; d < 3; ++d) x[d * n + p] = xs[d * n + i];
    if (v)
      for (int d = 0; d < 3; ++d) v[d * n + p] = vcs[d * n + i];
    if (C)
      for (int d = 0; d < 9; ++d) C[d * n + p] = vcs[(3 + d) * n + i];
  }
}

template <typename T>
void launch_unpermute(const uint32_t *orig, int64_t n, const T *x_sorted, const T *vc_sorted,
                      T *x_out, T *v_out, T *C_out, hipStream_t st) {
  unsigned g = (unsigned)std::min<int64_t>(8192, (n + 255) / 256);
  APIC_LAUNCH((k_unpermute<T>), dim3(g ? g : 1), dim3(256), 0, st, orig, n, x_sorted, vc_sorted, x_out, v_out, C_out);
}

// ---------------------------------------------------------------------------
// bodies per grid node
// ---------------------------------------------------------------------------
__global__ void k_bodies_zero(const Counters *cnt, int32_t *count, int64_t sblk_cap,
                              int32_t *body_max, int ns) {
  const int64_t sb = cnt->n_sblocks < sblk_cap ? cnt->n_sblocks : sblk_cap;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < sb * kNodesPerBlock;
       q += (int64_t)gridDim.x * blockDim.x)
    count[q] = 0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < ns;
       q += (int64_t)gridDim.x * blockDim.x)
    body_max[q] = 0;
}

// One count per (body block, node) with mass: the node of the shared grid
// that the body block overlays gains one body.
template <typename T>
__global__ void k_bodies_count(const Counters *cnt, const T *bmass, const int32_t *b2s,
                               int64_t bblk_cap, int32_t *count) {
  if (cnt->err) return;
  const int64_t bb = cnt->n_bblocks < bblk_cap ? cnt->n_bblocks : bblk_cap;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < bb * kNodesPerBlock;
       q += (int64_t)gridDim.x * blockDim.x) {
    if (!(bmass[q] > T(0))) continue;
    const int32_t s = b2s[q / kNodesPerBlock];
    if (s >= 0) atomicAdd(&count[(int64_t)s * kNodesPerBlock + (q % kNodesPerBlock)], 1);
  }
}

// The largest count over each segment's 8 shared node blocks; one wave per
// (segment, node block), 64 nodes per wave.
__global__ __launch_bounds__(256) void k_bodies_max(const Counters *cnt, const Segment *seg,
                                                    int64_t seg_cap, const int32_t *count,
                                                    int32_t *body_max) {
  if (cnt->err) return;
  const int64_t nseg = cnt->n_seg < seg_cap ? cnt->n_seg : seg_cap;
  const int64_t total = nseg * 8 * kNodesPerBlock;  // a multiple of 64: whole waves
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
       q - (threadIdx.x & 63) < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = q / (8 * kNodesPerBlock);
    const int j = (int)((q / kNodesPerBlock) & 7);
    int c = 0;
    int scene = 0;
    if (q < total) {
      const int32_t s = seg[k].sslot[j];
      scene = seg[k].scene;
      if (s >= 0) c = count[(int64_t)s * kNodesPerBlock + (q % kNodesPerBlock)];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c = max(c, __shfl_xor(c, o, 64));
    if ((threadIdx.x & 63) == 0 && q < total && c > 0) atomicMax(&body_max[scene], c);
  }
}

template <typename T>
void launch_bodies_per_node(const Counters *cnt, const Segment *seg, int64_t seg_cap,
                            const T *bmass, const int32_t *b2s, int64_t bblk_cap,
                            int64_t sblk_cap, int32_t *count, int32_t *body_max, int ns,
                            hipStream_t st) {
  auto blocks = [](int64_t work) {
    return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (work + 255) / 256)));
  };
  APIC_LAUNCH(k_bodies_zero, blocks(std::max<int64_t>(sblk_cap * kNodesPerBlock, ns)), dim3(256),
              0, st, cnt, count, sblk_cap, body_max, ns);
  APIC_LAUNCH((k_bodies_count<T>), blocks(bblk_cap * kNodesPerBlock), dim3(256), 0, st, cnt,
              bmass, b2s, bblk_cap, count);
  APIC_LAUNCH(k_bodies_max, blocks(seg_cap * 8 * kNodesPerBlock), dim3(256), 0, st, cnt, seg,
              seg_cap, count, body_max);
}
template void launch_bodies_per_node<float>(const Counters *, const Segment *, int64_t,
                                            const float *, const int32_t *, int64_t, int64_t,
                                            int32_t *, int32_t *, int, hipStream_t);
template void launch_bodies_per_node<double>(const Counters *, const Segment *, int64_t,
                                             const double *, const int32_t *, int64_t, int64_t,
                                             int32_t *, int32_t *, int, hipStream_t);

// ---------------------------------------------------------------------------
// device-side reports, status and scene tables of planned steps
// ---------------------------------------------------------------------------
__global__ void k_fill_reports(const double *red, const Counters *cnt, const int32_t *body_max,
                               int ns, apic_report *out) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += gridDim.x * blockDim.x) {
    const double *b = red + kRed * s, *af = red + kRed * (ns + s);
    apic_report R;
    for (int d = 0; d < 3; ++d) {
      R.P_before[d] = b[d];
      R.L_before[d] = b[3 + d];
      R.P_after[d] = af[d];
      R.L_after[d] = af[3 + d];
    }
    R.E_before = b[6];
    R.E_after = af[6];
    R.P_scale = b[7];
    R.L_scale = b[8];
    R.n_particles = llround(b[9]);
    R.n_unconstrained = llround(af[10]);
    R.grid_blocks = cnt->n_sblocks;
    R.max_bodies_per_node = body_max ? body_max[s] : 0;
    R.reserved = 0;
    out[s] = R;
  }
}

void launch_fill_reports(const double *red, const Counters *cnt, const int32_t *body_max, int ns,
                         apic_report *out, hipStream_t st) {
  APIC_LAUNCH(k_fill_reports, dim3((unsigned)std::max(1, (ns + 255) / 256)), dim3(256), 0, st,
              red, cnt, body_max, ns, out);
}

static __device__ int32_t status_of_err(int32_t err) {
  if (err & kErrTable) return APIC_E_TABLE;
  if (err & kErrNonFinite) return APIC_E_INVALID;
  if (err & kErrBody) return APIC_E_BODY;
  if (err & kErrOutOfGrid) return APIC_E_OUT_OF_GRID;
  if (err & kErrKeyOverflow) return APIC_E_KEY_OVERFLOW;
  if (err & (kErrCapacity | kErrResize)) return APIC_E_RESIZE;
  return err ? APIC_E_DEVICE : APIC_OK;
}

__global__ void k_status(const Counters *cnt, int32_t *status) { *status = status_of_err(cnt->err); }

void launch_status(const Counters *cnt, int32_t *status, hipStream_t st) {
  APIC_LAUNCH(k_status, dim3(1), dim3(1), 0, st, cnt, status);
}

__global__ void k_scene_table(const apic_scene *in, const SceneDev *plan_sc, int ns, int max_iter,
                              SceneDev *out, Counters *cnt) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += gridDim.x * blockDim.x) {
    const apic_scene a = in[s];
    SceneDev d = plan_sc[s];
    bool ok = a.offset == d.offset && a.count == d.count && a.n_bodies == d.n_bodies &&
              a.n_iter >= 0 && a.n_iter <= max_iter && a.mu >= 0.0 && a.grid.h > 0.0 &&
              isfinite(a.grid.h) && (a.flags & ~(APIC_PIC | APIC_RULE_SEPARATE)) == 0;
    const bool any = a.grid.dims[0] || a.grid.dims[1] || a.grid.dims[2];
    for (int k = 0; k < 3; ++k) {
      ok = ok && isfinite(a.grid.origin[k]) && isfinite(a.x_ref[k]) && isfinite(a.accel[k]) &&
           (any ? a.grid.dims[k] >= 4 : a.grid.dims[k] == 0);
      d.origin[k] = a.grid.origin[k];
      d.dims[k] = a.grid.dims[k];
      d.x_ref[k] = a.x_ref[k];
      d.accel[k] = a.accel[k];
    }
    d.h = a.grid.h;
    d.mu = a.mu;
    d.n_iter = a.n_iter;
    d.flags = a.flags;
    if (!ok) {
      atomicOr(&cnt->err, kErrTable);
      d = plan_sc[s];  // keep the layout kernels on sane values; nothing is written
    }
    out[s] = d;
  }
}

void launch_scene_table(const apic_scene *in, const SceneDev *plan_sc, int ns, int max_iter,
                        SceneDev *out, Counters *cnt, hipStream_t st) {
  APIC_LAUNCH(k_scene_table, dim3((unsigned)std::max(1, (ns + 255) / 256)), dim3(256), 0, st,
              in, plan_sc, ns, max_iter, out, cnt);
}

template void launch_unpermute<float>(const uint32_t *, int64_t, const float *, const float *,
                                      float *, float *, float *, hipStream_t);
template void launch_unpermute<double>(const uint32_t *, int64_t, const double *, const double *,
                                       double *, double *, double *, hipStream_t);

}  // namespace apic
