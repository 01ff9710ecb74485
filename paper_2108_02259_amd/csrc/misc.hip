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

template void launch_unpermute<float>(const uint32_t *, int64_t, const float *, const float *,
                                      float *, float *, float *, hipStream_t);
template void launch_unpermute<double>(const uint32_t *, int64_t, const double *, const double *,
                                       double *, double *, double *, hipStream_t);

}  // namespace apic
