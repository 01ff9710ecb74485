// server.hip -- the continuous-batching request loop behind apic_server_*.
//
// Resident requests live in one packed arena (component-major columns with
// stride n_res, requests in admission order).  A tick admits queued requests
// that fit, repacks the arena into its second copy when the resident set has
// changed (survivors move to their new offsets, newcomers are copied in from
// the caller's arrays), runs the planned contact step over all residents
// (planned once per resident set; replayed from a graph once the set has
// settled), advances x, reads the step's status with the tick's one
// synchronisation, and copies the finished requests out.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

#include "apic_api_internal.h"

namespace apic {

// One contiguous particle range copied between two component-major layouts.
struct CopySeg {
  const void *sx, *sv, *sC, *sm;
  const uint16_t *sb;
  void *dx, *dv, *dC, *dm;
  uint16_t *db;
  int64_t s_stride, s_off, d_stride, d_off, count, start;  // start: prefix of counts
};

template <typename T>
__global__ __launch_bounds__(256) void k_copy_segs(const CopySeg *segs, int nseg, int64_t total) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].start <= q) lo = mid; else hi = mid - 1;
    }
    const CopySeg &s = segs[lo];
    const int64_t r = q - s.start;
    const int64_t si = s.s_off + r, di = s.d_off + r;
    const int64_t ss = s.s_stride, ds = s.d_stride;
    const T *sx = (const T *)s.sx, *sv = (const T *)s.sv, *sC = (const T *)s.sC;
    T *dx = (T *)s.dx, *dv = (T *)s.dv, *dC = (T *)s.dC;
#pragma unroll
    for (int c = 0; c < 3; ++c) dx[c * ds + di] = sx[c * ss + si];
#pragma unroll
    for (int c = 0; c < 3; ++c) dv[c * ds + di] = sv[c * ss + si];
#pragma unroll
    for (int c = 0; c < 9; ++c) dC[c * ds + di] = sC[c * ss + si];
    if (s.dm) ((T *)s.dm)[di] = ((const T *)s.sm)[si];
    if (s.db) s.db[di] = s.sb[si];
  }
}

// Driver position update x <- x + dt v (dt of the particle's scene), with
// the same rounding as the resident driver; skipped when the step that
// precedes it reported an error in *status.
template <typename T>
__global__ __launch_bounds__(256) void k_advance(T *x, const T *v, int64_t n, const int64_t *offs,
                                                 const double *dt, int ns,
                                                 const int32_t *status) {
  if (*status != 0) return;  // the step did nothing: neither does the drift
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (offs[mid] <= p) lo = mid; else hi = mid - 1;
    }
    const double d = dt[lo];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c * n + p] = x[c * n + p] + (T)(d * (double)v[c * n + p]);
  }
}

static unsigned grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

}  // namespace apic

using namespace apic;

// Graph capture of the tick's step: after this many ticks of one resident
// set, and only for sets of at most this many particles.
constexpr int32_t kStableTicks = 8;
constexpr int64_t kGraphMaxParticles = 4 << 20;
// Capacity headroom of a resident set's plan (grown 1.5x on each resize of
// that set, back to this value for the next set).
constexpr double kHeadroom = 1.25;

struct ServerReq {
  int64_t tag = 0;
  apic_scene scene{};
  double dt = 0.0;
  int32_t steps = 0, done = 0;
  int64_t n = 0;
  const void *x = nullptr, *v = nullptr, *C = nullptr, *m = nullptr;
  const uint16_t *body = nullptr;
  void *xo = nullptr, *vo = nullptr, *Co = nullptr;
  int64_t offset = 0;  // in the arena while resident
  int64_t footprint = 0;
  bool cancelled = false;
};

struct apic_server {
  apic_ctx *ctx = nullptr;
  apic_precision prec = APIC_FP32_MIXED;
  int64_t cap = 0;
  int32_t max_scenes = 0;
  int64_t budget = 0;
  // arena copies: x[3][n], v[3][n], C[9][n], m[n] (T) and body[n]
  void *col[2] = {nullptr, nullptr};
  uint16_t *body[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t n_res = 0;
  std::deque<ServerReq> queue;
  std::vector<ServerReq> resident;
  int64_t used = 0;  // summed footprint of residents
  // device tables and their pinned staging
  CopySeg *segs = nullptr;
  int64_t *offs = nullptr;
  double *dts = nullptr;
  void *stage = nullptr;
  size_t stage_bytes = 0;
  bool tables_ok = false;
  // planned step of the current resident set: measured when the set changes,
  // enqueued without host synchronisation, and once the set has been stepped
  // unchanged, captured with the drift into a graph that later ticks replay
  apic_plan *plan = nullptr;
  bool plan_ok = false;
  double headroom = kHeadroom;
  int32_t *status_dev = nullptr;   // the step's apic_status (device)
  int32_t *status_host = nullptr;  // its copy (pinned)
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t stable = 0;              // ticks stepped with the current plan
};

// The plan and graph no longer match the resident set.
static void drop_plan(apic_server *S) {
  S->plan_ok = false;
  S->stable = 0;
  if (S->exec) {
    (void)hipGraphExecDestroy(S->exec);
    S->exec = nullptr;
  }
}

static size_t tsize(apic_precision p) { return p == APIC_FP64 ? 8 : 4; }


// Column pointers of arena copy k at stride n.
static void arena_cols(apic_server *S, int k, int64_t n, void **x, void **v, void **C, void **m) {
  char *b = (char *)S->col[k];
  const size_t t = tsize(S->prec);
  *x = b;
  *v = b + t * 3 * n;
  *C = b + t * 6 * n;
  *m = b + t * 15 * n;
}

template <typename T>
static apic_status copy_segs(apic_server *S, hipStream_t st, const std::vector<CopySeg> &segs,
                             size_t stage_off) {
  if (segs.empty()) return APIC_OK;
  const size_t bytes = sizeof(CopySeg) * segs.size();
  std::memcpy((char *)S->stage + stage_off, segs.data(), bytes);
  CopySeg *dev = S->segs + stage_off / sizeof(CopySeg);
  HIPOK(hipMemcpyAsync(dev, (char *)S->stage + stage_off, bytes, hipMemcpyHostToDevice, st));
  const int64_t total = segs.back().start + segs.back().count;
  hipLaunchKernelGGL(k_copy_segs<T>, dim3(grid_for(total)), dim3(256), 0, st, dev,
                     (int)segs.size(), total);
  HIPOK(hipGetLastError());
  return APIC_OK;
}

// Repack the arena into its other copy: the residents (survivors at their
// current offsets) then the newcomers (from the caller's arrays), and upload
// the scene offsets and time steps of the position update.  The copy
// completes before the next host write of the staging buffer (the tick
// synchronises before returning).
template <typename T>
static apic_status repack(apic_server *S, hipStream_t st, std::vector<ServerReq> &joined) {
  int64_t n_new = 0;
  for (const ServerReq &r : S->resident) n_new += r.n;
  for (const ServerReq &r : joined) n_new += r.n;
  const int src = S->cur, dst = 1 - S->cur;
  void *sx, *sv, *sC, *sm, *dx, *dv, *dC, *dm;
  arena_cols(S, src, S->n_res, &sx, &sv, &sC, &sm);
  arena_cols(S, dst, n_new, &dx, &dv, &dC, &dm);
  std::vector<CopySeg> segs;
  int64_t off = 0;
  auto add = [&](const void *ax, const void *av, const void *aC, const void *am,
                 const uint16_t *ab, int64_t s_stride, int64_t s_off, int64_t count) {
    CopySeg c;
    c.sx = ax, c.sv = av, c.sC = aC, c.sm = am, c.sb = ab;
    c.dx = dx, c.dv = dv, c.dC = dC, c.dm = dm, c.db = S->body[dst];
    c.s_stride = s_stride, c.s_off = s_off, c.d_stride = n_new, c.d_off = off;
    c.count = count, c.start = off;
    segs.push_back(c);
    off += count;
  };
  for (ServerReq &r : S->resident) {
    if (r.n > 0) add(sx, sv, sC, sm, S->body[src], S->n_res, r.offset, r.n);
    r.offset = off - r.n;
  }
  for (ServerReq &r : joined) {
    if (r.n > 0) add(r.x, r.v, r.C, r.m, r.body, r.n, 0, r.n);
    r.offset = off - r.n;
    S->resident.push_back(r);
  }
  joined.clear();
  TRY(copy_segs<T>(S, st, segs, 0));
  S->cur = dst;
  S->n_res = n_new;
  const int ns = (int)S->resident.size();
  size_t toff = sizeof(CopySeg) * (size_t)(2 * S->max_scenes + 2);
  int64_t *ho = (int64_t *)((char *)S->stage + toff);
  double *hd = (double *)((char *)S->stage + toff + sizeof(int64_t) * (S->max_scenes + 1));
  for (int i = 0; i < ns; ++i) ho[i] = S->resident[i].offset, hd[i] = S->resident[i].dt;
  if (ns > 0) {
    HIPOK(hipMemcpyAsync(S->offs, ho, sizeof(int64_t) * ns, hipMemcpyHostToDevice, st));
    HIPOK(hipMemcpyAsync(S->dts, hd, sizeof(double) * ns, hipMemcpyHostToDevice, st));
  }
  S->tables_ok = true;
  drop_plan(S);
  S->headroom = kHeadroom;
  return APIC_OK;
}

template <typename T>
static apic_status server_tick(apic_server *S, hipStream_t st, apic_tick *info, int64_t *done_tags,
                               int32_t *done_status, int32_t max_done) {
  apic_tick tk{};
  int32_t reported = 0;
  auto report_done = [&](int64_t tag, apic_status status) {
    if (reported < max_done) {
      if (done_tags) done_tags[reported] = tag;
      if (done_status) done_status[reported] = status;
    }
    reported += 1;
  };
  // ---- cancelled residents leave first (outputs untouched) -------------
  {
    std::vector<ServerReq> keep;
    for (ServerReq &r : S->resident) {
      if (r.cancelled) {
        S->used -= r.footprint;
        S->tables_ok = false;
      } else {
        keep.push_back(r);
      }
    }
    S->resident.swap(keep);
  }
  // ---- admission (FIFO) -------------------------------------------------
  std::vector<ServerReq> joined;
  int64_t n_new = 0;
  for (const ServerReq &r : S->resident) n_new += r.n;
  while (!S->queue.empty()) {
    const ServerReq &r = S->queue.front();
    const int32_t ns = (int32_t)(S->resident.size() + joined.size());
    if (ns >= S->max_scenes || n_new + r.n > S->cap ||
        (S->budget > 0 && S->used + r.footprint > S->budget))
      break;
    joined.push_back(r);
    S->used += r.footprint;
    n_new += r.n;
    S->queue.pop_front();
  }
  tk.admitted = (int32_t)joined.size();
  tk.deferred = (int32_t)S->queue.size();  // waiting for room, a slot or budget
  if (!joined.empty() || !S->tables_ok) TRY(repack<T>(S, st, joined));
  // ---- one driver step of every resident request -------------------------
  // Vbar = V + dt {a, 0} is formed inside the step, so a failed step leaves
  // the arena untouched (and the drift is skipped on the device).  A request
  // whose particles the device rejects (non-finite values, a body id beyond
  // its bodies, a stencil node outside its dense grid) is retired with that
  // status and the step is re-run for the others; a step that outgrows its
  // plan is re-planned with more headroom and re-run.
  void *x = nullptr, *v = nullptr, *C = nullptr, *m = nullptr;
  std::vector<apic_scene> table;
  std::vector<double> dts;
  std::vector<int32_t> serr;
  // retire the requests the device flagged; false if none was flagged
  auto retire_flagged = [&]() -> bool {
    bool any = false;
    std::vector<ServerReq> keep;
    for (size_t i = 0; i < S->resident.size(); ++i) {
      ServerReq &r = S->resident[i];
      if (serr[i]) {
        any = true;
        report_done(r.tag, status_of_error_bits(serr[i]));
        tk.failed += 1;
        S->used -= r.footprint;
      } else {
        keep.push_back(r);
      }
    }
    if (any) S->resident.swap(keep);
    return any;
  };
  for (int attempt = 0;; ++attempt) {
    const int ns = (int)S->resident.size();
    if (ns == 0 || S->n_res == 0) break;
    if (attempt >= 16) return APIC_E_DEVICE;
    arena_cols(S, S->cur, S->n_res, &x, &v, &C, &m);
    serr.assign(ns, 0);
    if (!S->plan_ok) {
      table.resize(ns);
      dts.resize(ns);
      for (int i = 0; i < ns; ++i) {
        table[i] = S->resident[i].scene;
        table[i].offset = S->resident[i].offset;
        table[i].count = S->resident[i].n;
        dts[i] = S->resident[i].dt;
      }
      drop_plan(S);
      if (!S->plan) S->plan = plan_new(S->ctx, 1.5);
      const apic_status rc = plan_measure(S->plan, st, table.data(), ns, S->n_res, x,
                                          S->body[S->cur], S->prec, S->headroom, dts.data());
      if (rc != APIC_OK) {
        // a particle error found by the layout: name the scenes, retire them
        if (plan_scene_errors(S->plan, st, serr.data()) != APIC_OK || !retire_flagged())
          return rc;
        std::vector<ServerReq> none;
        TRY(repack<T>(S, st, none));
        continue;
      }
      S->plan_ok = true;
    }
    tk.replayed = S->exec != nullptr;
    if (S->exec) {
      HIPOK(hipGraphLaunch(S->exec, st));
    } else {
      TRY(apic_plan_step(S->plan, st, nullptr, x, v, C, m, S->body[S->cur], nullptr, nullptr,
                         S->status_dev));
      hipLaunchKernelGGL(k_advance<T>, dim3(grid_for(S->n_res)), dim3(256), 0, st, (T *)x,
                         (const T *)v, S->n_res, S->offs, S->dts, ns, S->status_dev);
      HIPOK(hipGetLastError());
    }
    HIPOK(hipMemcpyAsync(S->status_host, S->status_dev, sizeof(int32_t), hipMemcpyDeviceToHost,
                         st));
    HIPOK(hipStreamSynchronize(st));
    const apic_status rc = (apic_status)*S->status_host;
    if (rc == APIC_OK) {
      S->stable += 1;
      break;
    }
    if (rc == APIC_E_RESIZE) {  // nothing was written: plan again with more room
      S->headroom = std::min(64.0, S->headroom * 1.5);
      drop_plan(S);
      continue;
    }
    TRY(plan_scene_errors(S->plan, st, serr.data()));
    if (!retire_flagged()) return rc;  // not attributable to a request
    std::vector<ServerReq> none;
    TRY(repack<T>(S, st, none));
  }
  const int ns = (int)S->resident.size();
  tk.resident = ns;
  tk.particles = S->n_res;
  tk.footprint = S->used;
  tk.queued = (int32_t)S->queue.size();
  if (ns == 0) {
    HIPOK(hipStreamSynchronize(st));
    if (info) *info = tk;
    return APIC_OK;
  }
  // ---- finish: copy out, retire ------------------------------------------
  std::vector<CopySeg> outs;
  int64_t start = 0;
  for (ServerReq &r : S->resident) {
    r.done += 1;
    if (r.done < r.steps || r.n == 0) continue;
    CopySeg c;
    c.sx = x, c.sv = v, c.sC = C, c.sm = nullptr, c.sb = nullptr;
    c.dx = r.xo, c.dv = r.vo, c.dC = r.Co, c.dm = nullptr, c.db = nullptr;
    c.s_stride = S->n_res, c.s_off = r.offset, c.d_stride = r.n, c.d_off = 0;
    c.count = r.n, c.start = start;
    start += r.n;
    outs.push_back(c);
  }
  TRY(copy_segs<T>(S, st, outs, sizeof(CopySeg) * (size_t)(S->max_scenes + 1)));
  HIPOK(hipStreamSynchronize(st));
  // retire: survivors keep their data at their offsets in the current copy
  // (stride n_res) until the next tick repacks them
  std::vector<ServerReq> keep;
  keep.reserve(S->resident.size());
  for (ServerReq &r : S->resident) {
    if (r.done >= r.steps) {
      report_done(r.tag, APIC_OK);
      tk.completed += 1;
      S->used -= r.footprint;
      S->tables_ok = false;
    } else {
      keep.push_back(r);
    }
  }
  S->resident.swap(keep);
  // A small set stepped kStableTicks times with one plan, with nobody
  // waiting to join, is likely to stay: capture its step and drift for the
  // next ticks to replay (large sets gain nothing from a graph: their
  // kernels dwarf the launches).
  if (S->tables_ok && S->plan_ok && !S->exec && S->stable >= kStableTicks &&
      S->queue.empty() && !S->resident.empty() && S->n_res > 0 &&
      S->n_res <= kGraphMaxParticles) {
    arena_cols(S, S->cur, S->n_res, &x, &v, &C, &m);
    hipGraph_t g = nullptr;
    HIPOK(hipStreamBeginCapture(S->capture_stream, hipStreamCaptureModeThreadLocal));
    const apic_status rc = apic_plan_step(S->plan, S->capture_stream, nullptr, x, v, C, m,
                                          S->body[S->cur], nullptr, nullptr, S->status_dev);
    hipLaunchKernelGGL(k_advance<T>, dim3(grid_for(S->n_res)), dim3(256), 0, S->capture_stream,
                       (T *)x, (const T *)v, S->n_res, S->offs, S->dts,
                       (int)S->resident.size(), S->status_dev);
    const hipError_t e = hipStreamEndCapture(S->capture_stream, &g);
    if (rc != APIC_OK || e != hipSuccess ||
        hipGraphInstantiate(&S->exec, g, nullptr, nullptr, 0) != hipSuccess)
      S->exec = nullptr;  // eager steps go on
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
  }
  if (info) *info = tk;
  return APIC_OK;
}

extern "C" {

apic_status apic_server_create(apic_ctx *ctx, apic_precision prec, int64_t max_particles,
                               int32_t max_scenes, int64_t budget_bytes, apic_server **out) {
  if (!ctx || !out || max_particles < 1 || max_particles >= ((int64_t)1 << 31) ||
      max_scenes < 1 || max_scenes > (1 << 20) || budget_bytes < 0 ||
      (prec != APIC_FP64 && prec != APIC_FP32_MIXED))
    return APIC_E_INVALID;
  if (hipSetDevice(ctx->device) != hipSuccess) return APIC_E_DEVICE;
  apic_server *S = new apic_server();
  S->ctx = ctx;
  S->prec = prec;
  S->cap = max_particles;
  S->max_scenes = max_scenes;
  S->budget = budget_bytes;
  const size_t t = tsize(prec);
  bool ok = true;
  for (int k = 0; k < 2 && ok; ++k) {
    ok = hipMalloc(&S->col[k], t * 16 * (size_t)max_particles) == hipSuccess &&
         hipMalloc((void **)&S->body[k], sizeof(uint16_t) * (size_t)max_particles) == hipSuccess;
  }
  const size_t nseg = 2 * (size_t)max_scenes + 2;
  S->stage_bytes = sizeof(CopySeg) * nseg + (sizeof(int64_t) + sizeof(double)) * (max_scenes + 1);
  ok = ok && hipMalloc((void **)&S->segs, sizeof(CopySeg) * nseg) == hipSuccess &&
       hipMalloc((void **)&S->offs, sizeof(int64_t) * (max_scenes + 1)) == hipSuccess &&
       hipMalloc((void **)&S->dts, sizeof(double) * (max_scenes + 1)) == hipSuccess &&
       hipHostMalloc(&S->stage, S->stage_bytes, hipHostMallocDefault) == hipSuccess &&
       hipMalloc((void **)&S->status_dev, sizeof(int32_t)) == hipSuccess &&
       hipHostMalloc((void **)&S->status_host, sizeof(int32_t), hipHostMallocDefault) ==
           hipSuccess &&
       hipStreamCreateWithFlags(&S->capture_stream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    apic_server_destroy(S);
    return APIC_E_NOMEM;
  }
  *out = S;
  return APIC_OK;
}

apic_status apic_server_submit(apic_server *S, int64_t tag, const apic_scene *scene, double dt,
                               int32_t steps, const void *x, const void *v, const void *C,
                               const void *m, const uint16_t *body_id, void *x_out, void *v_out,
                               void *C_out) {
  if (!S || !scene || steps < 1 || !std::isfinite(dt)) return APIC_E_INVALID;
  apic_scene sc = *scene;
  sc.offset = 0;
  TRY(validate_scenes(&sc, 1, sc.count));
  if (sc.count > 0 && (!x || !v || !C || !m || !body_id || !x_out || !v_out || !C_out))
    return APIC_E_INVALID;
  ServerReq r;
  r.tag = tag;
  r.scene = sc;
  r.dt = dt;
  r.steps = steps;
  r.n = sc.count;
  r.x = x, r.v = v, r.C = C, r.m = m, r.body = body_id;
  r.xo = x_out, r.vo = v_out, r.Co = C_out;
  r.footprint = apic_scene_footprint(r.n, &sc.grid, S->prec);
  if (r.n > S->cap || (S->budget > 0 && r.footprint > S->budget)) return APIC_E_BUDGET;
  S->queue.push_back(r);
  return APIC_OK;
}

apic_status apic_server_tick(apic_server *S, void *stream, apic_tick *info, int64_t *done_tags,
                             int32_t *done_status, int32_t max_done) {
  if (!S || ((done_tags || done_status) && max_done < 0)) return APIC_E_INVALID;
  if (hipSetDevice(S->ctx->device) != hipSuccess) return APIC_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (!done_tags && !done_status) max_done = 0;
  return S->prec == APIC_FP64
             ? server_tick<double>(S, st, info, done_tags, done_status, max_done)
             : server_tick<float>(S, st, info, done_tags, done_status, max_done);
}

apic_status apic_server_cancel(apic_server *S, int64_t tag) {
  if (!S) return APIC_E_INVALID;
  for (auto it = S->queue.begin(); it != S->queue.end(); ++it)
    if (it->tag == tag) {
      S->queue.erase(it);
      return APIC_OK;
    }
  for (ServerReq &r : S->resident)
    if (r.tag == tag && !r.cancelled) {
      r.cancelled = true;
      return APIC_OK;
    }
  return APIC_E_INVALID;
}

void apic_server_destroy(apic_server *S) {
  if (!S) return;
  (void)hipSetDevice(S->ctx->device);
  (void)hipDeviceSynchronize();
  drop_plan(S);
  if (S->plan) apic_plan_destroy(S->plan);
  if (S->status_dev) (void)hipFree(S->status_dev);
  if (S->status_host) (void)hipHostFree(S->status_host);
  if (S->capture_stream) (void)hipStreamDestroy(S->capture_stream);
  for (int k = 0; k < 2; ++k) {
    if (S->col[k]) (void)hipFree(S->col[k]);
    if (S->body[k]) (void)hipFree(S->body[k]);
  }
  if (S->segs) (void)hipFree(S->segs);
  if (S->offs) (void)hipFree(S->offs);
  if (S->dts) (void)hipFree(S->dts);
  if (S->stage) (void)hipHostFree(S->stage);
  delete S;
}

}  // extern "C"
