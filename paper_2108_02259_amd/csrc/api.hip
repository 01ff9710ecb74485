// api.hip -- context, workspace and the C ABI entry points of the contact
// library (declared in include/apic_contact.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "apic_api_internal.h"
#include "kernels.h"

using namespace apic;

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
apic_status Workspace::ensure(int id, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~(size_t)255;
  if (size[id] >= bytes) return APIC_OK;
  size_t held_after = held - size[id] + bytes;
  if (budget && held_after > budget) return APIC_E_BUDGET;
  if (ptr[id]) {
    (void)hipFree(ptr[id]);
    held -= size[id];
    ptr[id] = nullptr;
    size[id] = 0;
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return APIC_E_NOMEM;
  }
  ptr[id] = p;
  size[id] = bytes;
  held += bytes;
  return APIC_OK;
}

void Workspace::release() {
  for (int i = 0; i < kNumBufs; ++i) {
    if (ptr[i]) (void)hipFree(ptr[i]);
    ptr[i] = nullptr;
    size[i] = 0;
  }
  held = 0;
}

static apic_status status_from_err(int32_t err) {
  if (err & kErrNonFinite) return APIC_E_INVALID;
  if (err & kErrBody) return APIC_E_BODY;
  if (err & kErrOutOfGrid) return APIC_E_OUT_OF_GRID;
  if (err & kErrKeyOverflow) return APIC_E_KEY_OVERFLOW;
  if (err & kErrCapacity) return APIC_E_DEVICE;
  return APIC_OK;
}

#define HIPOK(expr)                                   \
  do {                                                \
    if ((expr) != hipSuccess) {                       \
      (void)hipGetLastError();                        \
      return APIC_E_DEVICE;                           \
    }                                                 \
  } while (0)

#define TRY(expr)                       \
  do {                                  \
    apic_status _s = (expr);            \
    if (_s != APIC_OK) return _s;       \
  } while (0)

apic_status apic_ctx::host_stage(size_t bytes) {
  if (stage_bytes >= bytes) return APIC_OK;
  if (stage) (void)hipHostFree(stage);
  stage = nullptr;
  stage_bytes = 0;
  size_t b = std::max<size_t>(bytes, 4096);
  if (hipHostMalloc(&stage, b, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return APIC_E_NOMEM;
  }
  stage_bytes = b;
  return APIC_OK;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
static bool grid_ok(const apic_grid *g) {
  if (!g) return false;
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return false;
  for (int d = 0; d < 3; ++d) {
    if (!std::isfinite(g->origin[d])) return false;
    if (g->dims[d] < 0) return false;
  }
  bool any = g->dims[0] || g->dims[1] || g->dims[2];
  bool all = g->dims[0] && g->dims[1] && g->dims[2];
  if (any && !all) return false;
  if (all && (g->dims[0] < 4 || g->dims[1] < 4 || g->dims[2] < 4)) return false;
  return true;
}

apic_status validate_scenes(const apic_scene *scenes, int32_t ns, int64_t n_total) {
  if (ns < 1 || !scenes || n_total < 0) return APIC_E_INVALID;
  if (n_total >= ((int64_t)1 << 31)) return APIC_E_INVALID;
  int64_t expect = 0;
  int64_t bodies = 0;
  for (int32_t s = 0; s < ns; ++s) {
    const apic_scene &sc = scenes[s];
    if (sc.offset != expect || sc.count < 0) return APIC_E_INVALID;
    expect += sc.count;
    if (!grid_ok(&sc.grid)) return APIC_E_INVALID;
    if (!(sc.mu >= 0.0) || std::isnan(sc.mu)) return APIC_E_INVALID;
    if (sc.n_iter < 0 || sc.n_iter > 64) return APIC_E_INVALID;
    if (sc.n_bodies < 1 || sc.n_bodies > 65536) return APIC_E_INVALID;
    bodies += sc.n_bodies;
  }
  if (expect != n_total) return APIC_E_INVALID;
  if (bodies > ((int64_t)1 << 30)) return APIC_E_INVALID;
  return APIC_OK;
}

// ---------------------------------------------------------------------------
// the layout phase (cells, boxes, keys, sort) shared by every entry point
// ---------------------------------------------------------------------------
template <typename T>
apic_status layout_phase(apic_ctx *ctx, hipStream_t st, const apic_scene *scenes, int32_t ns,
                         int64_t n, const T *x, const uint16_t *body, LayoutResult *out) {
  Workspace &W = ctx->ws;
  std::vector<SceneDev> sd(ns);
  int64_t nb_cap = 0;
  int32_t kmax = 0;
  for (int32_t s = 0; s < ns; ++s) {
    SceneDev d{};
    for (int k = 0; k < 3; ++k) {
      d.origin[k] = scenes[s].grid.origin[k];
      d.dims[k] = scenes[s].grid.dims[k];
    }
    d.h = scenes[s].grid.h;
    d.mu = scenes[s].mu;
    d.offset = scenes[s].offset;
    d.count = scenes[s].count;
    d.n_iter = scenes[s].n_iter;
    d.body_base = (int32_t)nb_cap;
    d.n_bodies = scenes[s].n_bodies;
    nb_cap += scenes[s].n_bodies;
    kmax = std::max(kmax, scenes[s].n_iter);
    sd[s] = d;
  }
  out->nb_cap = nb_cap;
  out->max_iter = kmax;
  TRY(W.ensure(kScenes, sizeof(SceneDev) * ns));
  TRY(W.ensure(kSceneAcc, sizeof(SceneAcc) * ns));
  TRY(W.ensure(kSceneLay, sizeof(SceneLay) * ns));
  TRY(W.ensure(kBodyAcc, sizeof(BodyAcc) * nb_cap));
  TRY(W.ensure(kBodyLay, sizeof(BodyLay) * nb_cap));
  TRY(W.ensure(kCounters, sizeof(Counters)));
  TRY(W.ensure(kTot, sizeof(int64_t) * 16));
  TRY(ctx->host_stage(std::max(sizeof(SceneDev) * ns, sizeof(Counters))));
  std::memcpy(ctx->stage, sd.data(), sizeof(SceneDev) * ns);
  HIPOK(hipMemcpyAsync(W.ptr[kScenes], ctx->stage, sizeof(SceneDev) * ns, hipMemcpyHostToDevice,
                       st));
  SceneDev *dsc = (SceneDev *)W.ptr[kScenes];
  SceneAcc *sacc = (SceneAcc *)W.ptr[kSceneAcc];
  BodyAcc *bacc = (BodyAcc *)W.ptr[kBodyAcc];
  Counters *cnt = (Counters *)W.ptr[kCounters];
  launch_layout_init(sacc, ns, bacc, (int)nb_cap, cnt, st);
  launch_cells<T>(x, body, n, dsc, ns, sacc, bacc, cnt, st);
  launch_domains(dsc, ns, sacc, bacc, (SceneLay *)W.ptr[kSceneLay], (BodyLay *)W.ptr[kBodyLay],
                 cnt, st);
  HIPOK(hipMemcpyAsync(ctx->stage, cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  Counters c;
  std::memcpy(&c, ctx->stage, sizeof(Counters));
  TRY(status_from_err(c.err));
  out->key_blocks = c.key_blocks;
  out->smap_total = c.smap_total;
  out->bmap_total = c.bmap_total;
  // keys and sort
  const int64_t ntiles = sort_tiles(n);
  TRY(W.ensure(kKeysA, sizeof(uint32_t) * n));
  TRY(W.ensure(kValsA, sizeof(uint32_t) * n));
  TRY(W.ensure(kKeysB, sizeof(uint32_t) * n));
  TRY(W.ensure(kValsB, sizeof(uint32_t) * n));
  TRY(W.ensure(kHist, sizeof(uint32_t) * 256 * std::max<int64_t>(ntiles, 1)));
  int64_t pcap = std::max(scan_partials_needed(256 * std::max<int64_t>(ntiles, 1)),
                          scan_partials_needed(std::max<int64_t>(
                              {n * 2, out->smap_total, out->bmap_total, (int64_t)1})));
  TRY(W.ensure(kPartial, sizeof(int32_t) * pcap));
  launch_keys<T>(x, body, n, dsc, ns, (const BodyLay *)W.ptr[kBodyLay], (uint32_t *)W.ptr[kKeysA],
                 st);
  int64_t key_space = (int64_t)std::max(out->key_blocks, 1) * 64;
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) < key_space) ++bits;
  out->sort_bits = bits;
  int where = 0;
  if (n > 0)
    where = radix_sort((uint32_t *)W.ptr[kKeysA], (uint32_t *)W.ptr[kValsA],
                       (uint32_t *)W.ptr[kKeysB], (uint32_t *)W.ptr[kValsB], n, bits,
                       (uint32_t *)W.ptr[kHist], (int32_t *)W.ptr[kPartial],
                       (int64_t *)W.ptr[kTot] + 9, st);
  out->keys = (uint32_t *)W.ptr[where ? kKeysB : kKeysA];
  out->perm = (uint32_t *)W.ptr[where ? kValsB : kValsA];
  return APIC_OK;
}

// ---------------------------------------------------------------------------
// the stateless contact step
// ---------------------------------------------------------------------------
template <typename T>
apic_status step_impl(apic_ctx *ctx, hipStream_t st, const apic_scene *scenes, int32_t ns,
                      int64_t n, const T *x, T *v, T *C, const T *m, const uint16_t *body,
                      apic_report *reports) {
  Workspace &W = ctx->ws;
  LayoutResult L;
  TRY(layout_phase<T>(ctx, st, scenes, ns, n, x, body, &L));
  if (n == 0) {
    if (reports)
      for (int s = 0; s < ns; ++s) std::memset(&reports[s], 0, sizeof(apic_report));
    return APIC_OK;
  }
  SceneDev *dsc = (SceneDev *)W.ptr[kScenes];
  Counters *cnt = (Counters *)W.ptr[kCounters];
  int64_t *tot = (int64_t *)W.ptr[kTot];
  // sorted particle state
  TRY(W.ensure(kT, sizeof(T) * 3 * n));
  TRY(W.ensure(kVbar, sizeof(T) * 12 * n));
  TRY(W.ensure(kMs, sizeof(T) * n));
  TRY(W.ensure(kSbody, sizeof(int32_t) * n));
  TRY(W.ensure(kNrm, sizeof(T) * 3 * n));
  TRY(W.ensure(kY, sizeof(T) * 12 * n));
  TRY(W.ensure(kRedBuf, sizeof(double) * kRed * 2 * ns));
  double *red = (double *)W.ptr[kRedBuf];
  fill_bytes_zero(red, sizeof(double) * kRed * 2 * ns, st);
  launch_gather<T>(L.perm, n, x, v, C, m, body, dsc, ns, (T *)W.ptr[kT], (T *)W.ptr[kVbar],
                   (T *)W.ptr[kMs], (int32_t *)W.ptr[kSbody], nullptr, nullptr, red, st);
  // segments, items, maps
  const int64_t seg_cap = n;
  const int64_t item_cap = n + n / kItem + 1;
  TRY(W.ensure(kSeg, sizeof(Segment) * seg_cap));
  TRY(W.ensure(kSegTmp, sizeof(int32_t) * (seg_cap + 1)));
  TRY(W.ensure(kFlags, sizeof(int32_t) * n));
  TRY(W.ensure(kItems, sizeof(Item) * item_cap));
  const int64_t smap_cap = std::max<int64_t>(L.smap_total, 1);
  const int64_t bmap_cap = std::max<int64_t>(L.bmap_total, 1);
  TRY(W.ensure(kSmap, sizeof(int32_t) * smap_cap));
  TRY(W.ensure(kBmap, sizeof(int32_t) * bmap_cap));
  const int64_t sblk_cap = std::max<int64_t>(1, std::min<int64_t>(L.smap_total, 8 * n));
  const int64_t bblk_cap = std::max<int64_t>(1, std::min<int64_t>(L.bmap_total, 8 * n));
  TRY(W.ensure(kGMass, sizeof(T) * kNodesPerBlock * sblk_cap));
  TRY(W.ensure(kGBuf0, sizeof(T) * 3 * kNodesPerBlock * sblk_cap));
  TRY(W.ensure(kGBuf1, sizeof(T) * 3 * kNodesPerBlock * sblk_cap));
  TRY(W.ensure(kBMass, sizeof(double) * kNodesPerBlock * bblk_cap));
  Segment *seg = (Segment *)W.ptr[kSeg];
  Item *items = (Item *)W.ptr[kItems];
  int32_t *partial = (int32_t *)W.ptr[kPartial];
  launch_segments(L.keys, n, (int32_t *)W.ptr[kFlags], partial, tot,
                  (const int32_t *)W.ptr[kSbody], (const BodyLay *)W.ptr[kBodyLay], seg, seg_cap,
                  items, item_cap, (int32_t *)W.ptr[kSegTmp], cnt, st);
  launch_maps(seg, seg_cap, (const SceneLay *)W.ptr[kSceneLay], (const BodyLay *)W.ptr[kBodyLay],
              (int32_t *)W.ptr[kSmap], smap_cap, (int32_t *)W.ptr[kBmap], bmap_cap, partial, tot,
              cnt, sblk_cap, bblk_cap, st);
  // transfers
  GridPtrs g;
  g.mass = W.ptr[kGMass];
  g.buf[0] = W.ptr[kGBuf0];
  g.buf[1] = W.ptr[kGBuf1];
  g.bmass = (double *)W.ptr[kBMass];
  fill_zero_f(g.mass, sblk_cap, &cnt->n_sblocks, kNodesPerBlock, sizeof(T), st);
  fill_zero_f(g.buf[0], sblk_cap, &cnt->n_sblocks, 3 * kNodesPerBlock, sizeof(T), st);
  fill_zero_f(g.bmass, bblk_cap, &cnt->n_bblocks, kNodesPerBlock, sizeof(double), st);
  StepArgs a;
  a.sc = dsc;
  a.seg = seg;
  a.items = items;
  a.cnt = cnt;
  a.keys = L.keys;
  a.n = n;
  a.grid_wg = (int)std::max<int64_t>(1, std::min<int64_t>(ctx->persistent_wg, (n + 63) / 64 * 2));
  const T *t = (const T *)W.ptr[kT];
  const T *ms = (const T *)W.ptr[kMs];
  const T *vbar = (const T *)W.ptr[kVbar];
  T *nrm = (T *)W.ptr[kNrm];
  T *Y = (T *)W.ptr[kY];
  launch_p2g0<T>(a, t, ms, vbar, g, st);
  launch_gridvel<T>(a, g, 0, st);
  int cur = 0;
  for (int k = 1; k <= L.max_iter; ++k) {
    launch_iter<T>(a, k, t, ms, vbar, nrm, Y, g, cur, L.perm, v, C, nullptr, 0.0,
                   red + kRed * ns, st);
    launch_gridvel<T>(a, g, 1 - cur, st);
    cur = 1 - cur;
  }
  launch_iter<T>(a, L.max_iter + 1, t, ms, vbar, nrm, Y, g, cur, L.perm, v, C, nullptr, 0.0,
                 red + kRed * ns, st);
  // results
  const size_t rbytes = sizeof(double) * kRed * 2 * ns;
  TRY(ctx->host_stage(rbytes + sizeof(Counters)));
  HIPOK(hipMemcpyAsync(ctx->stage, red, rbytes, hipMemcpyDeviceToHost, st));
  HIPOK(hipMemcpyAsync((char *)ctx->stage + rbytes, cnt, sizeof(Counters), hipMemcpyDeviceToHost,
                       st));
  HIPOK(hipStreamSynchronize(st));
  Counters c;
  std::memcpy(&c, (char *)ctx->stage + rbytes, sizeof(Counters));
  TRY(status_from_err(c.err));
  ctx->last_sblocks = c.n_sblocks;
  if (reports) {
    const double *r = (const double *)ctx->stage;
    for (int s = 0; s < ns; ++s) {
      apic_report &R = reports[s];
      const double *b = r + kRed * s, *af = r + kRed * (ns + s);
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
      R.n_particles = (int64_t)llround(b[9]);
      R.n_unconstrained = (int64_t)llround(af[10]);
      R.grid_blocks = c.n_sblocks;
    }
  }
  return APIC_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

apic_status apic_create(apic_ctx **out, int device, size_t hbm_budget_bytes) {
  if (!out) return APIC_E_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return APIC_E_DEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    return APIC_E_DEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    (void)hipGetLastError();
    return APIC_E_DEVICE;
  }
  apic_ctx *c = new apic_ctx();
  c->device = device;
  c->ws.budget = hbm_budget_bytes;
  c->cus = prop.multiProcessorCount;
  c->persistent_wg = std::max(1, prop.multiProcessorCount) * 8;
  *out = c;
  return APIC_OK;
}

void apic_destroy(apic_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->ws.release();
  if (ctx->stage) (void)hipHostFree(ctx->stage);
  delete ctx;
}

const char *apic_status_string(apic_status s) {
  switch (s) {
    case APIC_OK: return "ok";
    case APIC_E_INVALID: return "invalid argument";
    case APIC_E_NOMEM: return "device allocation failed";
    case APIC_E_OUT_OF_GRID: return "particle stencil outside the grid";
    case APIC_E_DEVICE: return "HIP runtime error";
    case APIC_E_BUDGET: return "HBM budget exceeded";
    case APIC_E_KEY_OVERFLOW: return "cell-key space overflow";
    case APIC_E_BODY: return "body id out of range";
  }
  return "unknown status";
}

apic_status apic_contact_step_batched(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                                      int32_t n_scenes, int64_t n_total, const void *x, void *v,
                                      void *C, const void *m, const uint16_t *body_id,
                                      apic_precision prec, apic_report *per_scene) {
  if (!ctx) return APIC_E_INVALID;
  TRY(validate_scenes(scenes, n_scenes, n_total));
  if (n_total > 0 && (!x || !v || !C || !m || !body_id)) return APIC_E_INVALID;
  if (prec != APIC_FP64 && prec != APIC_FP32_MIXED) return APIC_E_INVALID;
  if (hipSetDevice(ctx->device) != hipSuccess) return APIC_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (prec == APIC_FP64)
    return step_impl<double>(ctx, st, scenes, n_scenes, n_total, (const double *)x, (double *)v,
                             (double *)C, (const double *)m, body_id, per_scene);
  return step_impl<float>(ctx, st, scenes, n_scenes, n_total, (const float *)x, (float *)v,
                          (float *)C, (const float *)m, body_id, per_scene);
}

apic_status apic_contact_step(apic_ctx *ctx, void *stream, const apic_grid *grid, int64_t n,
                              const void *x, void *v, void *C, const void *m,
                              const uint16_t *body_id, double mu, int32_t n_iter,
                              apic_precision prec, apic_report *report) {
  if (!ctx || !grid) return APIC_E_INVALID;
  apic_scene s;
  s.offset = 0;
  s.count = n;
  s.grid = *grid;
  s.mu = mu;
  s.n_iter = n_iter;
  s.n_bodies = 65536;
  return apic_contact_step_batched(ctx, stream, &s, 1, n, x, v, C, m, body_id, prec, report);
}

apic_status apic_sort_keys(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                           int32_t n_scenes, int64_t n_total, const void *x,
                           const uint16_t *body_id, apic_precision prec, uint32_t *keys_sorted,
                           uint32_t *perm) {
  if (!ctx) return APIC_E_INVALID;
  TRY(validate_scenes(scenes, n_scenes, n_total));
  if (n_total > 0 && (!x || !body_id || !keys_sorted || !perm)) return APIC_E_INVALID;
  if (prec != APIC_FP64 && prec != APIC_FP32_MIXED) return APIC_E_INVALID;
  if (hipSetDevice(ctx->device) != hipSuccess) return APIC_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  LayoutResult L;
  if (prec == APIC_FP64)
    TRY(layout_phase<double>(ctx, st, scenes, n_scenes, n_total, (const double *)x, body_id, &L));
  else
    TRY(layout_phase<float>(ctx, st, scenes, n_scenes, n_total, (const float *)x, body_id, &L));
  if (n_total > 0) {
    HIPOK(hipMemcpyAsync(keys_sorted, L.keys, sizeof(uint32_t) * n_total,
                         hipMemcpyDeviceToDevice, st));
    HIPOK(hipMemcpyAsync(perm, L.perm, sizeof(uint32_t) * n_total, hipMemcpyDeviceToDevice, st));
  }
  HIPOK(hipStreamSynchronize(st));
  return APIC_OK;
}

int64_t apic_scene_footprint(int64_t n, int64_t blocks_hint, apic_precision prec) {
  if (n < 0) return -1;
  const int64_t tb = prec == APIC_FP64 ? 8 : 4;
  if (blocks_hint <= 0) blocks_hint = n / 16 + 64;  // about 1.3 node blocks per 64 particles x 8
  // particle state (input copies, sorted copies, series, normals) + sort + tables
  int64_t per_particle = tb * (3 + 12 + 1 + 3 + 12 + 3 + 12 + 3) + 4 * 8 + sizeof(Segment) +
                         sizeof(Item) * 2;
  int64_t per_block = kNodesPerBlock * (tb * 7 + 8) + 8 * 2;
  return n * per_particle + blocks_hint * per_block + (1 << 20);
}

}  // extern "C"
