// api.hip -- context, plans, the stateless contact step and the resident
// (graph-capturable) driver behind the C ABI of include/apic_contact.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
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
  if (arena) {  // carve: each buffer once per call, 256-byte aligned
    if (size[id] >= bytes) return APIC_OK;
    if (bytes > arena_size - held) return APIC_E_SCRATCH;
    ptr[id] = arena + held;
    size[id] = bytes;
    held += bytes;
    fresh[id] = true;
    return APIC_OK;
  }
  if (size[id] >= bytes) return APIC_OK;
  // a growing workspace rounds up by `slack` (within the budget), so that a
  // slowly growing batch reallocates a logarithmic number of times
  if (slack > 1.0) {
    const size_t want = ((size_t)((double)bytes * slack) + 255) & ~(size_t)255;
    if (!budget || held - size[id] + want <= budget) bytes = want;
  }
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
  fresh[id] = true;
  return APIC_OK;
}

void Workspace::release() {
  if (arena) {  // nothing was allocated
    for (int i = 0; i < kNumBufs; ++i) ptr[i] = nullptr, size[i] = 0;
    held = 0;
    return;
  }
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

// ---------------------------------------------------------------------------
// launch tuning
// ---------------------------------------------------------------------------
static int size_bucket(int64_t n) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << (b + 1)) <= n) ++b;
  return b;
}

static apic_tuning default_tuning() {
  apic_tuning t;
  t.item_waves_per_cu = 32;
  t.node_wg_per_cu = 8;
  t.xcd_split = 0;
  t.p2g_group = 4;
  t.p2g_pairs = 0;
  return t;
}

static bool tuning_ok(const apic_tuning &t) {
  return t.item_waves_per_cu >= 1 && t.item_waves_per_cu <= 64 && t.node_wg_per_cu >= 1 &&
         t.node_wg_per_cu <= 64 && (t.xcd_split == 0 || t.xcd_split == 1) &&
         (t.p2g_group == 1 || t.p2g_group == 4 || t.p2g_group == 8) &&
         (t.p2g_pairs == 0 || t.p2g_pairs == 1);
}

apic_tuning apic_ctx::tuning_for(apic_precision prec, int64_t n) const {
  auto it = tuning.find({(int)prec, size_bucket(n)});
  return it == tuning.end() ? default_tuning() : it->second;
}

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
    if ((sc.flags & ~(APIC_PIC | APIC_RULE_SEPARATE)) != 0 || sc.reserved != 0)
      return APIC_E_INVALID;
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(sc.accel[d]) || !std::isfinite(sc.x_ref[d])) return APIC_E_INVALID;
    bodies += sc.n_bodies;
  }
  if (expect != n_total) return APIC_E_INVALID;
  if (bodies > ((int64_t)1 << 30)) return APIC_E_INVALID;
  return APIC_OK;
}

// ---------------------------------------------------------------------------
// plan: tables, capacities and buffer pointers of one step
// ---------------------------------------------------------------------------
static apic_status plan_tables(apic_ctx *ctx, Workspace &W, Plan &P, const apic_scene *scenes,
                               int32_t ns, int64_t n, apic_precision prec, const double *dt,
                               hipStream_t st) {
  P.prec = prec;
  P.tbytes = prec == APIC_FP64 ? 8 : 4;
  P.n = n;
  P.ns = ns;
  // arena mode (the allocation-free entry point, one scene): the table goes
  // to the device as a kernel argument, with no host buffer
  const bool arena = W.arena != nullptr;
  if (arena && ns != 1) return APIC_E_INVALID;
  SceneDev one{};
  std::vector<SceneDev> many;
  if (!arena) many.resize(ns);
  SceneDev *sd = arena ? &one : many.data();
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
    d.dt = dt ? dt[s] : 0.0;
    for (int k = 0; k < 3; ++k) {
      d.accel[k] = scenes[s].accel[k];
      d.x_ref[k] = scenes[s].x_ref[k];
    }
    d.flags = scenes[s].flags;
    if (d.flags) P.variants = true;
    d.offset = scenes[s].offset;
    d.count = scenes[s].count;
    d.n_iter = scenes[s].n_iter;
    d.body_base = (int32_t)nb_cap;
    d.n_bodies = scenes[s].n_bodies;
    nb_cap += scenes[s].n_bodies;
    kmax = std::max(kmax, scenes[s].n_iter);
    sd[s] = d;
  }
  P.nb_cap = nb_cap;
  P.max_iter = kmax;
  TRY(W.ensure(kScenes, sizeof(SceneDev) * ns));
  TRY(W.ensure(kSceneAcc, sizeof(SceneAcc) * ns));
  TRY(W.ensure(kSceneLay, sizeof(SceneLay) * ns));
  TRY(W.ensure(kBodyAcc, sizeof(BodyAcc) * nb_cap));
  TRY(W.ensure(kBodyLay, sizeof(BodyLay) * nb_cap));
  TRY(W.ensure(kCounters, sizeof(Counters)));
  TRY(W.ensure(kTot, sizeof(int64_t) * 16));
  TRY(W.ensure(kRedBuf, sizeof(double) * kRed * 2 * ns));
  TRY(W.ensure(kBoxRec, sizeof(BoxRec) * std::max<int64_t>(wave_records(n), 1)));
  TRY(W.ensure(kSceneErr, sizeof(int32_t) * ns));
  P.scene_err = (int32_t *)W.ptr[kSceneErr];
  P.box_rec = (BoxRec *)W.ptr[kBoxRec];
  P.sc = (SceneDev *)W.ptr[kScenes];
  P.sacc = (SceneAcc *)W.ptr[kSceneAcc];
  P.slay = (SceneLay *)W.ptr[kSceneLay];
  P.bacc = (BodyAcc *)W.ptr[kBodyAcc];
  P.blay = (BodyLay *)W.ptr[kBodyLay];
  P.cnt = (Counters *)W.ptr[kCounters];
  P.tot = (int64_t *)W.ptr[kTot];
  P.red = (double *)W.ptr[kRedBuf];
  if (arena) {
    launch_store_scene(P.sc, one, st);
    return APIC_OK;
  }
  TRY(ctx->host_stage(sizeof(SceneDev) * ns));
  std::memcpy(ctx->stage, sd, sizeof(SceneDev) * ns);
  HIPOK(hipMemcpyAsync(P.sc, ctx->stage, sizeof(SceneDev) * ns, hipMemcpyHostToDevice, st));
  HIPOK(hipStreamSynchronize(st));  // the staging buffer is reused right after
  return APIC_OK;
}

// Device-to-host copy of a few bytes, completed on return: through the
// context's pinned staging buffer, or (arena mode, which allocates nothing)
// straight into the caller's host memory.
static apic_status read_back(apic_ctx *ctx, const Workspace &W, void *dst, const void *src,
                             size_t bytes, hipStream_t st) {
  if (W.arena) {
    HIPOK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    return APIC_OK;
  }
  TRY(ctx->host_stage(bytes));
  HIPOK(hipMemcpyAsync(ctx->stage, src, bytes, hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  std::memcpy(dst, ctx->stage, bytes);
  return APIC_OK;
}

// Capacities from the sizes of a measured layout (times `headroom`), then
// every buffer of the step.
static apic_status plan_buffers(apic_ctx *ctx, Workspace &W, Plan &P, int32_t key_blocks,
                                int64_t smap_total, int64_t bmap_total, double headroom,
                                hipStream_t st) {
  const int64_t n = P.n;
  // with headroom (a plan kept while particles move), also an absolute
  // margin, so that a small scene whose box grows by one block per side
  // does not outgrow its plan at once
  const int64_t kmargin = headroom > 1.0 ? 64 : 0, mmargin = headroom > 1.0 ? 512 : 0;
  int64_t kb = std::max<int64_t>(
      1, std::max<int64_t>((int64_t)std::ceil(key_blocks * headroom), key_blocks + kmargin));
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) < kb * 64) ++bits;
  P.sort_bits = bits;
  P.smap_cap = std::max<int64_t>(
      1, std::max<int64_t>((int64_t)std::ceil(smap_total * headroom), smap_total + mmargin));
  P.bmap_cap = std::max<int64_t>(
      1, std::max<int64_t>((int64_t)std::ceil(bmap_total * headroom), bmap_total + mmargin));
  // segments are distinct (body, block) keys present
  P.seg_cap = std::max<int64_t>(1, std::min<int64_t>(n, kb));
  // items: one per segment plus one per 64 particles, plus the run padding
  // (fewer than the group size per run, one run per super block of a body,
  // and a body's super blocks number 8 block keys each); segments are
  // distinct (body, block) keys, so at most min(n, key blocks)
  P.item_cap = std::min<int64_t>(n, kb) + n / kItem + 1 + kb;
  P.sblk_cap = std::max<int64_t>(1, std::min<int64_t>(P.smap_cap, 8 * n));
  P.bblk_cap = std::max<int64_t>(1, std::min<int64_t>(P.bmap_cap, 8 * n));
  const apic_tuning tu = ctx->tuning_for(P.prec, n);
  {
    // particle kernels: a multiple of 8 workgroups (one share per XCD), never
    // more than twice the items a dense layout has; grouped kernels run
    // `group` waves per workgroup (FP64 at most 4: LDS)
    const int64_t cus = std::max(1, ctx->cus);
    const int grp = (P.prec == APIC_FP64) ? std::min(tu.p2g_group, 4) : tu.p2g_group;
    const int64_t dense_items = (n + 63) / 64 * 2;
    auto round8 = [](int64_t v) { return std::max<int64_t>(8, (v + 7) / 8 * 8); };
    P.item_wg = (int)round8(std::min<int64_t>(cus * tu.item_waves_per_cu, dense_items));
    P.grid_wg = (int)round8(std::min<int64_t>(cus * tu.item_waves_per_cu / grp,
                                              (dense_items + grp - 1) / grp));
    int64_t gn = cus * tu.node_wg_per_cu;
    gn = std::min<int64_t>(gn, (P.sblk_cap * kNodesPerBlock + 255) / 256);
    P.node_wg = (int)std::max<int64_t>(1, gn);
    P.xcd_split = tu.xcd_split;
    P.group = grp;
    P.pairs = P.prec == APIC_FP32_MIXED ? tu.p2g_pairs : 0;
  }
  const int64_t ntiles = std::max<int64_t>(sort_tiles(n), 1);
  const size_t T = P.tbytes;
  TRY(W.ensure(kKeysA, sizeof(uint32_t) * n));
  TRY(W.ensure(kValsA, sizeof(uint32_t) * n));
  TRY(W.ensure(kKeysB, sizeof(uint32_t) * n));
  TRY(W.ensure(kValsB, sizeof(uint32_t) * n));
  TRY(W.ensure(kGhist, sizeof(uint32_t) * radix_hist_words(n)));
  const int64_t lbcap = std::max<int64_t>(
      {scan_tile_count(std::max<int64_t>({n, 256 * ntiles})),
       scan_tile_count(P.smap_cap) + scan_tile_count(P.bmap_cap), scan_tile_count(P.seg_cap, 1)});
  TRY(W.ensure(kLbFlags, sizeof(uint64_t) * lbcap));
  TRY(W.ensure(kLbState, sizeof(uint32_t) * 2));
  TRY(W.ensure(kT, T * 3 * n));
  TRY(W.ensure(kMs, T * n));
  TRY(W.ensure(kSbody, sizeof(int32_t) * n));
  TRY(W.ensure(kNrm, T * 3 * n));
  TRY(W.ensure(kY, T * 12 * n));
  TRY(W.ensure(kSeg, sizeof(Segment) * P.seg_cap));
  TRY(W.ensure(kItems, sizeof(Item) * P.item_cap));
  TRY(W.ensure(kSmark, sizeof(int32_t) * P.smap_cap));
  TRY(W.ensure(kSmap, sizeof(int32_t) * P.smap_cap));
  TRY(W.ensure(kBmark, sizeof(int32_t) * P.bmap_cap));
  TRY(W.ensure(kBmap, sizeof(int32_t) * P.bmap_cap));
  TRY(W.ensure(kGMass, T * kNodesPerBlock * P.sblk_cap));
  TRY(W.ensure(kGBuf0, T * 3 * kNodesPerBlock * P.sblk_cap));
  TRY(W.ensure(kGBuf1, T * 3 * kNodesPerBlock * P.sblk_cap));
  TRY(W.ensure(kGBuf2, T * 3 * kNodesPerBlock * P.sblk_cap));
  TRY(W.ensure(kInvM, sizeof(double) * kNodesPerBlock * P.sblk_cap));
  TRY(W.ensure(kBMass, T * kNodesPerBlock * P.bblk_cap));
  TRY(W.ensure(kRecGather, sizeof(RedRec) * std::max<int64_t>(wave_records(n), 1)));
  TRY(W.ensure(kRecItems, sizeof(RedRec) * P.item_cap));  // one per work item
  TRY(W.ensure(kB2S, sizeof(int32_t) * P.bblk_cap));
  TRY(W.ensure(kNodeCount, sizeof(int32_t) * kNodesPerBlock * P.sblk_cap));
  TRY(W.ensure(kBodyMax, sizeof(int32_t) * P.ns));
  P.b2s = (int32_t *)W.ptr[kB2S];
  P.node_count = (int32_t *)W.ptr[kNodeCount];
  P.body_max = (int32_t *)W.ptr[kBodyMax];
  P.rec_gather = (RedRec *)W.ptr[kRecGather];
  P.rec_items = (RedRec *)W.ptr[kRecItems];
  P.ka = (uint32_t *)W.ptr[kKeysA];
  P.va = (uint32_t *)W.ptr[kValsA];
  P.kb = (uint32_t *)W.ptr[kKeysB];
  P.vb = (uint32_t *)W.ptr[kValsB];
  P.ghist = (uint32_t *)W.ptr[kGhist];
  P.lb.flags = (uint64_t *)W.ptr[kLbFlags];
  P.lb.capacity = (int64_t)(W.size[kLbFlags] / sizeof(uint64_t));
  P.lb.state = (uint32_t *)W.ptr[kLbState];
  P.smark = (int32_t *)W.ptr[kSmark];
  P.bmark = (int32_t *)W.ptr[kBmark];
  P.t = W.ptr[kT];
  P.ms = W.ptr[kMs];
  P.sbody = (int32_t *)W.ptr[kSbody];
  P.nrm = W.ptr[kNrm];
  P.Y = W.ptr[kY];
  P.seg = (Segment *)W.ptr[kSeg];
  P.items = (Item *)W.ptr[kItems];
  P.smap = (int32_t *)W.ptr[kSmap];
  P.bmap = (int32_t *)W.ptr[kBmap];
  P.g.mass = W.ptr[kGMass];
  P.g.buf[0] = W.ptr[kGBuf0];
  P.g.buf[1] = W.ptr[kGBuf1];
  P.g.buf[2] = W.ptr[kGBuf2];
  P.g.invm = (double *)W.ptr[kInvM];
  P.g.bmass = W.ptr[kBMass];
  // state that kernels keep between launches starts from zero (mark arrays)
  // or a fresh look-back epoch whenever its buffer is new
  if (W.fresh[kLbFlags] || W.fresh[kLbState]) lookback_init(P.lb, st);
  // (the whole allocation: a later plan may use more of it without growing it)
  if (W.fresh[kSmark]) fill_bytes_zero(P.smark, (int64_t)W.size[kSmark], st);
  if (W.fresh[kBmark]) fill_bytes_zero(P.bmark, (int64_t)W.size[kBmark], st);
  W.fresh[kLbFlags] = W.fresh[kLbState] = false;
  W.fresh[kSmark] = W.fresh[kBmark] = false;
  P.ready = true;
  return APIC_OK;
}

// ---------------------------------------------------------------------------
// enqueue helpers (no host synchronisation inside)
// ---------------------------------------------------------------------------
// table_in (device, ABI layout) and plan_sc: a planned step's scene table,
// checked against the plan's and converted into P.sc before the layout.
template <typename T>
static void enqueue_prefix(Plan &P, hipStream_t st, const T *x, const uint16_t *body,
                           const int32_t *sticky, bool check_caps,
                           const apic_scene *table_in = nullptr,
                           const SceneDev *plan_sc = nullptr) {
  launch_layout_init(P.sacc, P.ns, P.bacc, (int)P.nb_cap, P.cnt, sticky, P.red,
                     (int64_t)kRed * 2 * P.ns, P.scene_err, st);
  if (table_in) launch_scene_table(table_in, plan_sc, P.ns, P.max_iter, P.sc, P.cnt, st);
  launch_cells<T>(x, body, P.n, P.sc, P.ns, P.bacc, P.box_rec, P.cnt, P.scene_err, st);
  launch_reduce_box(P.box_rec, wave_records(P.n), P.bacc, P.cnt, st);
  launch_domains(P.sc, P.ns, (int)P.nb_cap, P.sacc, P.bacc, P.slay, P.blay, P.cnt,
                 check_caps ? P.sort_bits : 0, check_caps ? P.smap_cap : 0,
                 check_caps ? P.bmap_cap : 0, st);
}

// keys + sort; sets P.keys / P.perm.  The contact step needs particles
// grouped by (scene, body, block) only -- the per-cell pass ranking works in
// any order within a block -- so it sorts by the block part of the key
// (bits 6 and up) and keeps input order within a block (the gather then
// orders each wave's particles by cell, which costs no pass over memory);
// full_key sorts by the whole key (the ordering apic_sort_keys returns).
template <typename T>
static void enqueue_sort(Plan &P, hipStream_t st, const T *x, const uint16_t *body,
                         Profiler *prof, bool full_key = false) {
  const int lo = full_key ? 0 : 6;
  launch_keys<T>(x, body, P.n, P.sc, P.ns, P.blay, P.ka, lo, P.ghist, st);
  if (prof) prof->end(APIC_KC_LAYOUT, st), prof->begin(st);
  int where = radix_sort(P.ka, P.va, P.kb, P.vb, P.n, lo, P.sort_bits, P.ghist, P.lb, true, st);
  if (prof) prof->end(APIC_KC_SORT, st);
  P.keys = where ? P.kb : P.ka;
  P.perm = where ? P.vb : P.va;
}

// Everything after the sort.  Source arrays are read through P.perm; outputs
// go to (v_out, C_out) at perm positions (stateless) or in place in sorted
// order with drift (resident, perm_out = false).
template <typename T>
static void enqueue_body(Plan &P, hipStream_t st, const T *x, const T *v, const T *C, const T *m,
                         const uint16_t *body, T *vbar, T *x_sorted, uint16_t *body_sorted,
                         T *m_sorted, const uint32_t *orig_in, uint32_t *orig_out,
                         T *v_out, T *C_out, bool unpermute, Profiler *prof,
                         const T *normals = nullptr) {
  const int64_t n = P.n;
  if (prof) prof->begin(st);
  // the gather also orders each wave's particles by cell within a block, and
  // writes that order's keys and permutation into the sort's free buffers
  uint32_t *keys2 = P.keys == P.ka ? P.kb : P.ka;
  uint32_t *perm2 = P.perm == P.va ? P.vb : P.va;
  launch_gather<T>(P.perm, P.keys, n, x, v, C, m, body, P.sc, P.ns, (T *)P.t, vbar, m_sorted,
                   P.sbody, x_sorted, body_sorted, orig_in, orig_out, keys2, perm2, P.rec_gather,
                   P.red, normals, (T *)P.nrm, P.cnt, P.scene_err, st);
  P.keys = keys2;
  P.perm = perm2;
  if (prof) prof->end(APIC_KC_GATHER, st), prof->begin(st);
  launch_segments(P.keys, n, P.lb, P.tot, P.sbody, P.blay, P.slay, P.seg, P.seg_cap, P.items,
                  P.item_cap, P.smark, P.smap_cap, P.bmark, P.bmap_cap, P.group, P.cnt, st);
  launch_maps(P.seg, P.seg_cap, P.slay, P.blay, P.smark, P.smap, P.smap_cap, P.bmark, P.bmap,
              P.bmap_cap, P.lb, P.tot, P.cnt, P.sblk_cap, P.bblk_cap, P.item_cap, P.g,
              (int)P.tbytes, P.node_wg, P.rec_gather, wave_records(n), P.red, P.b2s, st);
  StepArgs a;
  a.sc = P.sc;
  a.seg = P.seg;
  a.items = P.items;
  a.cnt = P.cnt;
  a.keys = P.keys;
  a.n = n;
  a.grid_wg = P.grid_wg;
  a.node_wg = P.node_wg;
  a.xcd_split = P.xcd_split;
  a.item_wg = P.item_wg;
  a.group = P.group;
  a.given_normals = normals != nullptr ? 1 : 0;
  a.variants = P.variants ? 1 : 0;
  a.pairs = P.pairs;
  if (prof) prof->end(APIC_KC_SEGMENTS, st), prof->begin(st);
  const T *t = (const T *)P.t;
  T *nrm = (T *)P.nrm, *Y = (T *)P.Y;
  launch_mass<T>(a, t, m_sorted, P.g, st);
  if (prof) prof->end(APIC_KC_MASS, st), prof->begin(st);
  launch_p2g0<T>(a, t, m_sorted, vbar, nrm, P.items, P.g, st);
  if (prof) prof->end(APIC_KC_P2G0, st);
  const uint32_t *perm_out = unpermute ? P.perm : nullptr;
  for (int k = 1; k <= P.max_iter; ++k) {
    if (prof) prof->begin(st);
    launch_round<T>(a, k, t, m_sorted, vbar, nrm, Y, P.g, perm_out, v_out, C_out, st);
    if (prof) prof->end(k == 1 ? APIC_KC_ROUND1 : APIC_KC_ROUND, st);
  }
  // the last round also takes the FP64 momentum after the step and, for the
  // resident driver, the drift (positions at the output index)
  if (prof) prof->begin(st);
  T *x_after = unpermute ? (T *)x : x_sorted;
  launch_final<T>(a, P.max_iter + 1, t, m_sorted, vbar, nrm, Y, P.g, perm_out, v_out, C_out,
                  x_after, unpermute ? 0 : 1, P.rec_items, st);
  if (prof) prof->end(APIC_KC_FINAL, st), prof->begin(st);
  launch_reduce_red(P.rec_items, P.item_cap, &P.cnt->n_items, P.cnt, P.red + kRed * P.ns, st);
  if (prof) prof->end(APIC_KC_AFTER, st);
}

static void fill_report(const double *r, int ns, const Counters &c, apic_report *reports,
                        const int32_t *body_max = nullptr) {
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
    R.max_bodies_per_node = body_max ? body_max[s] : 0;
    R.reserved = 0;
  }
}

template <typename T>
static void enqueue_bodies_per_node(const Plan &P, hipStream_t st) {
  launch_bodies_per_node<T>(P.cnt, P.seg, P.seg_cap, (const T *)P.g.bmass, P.b2s, P.bblk_cap,
                            P.sblk_cap, P.node_count, P.body_max, P.ns, st);
}

// ---------------------------------------------------------------------------
// the stateless contact step
// ---------------------------------------------------------------------------
// The step on workspace W: the context's grow-only arena, or (arena mode)
// the allocation-free scratch region.  One readback measures the layout,
// then the step is enqueued and its status read back.
template <typename T>
static apic_status step_impl(apic_ctx *ctx, Workspace &W, hipStream_t st,
                             const apic_scene *scenes, int32_t ns, int64_t n, const T *x, T *v,
                             T *C, const T *m, const uint16_t *body, apic_report *reports,
                             const T *normals = nullptr) {
  Plan P;
  TRY(plan_tables(ctx, W, P, scenes, ns, n, sizeof(T) == 8 ? APIC_FP64 : APIC_FP32_MIXED,
                  nullptr, st));
  if (n == 0) {
    if (reports)
      for (int s = 0; s < ns; ++s) std::memset(&reports[s], 0, sizeof(apic_report));
    return APIC_OK;
  }
  enqueue_prefix<T>(P, st, x, body, nullptr, false);
  Counters c;
  TRY(read_back(ctx, W, &c, P.cnt, sizeof(Counters), st));
  TRY(status_from_err(c.err));
  TRY(plan_buffers(ctx, W, P, c.key_blocks, c.smap_total, c.bmap_total, 1.0, st));
  TRY(W.ensure(kVbar, sizeof(T) * 12 * n));
  enqueue_sort<T>(P, st, x, body, nullptr);
  enqueue_body<T>(P, st, x, v, C, m, body, (T *)W.ptr[kVbar], nullptr, nullptr, (T *)P.ms,
                  nullptr, nullptr, v, C, true, nullptr, normals);
  if (reports) enqueue_bodies_per_node<T>(P, st);
  if (W.arena) {  // one scene: the sums and counters on the stack
    double red[kRed * 2];
    int32_t bmax = 0;
    TRY(read_back(ctx, W, red, P.red, sizeof(red), st));
    TRY(read_back(ctx, W, &c, P.cnt, sizeof(Counters), st));
    if (reports) TRY(read_back(ctx, W, &bmax, P.body_max, sizeof(int32_t), st));
    TRY(status_from_err(c.err));
    if (c.err) return APIC_E_DEVICE;
    if (reports) fill_report(red, 1, c, reports, &bmax);
    return APIC_OK;
  }
  const size_t rbytes = sizeof(double) * kRed * 2 * ns;
  const size_t bbytes = reports ? sizeof(int32_t) * ns : 0;
  TRY(ctx->host_stage(rbytes + sizeof(Counters) + bbytes));
  char *stg = (char *)ctx->stage;
  HIPOK(hipMemcpyAsync(stg, P.red, rbytes, hipMemcpyDeviceToHost, st));
  HIPOK(hipMemcpyAsync(stg + rbytes, P.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
  if (bbytes)
    HIPOK(hipMemcpyAsync(stg + rbytes + sizeof(Counters), P.body_max, bbytes,
                         hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  std::memcpy(&c, stg + rbytes, sizeof(Counters));
  TRY(status_from_err(c.err));
  if (c.err) return APIC_E_DEVICE;
  if (reports) {
    std::vector<int32_t> bmax(ns);
    std::memcpy(bmax.data(), stg + rbytes + sizeof(Counters), bbytes);
    fill_report((const double *)stg, ns, c, reports, bmax.data());
  }
  return APIC_OK;
}

// ---------------------------------------------------------------------------
// profiler: an event pair per kernel launch of eager steps
// ---------------------------------------------------------------------------
namespace apic {
thread_local LaunchTimer *g_launch_timer = nullptr;
}

// A launch whose events cannot be created runs untimed (null events).
void Profiler::events(hipEvent_t *start, hipEvent_t *stop) {
  if (free_events.size() < 2)
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) == hipSuccess) free_events.push_back(e);
    }
  if (free_events.size() < 2) {
    (void)hipGetLastError();
    *start = *stop = nullptr;
    return;
  }
  *start = free_events.back();
  free_events.pop_back();
  *stop = free_events.back();
  free_events.pop_back();
  recs.push_back({-1, *start, *stop});
}

void Profiler::begin(hipStream_t) {
  if (!on) return;
  open_from = recs.size();
  g_launch_timer = this;
}

void Profiler::end(int kind, hipStream_t) {
  if (!on) return;
  for (size_t i = open_from; i < recs.size(); ++i) recs[i].kind = kind;
  g_launch_timer = nullptr;
  if (recs.size() > 8192) collect();
}

void Profiler::collect() {
  for (auto &r : recs) {
    (void)hipEventSynchronize(r.stop);
    float ms = 0.f;
    if (r.kind >= 0 && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      total_ms[r.kind] += ms;
      launches[r.kind] += 1;
    }
    free_events.push_back(r.start);
    free_events.push_back(r.stop);
  }
  recs.clear();
  open_from = 0;
}

void Profiler::release() {
  collect();
  for (auto e : free_events) (void)hipEventDestroy(e);
  free_events.clear();
}

// ---------------------------------------------------------------------------
// resident driver
// ---------------------------------------------------------------------------
template <typename T>
static void enqueue_sim_step(apic_sim *S, hipStream_t st, int parity, Profiler *prof) {
  Plan &P = S->plan;
  const int64_t n = P.n;
  SimState &A = S->state[parity], &B = S->state[1 - parity];
  if (prof) prof->begin(st);
  enqueue_prefix<T>(P, st, (const T *)A.x, A.body, &S->dev->sticky, true);
  enqueue_sort<T>(P, st, (const T *)A.x, A.body, prof);
  T *vc = (T *)B.vc;
  enqueue_body<T>(P, st, (const T *)A.x, (const T *)A.vc, (const T *)A.vc + 3 * n,
                  (const T *)A.m, A.body, vc, (T *)B.x, B.body, (T *)B.m, A.orig, B.orig, vc,
                  vc + 3 * n, false, prof);
  launch_step_end(P.cnt, P.red, P.ns, S->dev, S->drift, st);
}

static apic_status sim_capture(apic_sim *S, hipStream_t st);

template <typename T>
static apic_status sim_run(apic_sim *S, hipStream_t st, int32_t n_steps, int use_graph) {
  for (int32_t i = 0; i < n_steps; ++i) {
    if (use_graph && !S->prof.on) {
      if (!S->graph_ok) TRY(sim_capture(S, st));
      HIPOK(hipGraphLaunch(S->exec[S->parity], st));
    } else {
      enqueue_sim_step<T>(S, st, S->parity, S->prof.on ? &S->prof : nullptr);
    }
    S->parity ^= 1;
  }
  return APIC_OK;
}

static apic_status sim_capture(apic_sim *S, hipStream_t st) {
  for (int p = 0; p < 2; ++p) {
    if (S->exec[p]) {
      (void)hipGraphExecDestroy(S->exec[p]);
      S->exec[p] = nullptr;
    }
    hipGraph_t g = nullptr;
    HIPOK(hipStreamBeginCapture(S->capture_stream, hipStreamCaptureModeThreadLocal));
    if (S->plan.prec == APIC_FP64)
      enqueue_sim_step<double>(S, S->capture_stream, p, nullptr);
    else
      enqueue_sim_step<float>(S, S->capture_stream, p, nullptr);
    HIPOK(hipStreamEndCapture(S->capture_stream, &g));
    hipError_t e = hipGraphInstantiate(&S->exec[p], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return APIC_E_DEVICE;
    }
  }
  (void)st;
  S->graph_ok = true;
  return APIC_OK;
}

static apic_status sim_read_dev(apic_sim *S, hipStream_t st, SimDev *out) {
  TRY(S->ctx->host_stage(sizeof(SimDev)));
  HIPOK(hipMemcpyAsync(S->ctx->stage, S->dev, sizeof(SimDev), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  std::memcpy(out, S->ctx->stage, sizeof(SimDev));
  return APIC_OK;
}

// Measure the current layout, then size the plan with headroom.
template <typename T>
static apic_status sim_plan(apic_sim *S, hipStream_t st, double headroom) {
  Plan &P = S->plan;
  SimState &A = S->state[S->parity];
  enqueue_prefix<T>(P, st, (const T *)A.x, A.body, nullptr, false);
  Counters c;
  TRY(S->ctx->host_stage(sizeof(Counters)));
  HIPOK(hipMemcpyAsync(S->ctx->stage, P.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  std::memcpy(&c, S->ctx->stage, sizeof(Counters));
  TRY(status_from_err(c.err));
  TRY(plan_buffers(S->ctx, S->ws, P, c.key_blocks, c.smap_total, c.bmap_total, headroom, st));
  S->graph_ok = false;
  return APIC_OK;
}

static apic_status sim_step_impl(apic_sim *S, hipStream_t st, int32_t n_steps, int use_graph) {
  const bool f64 = S->plan.prec == APIC_FP64;
  int64_t target = S->steps_done + n_steps;
  for (int attempt = 0; attempt < 8; ++attempt) {
    int32_t todo = (int32_t)(target - S->steps_done);
    if (todo <= 0) return APIC_OK;
    apic_status rc = f64 ? sim_run<double>(S, st, todo, use_graph)
                         : sim_run<float>(S, st, todo, use_graph);
    TRY(rc);
    SimDev d;
    TRY(sim_read_dev(S, st, &d));
    if (S->prof.on) S->prof.collect();
    S->steps_done = d.steps_done;
    if (d.sticky == 0) return APIC_OK;
    if (d.sticky & ~(kErrResize | kErrCapacity)) return status_from_err(d.sticky);
    // grow: clear the sticky error, re-measure from the current state, retry
    launch_clear_sticky(S->dev, st);
    TRY(f64 ? sim_plan<double>(S, st, S->headroom * 1.5) : sim_plan<float>(S, st, S->headroom * 1.5));
    S->headroom *= 1.5;
    S->resizes += 1;
  }
  return APIC_E_DEVICE;
}

// ---------------------------------------------------------------------------
// planned (asynchronous) step
// ---------------------------------------------------------------------------
struct apic_plan {
  apic_ctx *ctx = nullptr;
  Workspace ws;
  Plan plan;
  SceneDev *sc_plan = nullptr;  // the scene table the plan was sized for (device)
  apic_scene *abi = nullptr;    // the same table in the ABI's layout (device)
};

template <typename T>
static void enqueue_plan_step(apic_plan *PL, hipStream_t st, const apic_scene *table,
                              const T *x, T *v, T *C, const T *m, const uint16_t *body,
                              const T *normals, apic_report *reports, int32_t *status) {
  Plan &P = PL->plan;
  // a caller's device table may set flags the plan's own table has not
  const bool plan_variants = P.variants;
  if (table) P.variants = true;
  enqueue_prefix<T>(P, st, x, body, nullptr, true, table ? table : PL->abi, PL->sc_plan);
  enqueue_sort<T>(P, st, x, body, nullptr);
  enqueue_body<T>(P, st, x, v, C, m, body, (T *)PL->ws.ptr[kVbar], nullptr, nullptr, (T *)P.ms,
                  nullptr, nullptr, v, C, true, nullptr, normals);
  if (reports) {
    enqueue_bodies_per_node<T>(P, st);
    launch_fill_reports(P.red, P.cnt, P.body_max, P.ns, reports, st);
  }
  if (status) launch_status(P.cnt, status, st);
  P.variants = plan_variants;
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free entry point
// ---------------------------------------------------------------------------
// A fixed device region (every GPU the library runs on holds its own copy
// until the process ends).  Host code must not pass `scratch` itself to a
// kernel -- on the host it is only a stand-in for the symbol; the device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current (apic_create) and kept in g_scratch_addr.
constexpr size_t kScratchBytes = (size_t)APIC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[kMaxDevices] = {};

// The calling thread's current device must be `device`.
static apic_status scratch_address(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return APIC_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return APIC_E_DEVICE;
    }
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return APIC_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
apic_plan *plan_new(apic_ctx *ctx, double slack) {
  apic_plan *PL = new apic_plan();
  PL->ctx = ctx;
  PL->ws.budget = ctx->ws.budget;
  PL->ws.slack = slack;
  return PL;
}

apic_status plan_measure(apic_plan *PL, hipStream_t st, const apic_scene *scenes,
                         int32_t n_scenes, int64_t n_total, const void *x,
                         const uint16_t *body_id, apic_precision prec, double headroom,
                         const double *dt) {
  TRY(validate_scenes(scenes, n_scenes, n_total));
  if (n_total < 1 || !x || !body_id) return APIC_E_INVALID;
  if (prec != APIC_FP64 && prec != APIC_FP32_MIXED) return APIC_E_INVALID;
  if (!(headroom >= 1.0) || !(headroom <= 64.0)) return APIC_E_INVALID;
  if (dt)
    for (int32_t s = 0; s < n_scenes; ++s)
      if (!std::isfinite(dt[s])) return APIC_E_INVALID;
  apic_ctx *ctx = PL->ctx;
  PL->plan = Plan{};  // every field is derived again below (buffers are kept)
  Plan &P = PL->plan;
  TRY(plan_tables(ctx, PL->ws, P, scenes, n_scenes, n_total, prec, dt, st));
  const size_t sbytes = sizeof(SceneDev) * n_scenes, abytes = sizeof(apic_scene) * n_scenes;
  TRY(PL->ws.ensure(kPlanSc, sbytes));
  TRY(PL->ws.ensure(kPlanAbi, abytes));
  PL->sc_plan = (SceneDev *)PL->ws.ptr[kPlanSc];
  PL->abi = (apic_scene *)PL->ws.ptr[kPlanAbi];
  TRY(ctx->host_stage(abytes));
  std::memcpy(ctx->stage, scenes, abytes);
  HIPOK(hipMemcpyAsync(PL->sc_plan, P.sc, sbytes, hipMemcpyDeviceToDevice, st));
  HIPOK(hipMemcpyAsync(PL->abi, ctx->stage, abytes, hipMemcpyHostToDevice, st));
  if (prec == APIC_FP64)
    enqueue_prefix<double>(P, st, (const double *)x, body_id, nullptr, false);
  else
    enqueue_prefix<float>(P, st, (const float *)x, body_id, nullptr, false);
  Counters c;
  TRY(read_back(ctx, PL->ws, &c, P.cnt, sizeof(Counters), st));
  TRY(status_from_err(c.err));
  TRY(plan_buffers(ctx, PL->ws, P, c.key_blocks, c.smap_total, c.bmap_total, headroom, st));
  TRY(PL->ws.ensure(kVbar, (size_t)P.tbytes * 12 * n_total));
  HIPOK(hipStreamSynchronize(st));
  return APIC_OK;
}

apic_status plan_scene_errors(apic_plan *PL, hipStream_t st, int32_t *out) {
  const Plan &P = PL->plan;
  if (!P.scene_err || P.ns < 1) return APIC_E_INVALID;  // no layout has run
  return read_back(PL->ctx, PL->ws, out, P.scene_err, sizeof(int32_t) * P.ns, st);
}

apic_status status_of_error_bits(int32_t err) {
  apic_status s = status_from_err(err);
  return s != APIC_OK ? s : (err ? APIC_E_DEVICE : APIC_OK);
}

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
  void *scr = nullptr;
  TRY(scratch_address(device, &scr));
  apic_ctx *c = new apic_ctx();
  c->device = device;
  c->ws.budget = hbm_budget_bytes;
  c->cus = prop.multiProcessorCount;
  c->scratch = scr;
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

const char *apic_status_string(int32_t status) {
  switch (status) {
    case APIC_OK: return "ok";
    case APIC_E_INVALID: return "invalid argument";
    case APIC_E_NOMEM: return "device allocation failed";
    case APIC_E_OUT_OF_GRID: return "particle stencil outside the grid";
    case APIC_E_DEVICE: return "HIP runtime error";
    case APIC_E_BUDGET: return "HBM budget exceeded";
    case APIC_E_KEY_OVERFLOW: return "cell-key space overflow";
    case APIC_E_BODY: return "body id out of range";
    case APIC_E_SCRATCH:
      return "scene needs more than the allocation-free entry point's fixed scratch";
    case APIC_E_RESIZE: return "planned step outgrew its plan (create a new plan)";
    case APIC_E_TABLE: return "device scene table does not match its plan";
  }
  return "unknown status";
}

apic_status apic_contact_step_batched(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                                      int32_t n_scenes, int64_t n_total, const void *x, void *v,
                                      void *C, const void *m, const uint16_t *body_id,
                                      const void *normals, apic_precision prec,
                                      apic_report *per_scene) {
  if (!ctx) return APIC_E_INVALID;
  TRY(validate_scenes(scenes, n_scenes, n_total));
  if (n_total > 0 && (!x || !v || !C || !m || !body_id)) return APIC_E_INVALID;
  if (prec != APIC_FP64 && prec != APIC_FP32_MIXED) return APIC_E_INVALID;
  if (hipSetDevice(ctx->device) != hipSuccess) return APIC_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (prec == APIC_FP64)
    return step_impl<double>(ctx, ctx->ws, st, scenes, n_scenes, n_total, (const double *)x,
                             (double *)v, (double *)C, (const double *)m, body_id, per_scene,
                             (const double *)normals);
  return step_impl<float>(ctx, ctx->ws, st, scenes, n_scenes, n_total, (const float *)x,
                          (float *)v, (float *)C, (const float *)m, body_id, per_scene,
                          (const float *)normals);
}

// The scene of a single-scene call: any body id below 65536, L about the
// grid origin, APIC transfers with the Coulomb rule.
static apic_scene single_scene(const apic_grid *grid, int64_t n, double mu, int32_t n_iter) {
  apic_scene s{};
  s.offset = 0;
  s.count = n;
  s.grid = *grid;
  s.mu = mu;
  s.n_iter = n_iter;
  s.n_bodies = 65536;
  for (int d = 0; d < 3; ++d) s.x_ref[d] = grid->origin[d];
  return s;
}

apic_status apic_contact_step(apic_ctx *ctx, void *stream, const apic_grid *grid, int64_t n,
                              const void *x, void *v, void *C, const void *m,
                              const uint16_t *body_id, double mu, int32_t n_iter,
                              apic_precision prec, apic_report *report) {
  if (!ctx || !grid) return APIC_E_INVALID;
  const apic_scene s = single_scene(grid, n, mu, n_iter);
  return apic_contact_step_batched(ctx, stream, &s, 1, n, x, v, C, m, body_id, nullptr, prec,
                                   report);
}

apic_status apic_contact_step_noalloc(apic_ctx *ctx, void *stream, const apic_grid *grid,
                                      int64_t n, const void *x, void *v, void *C, const void *m,
                                      const uint16_t *body_id, double mu, int32_t n_iter,
                                      apic_precision prec, apic_report *report) {
  if (!ctx || !grid) return APIC_E_INVALID;
  const apic_scene s = single_scene(grid, n, mu, n_iter);
  TRY(validate_scenes(&s, 1, n));
  if (n > 0 && (!x || !v || !C || !m || !body_id)) return APIC_E_INVALID;
  if (prec != APIC_FP64 && prec != APIC_FP32_MIXED) return APIC_E_INVALID;
  if (!ctx->scratch) return APIC_E_DEVICE;
  // the particle arrays alone must fit before anything is launched
  const int64_t tb = prec == APIC_FP64 ? 8 : 4;
  if (n > 0 && (uint64_t)n * (uint64_t)(tb * 31 + 24) > kScratchBytes) return APIC_E_SCRATCH;
  if (hipSetDevice(ctx->device) != hipSuccess) return APIC_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  Workspace W;  // carves the scratch region; allocates and frees nothing
  W.arena = (char *)ctx->scratch;
  W.arena_size = kScratchBytes;
  W.budget = kScratchBytes;
  if (prec == APIC_FP64)
    return step_impl<double>(ctx, W, st, &s, 1, n, (const double *)x, (double *)v,
                             (double *)C, (const double *)m, body_id, report);
  return step_impl<float>(ctx, W, st, &s, 1, n, (const float *)x, (float *)v, (float *)C,
                          (const float *)m, body_id, report);
}

apic_status apic_plan_create(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                             int32_t n_scenes, int64_t n_total, const void *x,
                             const uint16_t *body_id, apic_precision prec, double headroom,
                             apic_plan **out) {
  if (!ctx || !out) return APIC_E_INVALID;
  *out = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return APIC_E_DEVICE;
  apic_plan *PL = plan_new(ctx);
  const apic_status rc = plan_measure(PL, (hipStream_t)stream, scenes, n_scenes, n_total, x,
                                      body_id, prec, headroom, nullptr);
  if (rc != APIC_OK) {
    apic_plan_destroy(PL);
    return rc;
  }
  *out = PL;
  return APIC_OK;
}

apic_status apic_plan_step(apic_plan *PL, void *stream, const apic_scene *scenes_dev,
                           const void *x, void *v, void *C, const void *m,
                           const uint16_t *body_id, const void *normals,
                           apic_report *reports_dev, int32_t *status_dev) {
  if (!PL || !x || !v || !C || !m || !body_id) return APIC_E_INVALID;
  if (hipSetDevice(PL->ctx->device) != hipSuccess) return APIC_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (PL->plan.prec == APIC_FP64)
    enqueue_plan_step<double>(PL, st, scenes_dev, (const double *)x, (double *)v, (double *)C,
                              (const double *)m, body_id, (const double *)normals, reports_dev,
                              status_dev);
  else
    enqueue_plan_step<float>(PL, st, scenes_dev, (const float *)x, (float *)v, (float *)C,
                             (const float *)m, body_id, (const float *)normals, reports_dev,
                             status_dev);
  return APIC_OK;
}

void apic_plan_destroy(apic_plan *PL) {
  if (!PL) return;
  (void)hipSetDevice(PL->ctx->device);
  (void)hipDeviceSynchronize();
  PL->ws.release();
  delete PL;
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
  Workspace &W = ctx->ws;
  Plan P;
  TRY(plan_tables(ctx, W, P, scenes, n_scenes, n_total, prec, nullptr, st));
  if (n_total == 0) return APIC_OK;
  if (prec == APIC_FP64)
    enqueue_prefix<double>(P, st, (const double *)x, body_id, nullptr, false);
  else
    enqueue_prefix<float>(P, st, (const float *)x, body_id, nullptr, false);
  Counters c;
  TRY(ctx->host_stage(sizeof(Counters)));
  HIPOK(hipMemcpyAsync(ctx->stage, P.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIPOK(hipStreamSynchronize(st));
  std::memcpy(&c, ctx->stage, sizeof(Counters));
  TRY(status_from_err(c.err));
  TRY(plan_buffers(ctx, W, P, c.key_blocks, c.smap_total, c.bmap_total, 1.0, st));
  if (prec == APIC_FP64)
    enqueue_sort<double>(P, st, (const double *)x, body_id, nullptr, true);
  else
    enqueue_sort<float>(P, st, (const float *)x, body_id, nullptr, true);
  HIPOK(hipMemcpyAsync(keys_sorted, P.keys, sizeof(uint32_t) * n_total, hipMemcpyDeviceToDevice,
                       st));
  HIPOK(hipMemcpyAsync(perm, P.perm, sizeof(uint32_t) * n_total, hipMemcpyDeviceToDevice, st));
  HIPOK(hipStreamSynchronize(st));
  return APIC_OK;
}

int64_t apic_scene_footprint(int64_t n, const apic_grid *grid, apic_precision prec) {
  if (n < 0) return -1;
  const int64_t tb = prec == APIC_FP64 ? 8 : 4;
  // node blocks: about one per 16 particles plus a margin (lattice solids
  // touch about 1.3-2 node blocks per 64 particles, small scenes more), at
  // most what a dense grid holds
  int64_t blocks_hint = n / 16 + 64;
  if (grid && grid->dims[0] > 0 && grid->dims[1] > 0 && grid->dims[2] > 0) {
    int64_t dense = 1;
    for (int d = 0; d < 3; ++d) dense *= (int64_t)grid->dims[d] / kBlock + 2;
    blocks_hint = std::min(blocks_hint, dense);
  }
  // resident state x2 (x, vC, m, body, orig), sorted scratch (t, m, normals,
  // series), keys/values x2; work items and their reduction records (one per
  // 64 particles plus about two per block), one segment per block; grid mass,
  // 3 momentum buffers, 1/m and per-body mass per node block.
  const int64_t per_item = (int64_t)(sizeof(Item) + sizeof(RedRec));
  int64_t per_particle = 2 * (tb * 16 + 2 + 4) + tb * (3 + 1 + 3 + 12) + 4 * 5 + 16 +
                         per_item / kItem + 1;
  int64_t per_block = kNodesPerBlock * (tb * 11 + 8) + 8 * 2 + 2 * per_item +
                      (int64_t)sizeof(Segment);
  return n * per_particle + blocks_hint * per_block + (1 << 20);
}

apic_status apic_sim_create(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                            int32_t n_scenes, int64_t n_total, const double *dt, const void *x,
                            const void *v, const void *C, const void *m, const uint16_t *body_id,
                            apic_precision prec, apic_sim **out) {
  if (!ctx || !out || !dt) return APIC_E_INVALID;
  *out = nullptr;
  TRY(validate_scenes(scenes, n_scenes, n_total));
  if (n_total < 1 || !x || !v || !C || !m || !body_id) return APIC_E_INVALID;
  if (prec != APIC_FP64 && prec != APIC_FP32_MIXED) return APIC_E_INVALID;
  for (int s = 0; s < n_scenes; ++s)
    if (!std::isfinite(dt[s])) return APIC_E_INVALID;
  if (hipSetDevice(ctx->device) != hipSuccess) return APIC_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  apic_sim *S = new apic_sim();
  S->ctx = ctx;
  S->ws.budget = ctx->ws.budget;
  S->n_scenes = n_scenes;
  auto fail = [&](apic_status rc) {
    apic_sim_destroy(S);
    return rc;
  };
  apic_status rc = plan_tables(ctx, S->ws, S->plan, scenes, n_scenes, n_total, prec, dt, st);
  if (rc) return fail(rc);
  const size_t T = S->plan.tbytes;
  const int64_t n = n_total;
  for (int p = 0; p < 2; ++p) {
    SimState &A = S->state[p];
    if (hipMalloc(&A.x, T * 3 * n) != hipSuccess || hipMalloc(&A.vc, T * 12 * n) != hipSuccess ||
        hipMalloc(&A.m, T * n) != hipSuccess ||
        hipMalloc((void **)&A.body, sizeof(uint16_t) * n) != hipSuccess ||
        hipMalloc((void **)&A.orig, sizeof(uint32_t) * n) != hipSuccess) {
      (void)hipGetLastError();
      return fail(APIC_E_NOMEM);
    }
  }
  if (hipMalloc((void **)&S->dev, sizeof(SimDev)) != hipSuccess ||
      hipMalloc((void **)&S->drift, sizeof(double) * 2 * n_scenes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(APIC_E_NOMEM);
  }
  SimState &A = S->state[0];
  if (hipMemcpyAsync(A.x, x, T * 3 * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(A.vc, v, T * 3 * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync((char *)A.vc + T * 3 * n, C, T * 9 * n, hipMemcpyDeviceToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(A.m, m, T * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(A.body, body_id, sizeof(uint16_t) * n, hipMemcpyDeviceToDevice, st) !=
          hipSuccess) {
    (void)hipGetLastError();
    return fail(APIC_E_DEVICE);
  }
  launch_iota(A.orig, n, st);
  fill_bytes_zero(S->dev, sizeof(SimDev), st);
  fill_bytes_zero(S->drift, sizeof(double) * 2 * n_scenes, st);
  if (hipStreamCreateWithFlags(&S->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return fail(APIC_E_DEVICE);
  }
  rc = prec == APIC_FP64 ? sim_plan<double>(S, st, S->headroom) : sim_plan<float>(S, st, S->headroom);
  if (rc) return fail(rc);
  *out = S;
  return APIC_OK;
}

apic_status apic_sim_step(apic_sim *S, void *stream, int32_t n_steps, int32_t use_graph) {
  if (!S || n_steps < 0) return APIC_E_INVALID;
  if (hipSetDevice(S->ctx->device) != hipSuccess) return APIC_E_DEVICE;
  return sim_step_impl(S, (hipStream_t)stream, n_steps, use_graph);
}

apic_status apic_sim_read(apic_sim *S, void *stream, void *x, void *v, void *C) {
  if (!S) return APIC_E_INVALID;
  if (hipSetDevice(S->ctx->device) != hipSuccess) return APIC_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  const SimState &A = S->state[S->parity];
  const int64_t n = S->plan.n;
  if (S->plan.prec == APIC_FP64)
    launch_unpermute<double>(A.orig, n, (const double *)A.x, (const double *)A.vc, (double *)x,
                             (double *)v, (double *)C, st);
  else
    launch_unpermute<float>(A.orig, n, (const float *)A.x, (const float *)A.vc, (float *)x,
                            (float *)v, (float *)C, st);
  HIPOK(hipStreamSynchronize(st));
  return APIC_OK;
}

apic_status apic_sim_report(apic_sim *S, apic_report *per_scene, double *max_drift,
                            int64_t *steps_done) {
  if (!S) return APIC_E_INVALID;
  if (hipSetDevice(S->ctx->device) != hipSuccess) return APIC_E_DEVICE;
  const int ns = S->n_scenes;
  const size_t rbytes = sizeof(double) * kRed * 2 * ns;
  const size_t dbytes = sizeof(double) * 2 * ns, bbytes = sizeof(int32_t) * ns;
  TRY(S->ctx->host_stage(rbytes + sizeof(Counters) + dbytes + bbytes));
  char *stg = (char *)S->ctx->stage;
  // the last step's grids are still in place: count bodies per node from them
  if (per_scene && S->steps_done > 0) {
    if (S->plan.prec == APIC_FP64)
      enqueue_bodies_per_node<double>(S->plan, nullptr);
    else
      enqueue_bodies_per_node<float>(S->plan, nullptr);
  }
  HIPOK(hipMemcpy(stg, S->plan.red, rbytes, hipMemcpyDeviceToHost));
  HIPOK(hipMemcpy(stg + rbytes, S->plan.cnt, sizeof(Counters), hipMemcpyDeviceToHost));
  HIPOK(hipMemcpy(stg + rbytes + sizeof(Counters), S->drift, dbytes, hipMemcpyDeviceToHost));
  HIPOK(hipMemcpy(stg + rbytes + sizeof(Counters) + dbytes, S->plan.body_max, bbytes,
                  hipMemcpyDeviceToHost));
  Counters c;
  std::memcpy(&c, stg + rbytes, sizeof(Counters));
  if (per_scene) {
    std::vector<int32_t> bmax(ns, 0);
    if (S->steps_done > 0) std::memcpy(bmax.data(), stg + rbytes + sizeof(Counters) + dbytes, bbytes);
    fill_report((const double *)stg, ns, c, per_scene, bmax.data());
  }
  if (max_drift) std::memcpy(max_drift, stg + rbytes + sizeof(Counters), sizeof(double) * 2 * ns);
  if (steps_done) *steps_done = S->steps_done;
  return APIC_OK;
}

apic_status apic_sim_set_profiling(apic_sim *S, int32_t enable) {
  if (!S) return APIC_E_INVALID;
  if (!enable) S->prof.collect();
  S->prof.on = enable != 0;
  return APIC_OK;
}

apic_status apic_sim_kernel_times(apic_sim *S, double *ms, int64_t *launches) {
  if (!S) return APIC_E_INVALID;
  S->prof.collect();
  for (int k = 0; k < APIC_KC_COUNT; ++k) {
    if (ms) ms[k] = S->prof.total_ms[k];
    if (launches) launches[k] = S->prof.launches[k];
    S->prof.total_ms[k] = 0.0;
    S->prof.launches[k] = 0;
  }
  return APIC_OK;
}

apic_status apic_sim_info(apic_sim *S, int64_t *out) {
  if (!S || !out) return APIC_E_INVALID;
  if (hipSetDevice(S->ctx->device) != hipSuccess) return APIC_E_DEVICE;
  Counters c;
  HIPOK(hipMemcpy(&c, S->plan.cnt, sizeof(Counters), hipMemcpyDeviceToHost));
  out[0] = S->plan.n;
  out[1] = c.n_sblocks;
  out[2] = c.n_bblocks;
  out[3] = c.n_seg;
  out[4] = c.n_items;
  out[5] = S->plan.sort_bits;
  size_t held = S->ws.held;
  held += 2 * (size_t)S->plan.n * (S->plan.tbytes * 16 + 6);
  out[6] = (int64_t)held;
  return APIC_OK;
}

void apic_sim_destroy(apic_sim *S) {
  if (!S) return;
  (void)hipSetDevice(S->ctx->device);
  (void)hipDeviceSynchronize();
  for (int p = 0; p < 2; ++p) {
    if (S->exec[p]) (void)hipGraphExecDestroy(S->exec[p]);
    SimState &A = S->state[p];
    if (A.x) (void)hipFree(A.x);
    if (A.vc) (void)hipFree(A.vc);
    if (A.m) (void)hipFree(A.m);
    if (A.body) (void)hipFree(A.body);
    if (A.orig) (void)hipFree(A.orig);
  }
  if (S->dev) (void)hipFree(S->dev);
  if (S->drift) (void)hipFree(S->drift);
  if (S->capture_stream) (void)hipStreamDestroy(S->capture_stream);
  S->prof.release();
  S->ws.release();
  delete S;
}

apic_status apic_get_tuning(apic_ctx *ctx, apic_precision prec, int64_t n, apic_tuning *out) {
  if (!ctx || !out || n < 1 || (prec != APIC_FP64 && prec != APIC_FP32_MIXED))
    return APIC_E_INVALID;
  *out = ctx->tuning_for(prec, n);
  return APIC_OK;
}

apic_status apic_set_tuning(apic_ctx *ctx, apic_precision prec, int64_t n,
                            const apic_tuning *tuning) {
  if (!ctx || !tuning || n < 1 || (prec != APIC_FP64 && prec != APIC_FP32_MIXED) ||
      !tuning_ok(*tuning))
    return APIC_E_INVALID;
  ctx->tuning[{(int)prec, size_bucket(n)}] = *tuning;
  return APIC_OK;
}

apic_status apic_autotune(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                          int32_t n_scenes, int64_t n_total, const void *x, const void *v,
                          const void *C, const void *m, const uint16_t *body_id,
                          apic_precision prec, int32_t reps, apic_tuning *best,
                          apic_tuning *candidates, double *times_ms, int32_t max_candidates,
                          int32_t *n_tried) {
  if (!ctx || reps < 1 || reps > 100 || n_total < 1) return APIC_E_INVALID;
  TRY(validate_scenes(scenes, n_scenes, n_total));
  if (!x || !v || !C || !m || !body_id) return APIC_E_INVALID;
  if (prec != APIC_FP64 && prec != APIC_FP32_MIXED) return APIC_E_INVALID;
  if ((times_ms || candidates) && max_candidates < 0) return APIC_E_INVALID;
  if (hipSetDevice(ctx->device) != hipSuccess) return APIC_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  const size_t tb = prec == APIC_FP64 ? 8 : 4;
  TRY(ctx->ws.ensure(kTuneV, tb * 3 * n_total));
  TRY(ctx->ws.ensure(kTuneC, tb * 9 * n_total));
  void *tv = ctx->ws.ptr[kTuneV], *tC = ctx->ws.ptr[kTuneC];
  const std::pair<int, int> key{(int)prec, size_bucket(n_total)};
  const bool had = ctx->tuning.count(key) != 0;
  const apic_tuning before = ctx->tuning_for(prec, n_total);

  // one step on fresh copies of v and C, optionally with every launch timed
  Profiler prof;
  prof.on = true;
  auto run = [&](bool timed) -> apic_status {
    HIPOK(hipMemcpyAsync(tv, v, tb * 3 * n_total, hipMemcpyDeviceToDevice, st));
    HIPOK(hipMemcpyAsync(tC, C, tb * 9 * n_total, hipMemcpyDeviceToDevice, st));
    if (timed) prof.begin(st);
    apic_status rc =
        prec == APIC_FP64
            ? step_impl<double>(ctx, ctx->ws, st, scenes, n_scenes, n_total,
                                (const double *)x, (double *)tv, (double *)tC,
                                (const double *)m, body_id, nullptr)
            : step_impl<float>(ctx, ctx->ws, st, scenes, n_scenes, n_total, (const float *)x,
                               (float *)tv, (float *)tC, (const float *)m, body_id, nullptr);
    if (timed) prof.end(0, st);
    return rc;
  };
  auto score = [&](const apic_tuning &t, double *ms) -> apic_status {
    ctx->tuning[key] = t;
    TRY(run(false));
    for (int k = 0; k < APIC_KC_COUNT; ++k) prof.total_ms[k] = 0.0, prof.launches[k] = 0;
    for (int r = 0; r < reps; ++r) TRY(run(true));
    HIPOK(hipStreamSynchronize(st));
    prof.collect();
    *ms = prof.total_ms[0] / reps;
    return APIC_OK;
  };

  std::vector<apic_tuning> tried;
  std::vector<double> times;
  apic_status rc = APIC_OK;
  apic_tuning bestt = before;
  double best_ms = 1e300;
  // stage 1: work items merged per workgroup, waves per CU, XCD split
  const int group_opts[] = {1, 4, 8};
  const int wave_opts[] = {16, 24, 32, 40, 48};
  for (int grp : group_opts) {
    if (prec == APIC_FP64 && grp > 4) continue;
    for (int xs = 0; xs < 2 && rc == APIC_OK; ++xs)
      for (int wv : wave_opts) {
        apic_tuning t = before;
        t.item_waves_per_cu = wv;
        t.xcd_split = xs;
        t.p2g_group = grp;
        t.p2g_pairs = 0;
        double ms = 0;
        rc = score(t, &ms);
        if (rc != APIC_OK) break;
        tried.push_back(t);
        times.push_back(ms);
        if (ms < best_ms) best_ms = ms, bestt = t;
      }
    if (rc != APIC_OK) break;
  }
  // stage 2: node-kernel launch shape with the best of stage 1
  const int node_opts[] = {4, 8, 16, 32};
  const apic_tuning stage1 = bestt;
  for (int nw : node_opts) {
    if (rc != APIC_OK) break;
    apic_tuning t = stage1;
    t.node_wg_per_cu = nw;
    double ms = 0;
    rc = score(t, &ms);
    if (rc != APIC_OK) break;
    tried.push_back(t);
    times.push_back(ms);
    if (ms < best_ms) best_ms = ms, bestt = t;
  }
  // stage 3: the paired scatter (FP32-mixed kernels) with the best so far
  if (rc == APIC_OK && prec == APIC_FP32_MIXED) {
    apic_tuning t = bestt;
    t.p2g_pairs = 1;
    double ms = 0;
    rc = score(t, &ms);
    if (rc == APIC_OK) {
      tried.push_back(t);
      times.push_back(ms);
      if (ms < best_ms) best_ms = ms, bestt = t;
    }
  }
  prof.release();
  if (rc != APIC_OK) {
    if (had) ctx->tuning[key] = before; else ctx->tuning.erase(key);
    return rc;
  }
  ctx->tuning[key] = bestt;
  if (best) *best = bestt;
  for (int i = 0; i < (int)tried.size() && i < max_candidates; ++i) {
    if (candidates) candidates[i] = tried[i];
    if (times_ms) times_ms[i] = times[i];
  }
  if (n_tried) *n_tried = (int32_t)tried.size();
  return APIC_OK;
}

}  // extern "C"
