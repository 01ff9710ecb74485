// apic_api_internal.h -- the context, plan and resident-driver objects behind
// the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <utility>
#include <vector>

#include "apic_contact.h"
#include "apic_internal.h"
#include "kernels.h"

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

namespace apic {

enum BufId {
  kScenes, kSceneAcc, kSceneLay, kBodyAcc, kBodyLay, kCounters, kTot, kKeysA, kValsA, kKeysB,
  kValsB, kGhist, kLbFlags, kLbState, kT, kVbar, kMs, kSbody, kNrm, kY, kRedBuf, kSeg,
  kItems, kSmark, kSmap, kBmark, kBmap, kGMass, kGBuf0, kGBuf1, kGBuf2, kInvM, kBMass,
  kBoxRec, kRecGather, kRecItems, kTuneV, kTuneC, kB2S, kNodeCount, kBodyMax, kPlanSc,
  kPlanAbi, kSceneErr, kNumBufs
};

// Grow-only device buffers, bounded by an HBM budget.  In arena mode (arena
// set) buffers are carved one after another from a fixed device region
// instead of being allocated: nothing is allocated or freed, every buffer
// counts as fresh, and a request beyond the region fails with
// APIC_E_SCRATCH.
struct Workspace {
  void *ptr[kNumBufs] = {};
  size_t size[kNumBufs] = {};
  bool fresh[kNumBufs] = {};  // (re)allocated since the caller last cleared it
  size_t held = 0;
  size_t budget = 0;
  double slack = 1.0;         // growth factor of a reallocation (>= 1)
  char *arena = nullptr;      // arena mode: the region, its size and the bytes carved
  size_t arena_size = 0;
  apic_status ensure(int id, size_t bytes);
  void release();
};

// Capacities and device pointers of one step.  Everything a step enqueues is
// fixed by the plan, so a step can be captured into a graph and replayed.
struct Plan {
  apic_precision prec = APIC_FP32_MIXED;
  int tbytes = 4;
  int64_t n = 0;
  int ns = 0;
  int64_t nb_cap = 0;
  int max_iter = 0;
  int sort_bits = 32;
  int64_t seg_cap = 0, item_cap = 0, smap_cap = 0, bmap_cap = 0, sblk_cap = 0, bblk_cap = 0;
  int grid_wg = 1;
  int item_wg = 1;
  int node_wg = 1;
  int xcd_split = 0;
  int pairs = 0;
  int group = 1;
  bool ready = false;
  SceneDev *sc = nullptr;
  SceneAcc *sacc = nullptr;
  SceneLay *slay = nullptr;
  BodyAcc *bacc = nullptr;
  BodyLay *blay = nullptr;
  Counters *cnt = nullptr;
  int64_t *tot = nullptr;
  double *red = nullptr;
  BoxRec *box_rec = nullptr;
  RedRec *rec_gather = nullptr, *rec_items = nullptr;
  uint32_t *ka = nullptr, *va = nullptr, *kb = nullptr, *vb = nullptr, *ghist = nullptr;
  Lookback lb = {};
  uint32_t *keys = nullptr, *perm = nullptr;
  void *t = nullptr, *ms = nullptr, *nrm = nullptr, *Y = nullptr;
  int32_t *sbody = nullptr;
  Segment *seg = nullptr;
  Item *items = nullptr;
  int32_t *smark = nullptr, *smap = nullptr, *bmark = nullptr, *bmap = nullptr;
  int32_t *b2s = nullptr;         // body-grid block -> shared-grid block
  int32_t *node_count = nullptr;  // bodies with mass per shared node (reports)
  int32_t *body_max = nullptr;    // per scene: most bodies at one node
  int32_t *scene_err = nullptr;   // per scene: error bits of its particles
  bool variants = false;  // some scene carries flags (or a device table may set them)
  GridPtrs g = {};
};

// Kernel timing of eager steps: every launch between begin() and end(kind)
// gets its own event pair (recorded with the dispatch); end() files them
// under `kind`.
struct Profiler : LaunchTimer {
  struct Rec {
    int kind;
    hipEvent_t start, stop;
  };
  bool on = false;
  std::vector<hipEvent_t> free_events;
  std::vector<Rec> recs;
  size_t open_from = 0;  // first record of the current class
  double total_ms[APIC_KC_COUNT] = {};
  int64_t launches[APIC_KC_COUNT] = {};
  void events(hipEvent_t *start, hipEvent_t *stop) override;
  void begin(hipStream_t st);
  void end(int kind, hipStream_t st);
  void collect();
  void release();
};

// Resident particle state in sorted order (x, v|C as 12 rows, m, body, and the
// caller index of each particle).
struct SimState {
  void *x = nullptr, *vc = nullptr, *m = nullptr;
  uint16_t *body = nullptr;
  uint32_t *orig = nullptr;
};

// Device-side driver status.
struct SimDev {
  int32_t sticky;      // error bits of any step since the last clear
  int32_t pad;
  int64_t steps_done;  // completed steps
};

// ---- driver kernels (misc.hip) --------------------------------------------
void launch_clear_sticky(SimDev *dev, hipStream_t st);
void launch_step_end(const Counters *cnt, const double *red, int ns, SimDev *dev, double *drift,
                     hipStream_t st);
void launch_iota(uint32_t *p, int64_t n, hipStream_t st);
template <typename T>
void launch_unpermute(const uint32_t *orig, int64_t n, const T *x_sorted, const T *vc_sorted,
                      T *x_out, T *v_out, T *C_out, hipStream_t st);

}  // namespace apic

struct apic_ctx {
  int device = 0;
  int cus = 0;
  void *scratch = nullptr;  // device address of this device's allocation-free scratch
  apic::Workspace ws;
  // launch tuning per (precision, floor(log2 n))
  std::map<std::pair<int, int>, apic_tuning> tuning;
  apic_tuning tuning_for(apic_precision prec, int64_t n) const;
  void *stage = nullptr;  // pinned host staging
  size_t stage_bytes = 0;
  apic_status host_stage(size_t bytes);
};

struct apic_sim {
  apic_ctx *ctx = nullptr;
  apic::Workspace ws;
  apic::Plan plan;
  apic::SimState state[2];
  int parity = 0;            // state[parity] holds the current state
  int n_scenes = 0;
  apic::SimDev *dev = nullptr;
  double *drift = nullptr;   // per scene: max |dP|/P_scale, max |dL|/L_scale
  int64_t steps_done = 0;
  double headroom = 1.5;
  int resizes = 0;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  bool graph_ok = false;
  apic::Profiler prof;
};

apic_status validate_scenes(const apic_scene *scenes, int32_t ns, int64_t n_total);

// The apic_status an error word maps to.
apic_status status_of_error_bits(int32_t err);

// An empty plan on ctx (no buffers yet); filled by plan_measure.  Its
// buffers grow by `slack` when they grow (a plan re-measured for a growing
// batch, such as a serving loop's resident set).
apic_plan *plan_new(apic_ctx *ctx, double slack = 1.0);
// (Re)measure a batch into PL, reusing its buffers (they only grow):
// apic_plan_create's work, plus the driver's per-scene drift step dt (host,
// n_scenes entries, may be null), so that the planned step forms
// Vbar = V + dt {a, 0} on the device.  Synchronises st once.
apic_status plan_measure(apic_plan *PL, hipStream_t st, const apic_scene *scenes,
                         int32_t n_scenes, int64_t n_total, const void *x,
                         const uint16_t *body_id, apic_precision prec, double headroom,
                         const double *dt);
// Each scene's error bits from the plan's last step (host, n_scenes
// entries); synchronises st.
apic_status plan_scene_errors(apic_plan *PL, hipStream_t st, int32_t *out);
