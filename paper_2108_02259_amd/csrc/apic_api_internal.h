// apic_api_internal.h -- the context object behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "apic_contact.h"
#include "apic_internal.h"

namespace apic {

enum BufId {
  kScenes, kSceneAcc, kSceneLay, kBodyAcc, kBodyLay, kCounters, kTot, kKeysA, kValsA, kKeysB,
  kValsB, kHist, kPartial, kT, kVbar, kMs, kSbody, kNrm, kY, kRedBuf, kSeg, kSegTmp, kFlags,
  kItems, kSmap, kBmap, kGMass, kGBuf0, kGBuf1, kBMass, kNumBufs
};

// Grow-only device buffers, bounded by an HBM budget.
struct Workspace {
  void *ptr[kNumBufs] = {};
  size_t size[kNumBufs] = {};
  size_t held = 0;
  size_t budget = 0;
  apic_status ensure(int id, size_t bytes);
  void release();
};

struct LayoutResult {
  int64_t nb_cap = 0;
  int32_t max_iter = 0;
  int32_t key_blocks = 0;
  int64_t smap_total = 0, bmap_total = 0;
  int sort_bits = 0;
  uint32_t *keys = nullptr;  // sorted keys
  uint32_t *perm = nullptr;  // sorted position -> input index
};

}  // namespace apic

struct apic_ctx {
  int device = 0;
  int cus = 0;
  int persistent_wg = 2048;
  apic::Workspace ws;
  void *stage = nullptr;  // pinned host staging
  size_t stage_bytes = 0;
  int64_t last_sblocks = 0;
  apic_status host_stage(size_t bytes);
};

apic_status validate_scenes(const apic_scene *scenes, int32_t ns, int64_t n_total);
