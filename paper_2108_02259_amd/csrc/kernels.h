// kernels.h -- host-side launchers of the library's HIP kernels.
#pragma once

#include "apic_internal.h"

namespace apic {

// ---- scan / fill (sort.hip) ------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

inline int64_t scan_tile_count(int64_t n_cap, int items = kScanItems) {
  const int64_t tile = (int64_t)kScanThreads * items;
  return (n_cap + tile - 1) / tile + 1;
}

// Device state of the single-pass scans and sort passes (decoupled
// look-back): flag words and {finished tiles, epoch}.  Initialise once with
// lookback_init; launches on one Lookback must not overlap.
struct Lookback {
  uint64_t *flags;
  int64_t capacity;  // flag words: >= tiles of any scan, >= 256 * tiles of any sort pass
  uint32_t *state;
};
void lookback_init(const Lookback &lb, hipStream_t st);

// Exclusive prefix sum of in[0, n) into out (out must not alias in).  n is
// n_dev[0] when n_dev is non-null (n_cap bounds it), else n_cap.  The total is
// written to *total (int64).  mode 1 writes -1 where in[i] == 0 (slot maps).
void scan_exclusive(const int32_t *in, int32_t *out, int64_t n_cap, const int64_t *n_dev,
                    int64_t *total, const Lookback &lb, int mode, hipStream_t st);
// Two such scans in one launch (flags for scan_tile_count(cap0) +
// scan_tile_count(cap1) tiles).
void scan_exclusive_pair(const int32_t *in0, int32_t *out0, int64_t cap0, const int64_t *n0_dev,
                         int64_t *total0, const int32_t *in1, int32_t *out1, int64_t cap1,
                         const int64_t *n1_dev, int64_t *total1, const Lookback &lb, int mode,
                         hipStream_t st);

void fill_i32(int32_t *p, int32_t value, int64_t n_cap, const int64_t *n_dev, int64_t scale,
              hipStream_t st);
// One scene record written by a kernel that takes it as an argument (no host
// staging buffer).
void launch_store_scene(SceneDev *dst, const SceneDev &s, hipStream_t st);
void fill_bytes_zero(void *p, int64_t bytes, hipStream_t st);
void fill_zero_f(void *p, int64_t elems_cap, const int32_t *n_dev, int64_t per, int elem_bytes,
                 hipStream_t st);

// ---- radix sort (sort.hip) -------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;
constexpr int kSortTile = kSortThreads * kSortItems;

inline int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

// Stable LSD radix sort of (key, index) by key bits [lo, bits), 8 bits per
// pass (at most 4), each pass: per-tile digit counts, a single-pass scan of
// them in digit-major order, and the scatter.
// keys/vals ping-pong between the a and b buffers; the return value is 0 if
// the result is in (ka, va), 1 if in (kb, vb).  Values start as the identity
// permutation 0..n-1 (va need not be initialised).  hist holds
// radix_hist_words(n) words of scratch.
inline int64_t radix_hist_words(int64_t n) { return 2 * 256 * sort_tiles(n) + 4; }
// hist0_ready: the first pass's digit counts are already in hist (written by
// launch_keys with the sort's tile geometry).
int radix_sort(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, int64_t n, int lo,
               int bits, uint32_t *hist, const Lookback &lb, bool hist0_ready, hipStream_t st);

// Grid arrays of a step (slot-major, see the transfers).
struct GridPtrs {
  void *mass;        // [sblk][64] T
  void *buf[3];      // [sblk][3][64] T each: grid momenta, rotating over the rounds
  void *bmass;       // [bblk][64] T: per-body grid mass
  double *invm;      // [sblk][64]: 1 / mass (0 where the mass is 0)
};

// ---- layout (layout.hip) ---------------------------------------------------
// One box record per wavefront (rec has ceil(n/256)*4 entries), then reduced.
template <typename T>
void launch_cells(const T *x, const uint16_t *body, int64_t n, const SceneDev *sc, int ns,
                  BodyAcc *bacc, BoxRec *rec, Counters *cnt, int32_t *scene_err, hipStream_t st);
inline int64_t wave_records(int64_t n) { return (n + 255) / 256 * 4; }
// Empty boxes, zero counters (error word from sticky if given) and cleared
// per-scene sums red[0, red_n).
void launch_layout_init(SceneAcc *sacc, int ns, BodyAcc *bacc, int nb_cap, Counters *cnt,
                        const int32_t *sticky, double *red, int64_t red_n, int32_t *scene_err,
                        hipStream_t st);
// key_bits > 0: flag kErrResize if the key space needs more bits; smap_cap /
// bmap_cap > 0: flag kErrResize if the node-block maps need more entries.
void launch_domains(const SceneDev *sc, int ns, int nb_cap, SceneAcc *sacc, const BodyAcc *bacc,
                    SceneLay *slay, BodyLay *blay, Counters *cnt, int key_bits, int64_t smap_cap,
                    int64_t bmap_cap, hipStream_t st);
// Cell keys; also the digit counts of the sort's first pass (bits
// [shift, shift+8)) per sort tile into hist, as the radix sort lays them out.
template <typename T>
void launch_keys(const T *x, const uint16_t *body, int64_t n, const SceneDev *sc, int ns,
                 const BodyLay *blay, uint32_t *keys, int shift, uint32_t *hist, hipStream_t st);
// Gather the particle state into sorted order.  keys/perm come from the
// block-order sort; within each wave the particles are further ordered by
// cell (stable), and that final order's keys and permutation go to
// keys_out/perm_out (distinct from keys/perm).
template <typename T>
void launch_gather(const uint32_t *perm, const uint32_t *keys, int64_t n, const T *x,
                   const T *v, const T *C, const T *m, const uint16_t *body, const SceneDev *sc,
                   int ns, T *t_out, T *vbar_out, T *m_out, int32_t *sbody_out,
                   T *x_out, uint16_t *body_out, const uint32_t *orig_in, uint32_t *orig_out,
                   uint32_t *keys_out, uint32_t *perm_out, RedRec *rec, double *direct,
                   const T *nrm_in, T *nrm_out, Counters *cnt, int32_t *scene_err,
                   hipStream_t st);
// Segments (one per (body, cell block) of the sorted keys, with their node
// blocks marked in smark/bmark) and work items, from two single-pass scans;
// tot[0] = segments, tot[1] = items, tot[5]/tot[6] = slot-map extents.
void launch_segments(const uint32_t *keys, int64_t n, const Lookback &lb, int64_t *tot,
                     const int32_t *sbody, const BodyLay *blay, const SceneLay *slay,
                     Segment *seg, int64_t seg_cap, Item *items, int64_t item_cap, int32_t *smark,
                     int64_t smap_cap, int32_t *bmark, int64_t bmap_cap, int align, Counters *cnt,
                     hipStream_t st);
// Node-block maps: scan the marks into slots, store each segment's 8 slots
// and clear the marks again (so that the mark arrays are all zero between
// steps); publishes the segment, item and active-block counts, and zeroes
// the grid mass, momentum buffers 0 and 1 and the body mass over the active
// blocks (tbytes bytes per value); reduces the records grec[0, grec_count)
// into gred.
void launch_maps(Segment *seg, int64_t seg_cap, const SceneLay *slay, const BodyLay *blay,
                 int32_t *smark, int32_t *smap, int64_t smap_cap, int32_t *bmark, int32_t *bmap,
                 int64_t bmap_cap, const Lookback &lb, int64_t *tot, Counters *cnt,
                 int64_t sblk_cap, int64_t bblk_cap, int64_t item_cap, GridPtrs g, int tbytes,
                 int node_wg, const RedRec *grec, int64_t grec_count, double *gred,
                 int32_t *b2s, hipStream_t st);

// ---- transfers (transfer.hip) ---------------------------------------------

struct StepArgs {
  const SceneDev *sc;
  const Segment *seg;
  const Item *items;
  const Counters *cnt;
  const uint32_t *keys;  // sorted
  int64_t n;
  int grid_wg;           // workgroups of the grouped particle kernels (64*group lanes)
  int item_wg;           // workgroups of the one-wave particle kernels
  int node_wg;           // 256-lane workgroups of the node kernels
  int xcd_split;         // 1: each XCD walks one contiguous eighth of the items
  int group;             // work items merged per workgroup before the flush (1, 4, 8)
  int given_normals;     // 1: the normals array holds the caller's normals
  int variants;          // 1: some scene may carry flags (APIC_PIC, APIC_RULE_SEPARATE)
  int pairs;             // 1: paired scatter of same-cell particles (FP32 kernels)
};

template <typename T>
void launch_mass(const StepArgs &a, const T *t, const T *m, GridPtrs g, hipStream_t st);
// Contact normals (where a scene has series rounds) and P2G of Vbar into
// buffer 0, in one pass over the items (after launch_mass).  Sets each
// item's full_y to 1 if one of its particles has no normal (the rounds then
// keep full series-state rows for it).
template <typename T>
void launch_p2g0(const StepArgs &a, const T *t, const T *m, const T *vbar, T *nrm, Item *items,
                 GridPtrs g, hipStream_t st);
// One fused round k = 1 .. max n_iter: G2P of the momenta in buffer
// (k-1) mod 3 (turned into velocities q/m as the tile is loaded), the rule,
// P2G of the next series field into buffer k mod 3, and clearing of buffer
// (k+1) mod 3 for round k+1.  Scenes whose n_iter == k-1 finish here (writing
// Vhat to v_out/C_out at perm[i], or at i when perm is null).
template <typename T>
void launch_round(const StepArgs &a, int k, const T *t, const T *m, const T *vbar, const T *nrm,
                  T *Y, GridPtrs g, const uint32_t *perm, T *v_out, T *C_out, hipStream_t st);
// The last round k = max n_iter + 1: the remaining scenes finish, then every
// particle's FP64 momentum after the step (one record per work item into
// rec, item_cap entries) and, with drift set, x += dt v (x indexed like
// v_out).
template <typename T>
void launch_final(const StepArgs &a, int k, const T *t, const T *m, const T *vbar, const T *nrm,
                  const T *Y, GridPtrs g, const uint32_t *perm, T *v_out, T *C_out, T *x,
                  int drift, RedRec *rec, hipStream_t st);
// Reduce records [0, count) (count = *count_dev if non-null, skipped when the
// step has an error) into out[key * kRed + c].
void launch_reduce_red(const RedRec *rec, int64_t count_cap, const int32_t *count_dev,
                       const Counters *cnt, double *out, hipStream_t st);
// Reduce box records into the per-body boxes (and cnt->max_gb).
void launch_reduce_box(const BoxRec *rec, int64_t count, BodyAcc *bacc, Counters *cnt,
                       hipStream_t st);
// Most bodies with mass at one node, per scene, into body_max[scene]: node
// counts over the body-grid blocks (b2s maps a body block to its shared
// block), then a maximum over each segment's shared blocks.  count holds
// sblk_cap * 64 int32.
template <typename T>
void launch_bodies_per_node(const Counters *cnt, const Segment *seg, int64_t seg_cap,
                            const T *bmass, const int32_t *b2s, int64_t bblk_cap,
                            int64_t sblk_cap, int32_t *count, int32_t *body_max, int ns,
                            hipStream_t st);
// Per-scene reports on the device from the step's sums (red: before then
// after, kRed each per scene), counters and body maxima (may be null).
void launch_fill_reports(const double *red, const Counters *cnt, const int32_t *body_max, int ns,
                         apic_report *out, hipStream_t st);
// The step's status (0 or an apic_status) from the counters' error word.
void launch_status(const Counters *cnt, int32_t *status, hipStream_t st);
// Scene table of a planned step: the caller's device table (or the plan's,
// both in the ABI's layout) checked against the plan's and converted into
// `out`; a mismatch sets kErrTable.
void launch_scene_table(const apic_scene *in, const SceneDev *plan_sc, int ns, int max_iter,
                        SceneDev *out, Counters *cnt, hipStream_t st);

}  // namespace apic
