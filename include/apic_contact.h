/*
 * apic_contact.h -- C ABI of the MI355X (gfx950) APIC augury contact library.
 *
 * The library computes the contact step of Tupek, Koester and Mosby,
 * "A momentum preserving frictional contact algorithm based on affine
 * particle-in-cell grid transfers" (arXiv 2108.02259): given particle
 * positions x, masses m, body ids and a predicted generalized velocity
 * Vbar = {v, C} (Section 2.2: Vbar = V + tau A), it returns the preferred
 * generalized velocity Vhat = S(Vbar) of the augury-iteration series
 * (Section 2.3, eq. for Vhat with N iterations) with the Coulomb rule of
 * Section 2.4, using APIC transfers (Section 2.1.2, eqs. particleToGrid,
 * gridToParticle, scaledVelGrad) on the modified quadratic B-spline grid of
 * Appendix B.
 *
 * Conventions for every entry point:
 *  - Particle arrays are structure-of-arrays, component-major, length n:
 *      x[d*n + p], v[d*n + p] (d = 0..2), C[(3a+b)*n + p] = C_ab,
 *      m[p] (> 0), body_id[p].
 *    Element type is double for APIC_FP64 and float for APIC_FP32_MIXED.
 *  - C is the APIC affine matrix C_p = B_p D_p^{-1} = (2/h^2) B_p (the paper
 *    stores B_p; D_p = h^2/2 I for this basis, Appendix B), row-major,
 *    C_ab = d v_a / d x_b.
 *  - Grid node j (integer triple) sits at origin + h*j.  dims all zero means
 *    an unbounded sparse grid; dims > 0 declares a dense grid whose stencil
 *    nodes must satisfy 0 <= j < dims (else APIC_E_OUT_OF_GRID).
 *  - Particle pointers are DEVICE pointers owned by the caller; the library
 *    never frees them.  Scene tables and reports are HOST memory.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it; calls that return a status synchronise that stream before returning
 *    so that device-detected errors are reported.
 *  - Validation happens before any launch: a call that returns
 *    APIC_E_INVALID has not touched v or C.  A device-detected error
 *    (out-of-grid particle, key space overflow) leaves v and C untouched.
 *  - Contexts are not thread-safe; calls on one context must not overlap.
 *
 * Precision (APIC_FP32_MIXED): positions, fields, P2G/G2P weights and grid
 * momenta are float; cell keys, grid velocities (q/m), contact normals, the
 * friction rule and all momentum reductions are double.
 */
#ifndef APIC_CONTACT_H
#define APIC_CONTACT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  APIC_OK = 0,
  APIC_E_INVALID = -1,      /* bad argument (checked before any launch) */
  APIC_E_NOMEM = -2,        /* device allocation failed */
  APIC_E_OUT_OF_GRID = -3,  /* a stencil node left a dense grid, or a cell
                               index left the int32 range */
  APIC_E_DEVICE = -4,       /* a HIP runtime call failed */
  APIC_E_BUDGET = -5,       /* the context's HBM budget is too small */
  APIC_E_KEY_OVERFLOW = -6, /* more than 2^26 cell blocks in the key space */
  APIC_E_BODY = -7,         /* body id >= the scene's n_bodies */
  APIC_E_SCRATCH = -8,      /* the scene needs more device memory than the fixed
                               scratch of apic_contact_step_noalloc holds */
  APIC_E_RESIZE = -9,       /* a planned step outgrew its plan's capacities (the
                               step did nothing; create a new plan) */
  APIC_E_TABLE = -10        /* a device scene table does not match its plan */
} apic_status;

typedef enum { APIC_FP64 = 0, APIC_FP32_MIXED = 1 } apic_precision;

/* Background grid (Section 2, Appendix B): spacing h > 0, node j at
 * origin + h*j; dims = {0,0,0} for an unbounded sparse grid. */
typedef struct {
  double origin[3];
  double h;
  int32_t dims[3];
} apic_grid;

/* Momentum report of one step (all FP64).  "before" is the step's input
 * Vbar, "after" its output Vhat.  L is taken about the scene's x_ref (the
 * grid origin for the single-scene calls) and includes the affine spin
 * (h^2/2) (C_zy - C_yz, C_xz - C_zx, C_yx - C_xy) that the APIC transfers
 * conserve (Section 2.1.2); E = 1/2 sum m (|v|^2 + (h^2/2)|C|_F^2).
 * P_scale = sum m |v|, L_scale = sum m (|x - x_ref||v| + (h^2/2)|C|_F)
 * normalise drift when the totals vanish. */
typedef struct {
  double P_before[3], P_after[3];
  double L_before[3], L_after[3];
  double E_before, E_after;
  double P_scale, L_scale;
  int64_t n_particles;
  int64_t n_unconstrained;     /* particles without a contact normal (zero
                                  own-body mass gradient, or a zero given
                                  normal); 0 when N = 0 (no series, no normals) */
  int64_t grid_blocks;         /* active 4x4x4 node blocks of the shared grid */
  int32_t max_bodies_per_node; /* most bodies with mass at one grid node */
  int32_t reserved;
} apic_report;

/* Scene flags: variants of the method the paper contrasts. */
enum {
  /* PIC transfers (Section 2.1.1; the "PIC augury" of Section 2.2): the
   * particle-to-grid sum drops the affine term and C is not part of the
   * transferred state, so C passes through the step unchanged.  Linear
   * momentum is conserved, angular momentum in general is not. */
  APIC_PIC = 1,
  /* The separation-only rule of Section 2.3 instead of the Coulomb rule of
   * Section 2.4: W = (dv, dC) where dv.n > 0, else 0. */
  APIC_RULE_SEPARATE = 2
};

/* One scene of a packed batch: its particles are [offset, offset + count) of
 * the packed arrays, its body ids are < n_bodies. */
typedef struct {
  int64_t offset, count;
  apic_grid grid;
  double mu;         /* Coulomb coefficient, >= 0 (Section 2.4) */
  int32_t n_iter;    /* augury iterations N >= 0 (N + 1 applications of H) */
  int32_t n_bodies;
  int32_t flags;     /* APIC_PIC | APIC_RULE_SEPARATE, 0 = APIC + Coulomb */
  int32_t reserved;  /* 0 */
  double accel[3];   /* mechanical acceleration a of the scene (Section 2.2:
                        the resident driver and the server predict
                        Vbar = V + dt {a, 0} before each contact step; the
                        stateless calls take Vbar itself and ignore it) */
  double x_ref[3];   /* reference point of the reported angular momentum */
} apic_scene;

typedef struct apic_ctx apic_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * workspace the context may hold (0 = no bound).  Returns APIC_E_DEVICE if
 * the device is not usable. */
apic_status apic_create(apic_ctx **out, int device, size_t hbm_budget_bytes);

/* Release the context and its workspace (synchronises its device). */
void apic_destroy(apic_ctx *ctx);

/* Human-readable name of a status code (static storage); any int32 value is
 * accepted, values that are no apic_status give "unknown status". */
const char *apic_status_string(int32_t status);

/* The contact step S of one scene (Sections 2.1.2-2.4): overwrites v and C
 * with Vhat.  mu >= 0 is the Coulomb coefficient (Section 2.4), n_iter = N
 * >= 0 the number of augury iterations (Section 2.3; N = 0 is the plain,
 * sticky APIC transfer).  body_id < 65536 distinguishes bodies for the
 * contact normals.  `report` (host, optional) receives momentum before and
 * after. */
apic_status apic_contact_step(apic_ctx *ctx, void *stream, const apic_grid *grid,
                              int64_t n, const void *x, void *v, void *C,
                              const void *m, const uint16_t *body_id, double mu,
                              int32_t n_iter, apic_precision prec,
                              apic_report *report);

/* Bytes of the fixed device scratch behind apic_contact_step_noalloc. */
#define APIC_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* apic_contact_step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, semantics and results, but every work buffer
 * of the step is carved from one fixed device array of
 * APIC_NOALLOC_SCRATCH_BYTES per GPU, held from library load until the
 * process ends.  The call performs no hipMalloc, hipFree or other allocating
 * call (device or pinned host); its two small readbacks go straight to the
 * caller's stack.  The caller still owns x, v, C, m and body_id.
 *  - A scene whose particle arrays cannot fit is refused with APIC_E_SCRATCH
 *    before any launch; one whose measured grid does not fit is refused with
 *    APIC_E_SCRATCH after the layout pass, before v and C are touched.
 *    (Roughly: a compact scene of up to ~3e5 FP32 or ~1.5e5 FP64
 *    particles fits.)
 *  - Every call on one GPU shares that GPU's scratch, and each call starts
 *    by clearing what the step needs zeroed: calls that overlap on one GPU
 *    (different streams or threads) race and must be serialised by the
 *    caller.  Calls on apic_contact_step and the other entry points do not
 *    touch it.
 *  - It synchronises `stream` like apic_contact_step. */
apic_status apic_contact_step_noalloc(apic_ctx *ctx, void *stream, const apic_grid *grid,
                                      int64_t n, const void *x, void *v, void *C,
                                      const void *m, const uint16_t *body_id, double mu,
                                      int32_t n_iter, apic_precision prec,
                                      apic_report *report);

/* The contact step of many independent scenes in one set of launches over
 * packed arrays of n_total particles, each with its own grid, mu, N and
 * flags.  scenes (host, n_scenes entries) must tile [0, n_total) in
 * increasing offset order.  normals (device, optional, [3][n_total] of the
 * precision's type): the caller's particle normals -- the paper's n_p, an
 * area-weighted outward normal of the finite-element boundary faces at the
 * node (Section 2.3), which only the caller's mesh knows; a zero normal
 * marks an unconstrained particle -- used instead of the body-mass-gradient
 * normals.  per_scene (host, optional, n_scenes entries) receives each
 * scene's report.  Synchronises `stream` (twice: the layout is measured
 * before the step is sized); apic_plan_step is the asynchronous form. */
apic_status apic_contact_step_batched(apic_ctx *ctx, void *stream,
                                      const apic_scene *scenes, int32_t n_scenes,
                                      int64_t n_total, const void *x, void *v,
                                      void *C, const void *m,
                                      const uint16_t *body_id, const void *normals,
                                      apic_precision prec, apic_report *per_scene);

/* ------------------------------------------------------------------------
 * Planned (asynchronous, graph-capturable) contact step.
 *
 * apic_contact_step(_batched) measure each call's layout with a readback
 * before sizing it.  A plan measures a batch once and keeps device buffers
 * sized with headroom, so that apic_plan_step enqueues the whole step on the
 * caller's stream with no host synchronisation, no host memory access and
 * no allocation -- it can be captured into a HIP graph and replayed.  The
 * device checks every capacity; a step that would exceed one does nothing
 * (v and C untouched) and reports APIC_E_RESIZE through status_dev.
 * ------------------------------------------------------------------------ */
typedef struct apic_plan apic_plan;

/* Measure the batch (same arguments and rules as apic_contact_step_batched;
 * x and body_id are read, one synchronisation) and size a plan for it with
 * capacities `headroom` >= 1 times the measured ones.  The plan keeps a
 * device copy of the scene table. */
apic_status apic_plan_create(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                             int32_t n_scenes, int64_t n_total, const void *x,
                             const uint16_t *body_id, apic_precision prec, double headroom,
                             apic_plan **out);

/* Enqueue the contact step of the plan's batch on `stream` (the problem
 * statement of Section 2.2, V <- S(Vbar), per scene) and return at once.
 * x, v, C, m, body_id, normals as for apic_contact_step_batched (device,
 * n_total particles of the plan's precision).  Device-side optional
 * arguments:
 *  - scenes_dev: a DEVICE scene table for this call (n_scenes entries with
 *    the plan's offsets, counts and n_bodies; grid, mu, flags, x_ref may
 *    differ; n_iter at most the plan's largest).  NULL: the plan's table.  A
 *    mismatch makes the step do nothing and reports APIC_E_TABLE.
 *  - reports_dev: DEVICE array of n_scenes reports, written by the step.
 *  - status_dev: DEVICE int32, set to the step's apic_status (0 = ok).
 * The returned status covers host-side argument checks only.  Calls on one
 * plan must not overlap (they share its buffers). */
apic_status apic_plan_step(apic_plan *plan, void *stream, const apic_scene *scenes_dev,
                           const void *x, void *v, void *C, const void *m,
                           const uint16_t *body_id, const void *normals,
                           apic_report *reports_dev, int32_t *status_dev);

void apic_plan_destroy(apic_plan *plan);

/* Cell keys and the stable particle order of a batch (the layout step of the
 * contact step, exposed for verification): keys_sorted[i] is the 32-bit cell
 * key of the i-th particle in sorted order and perm[i] its input index.
 * key = block number * 64 + cell in block (x fastest), with cells
 * floor((x - origin)/h) in FP64 and 4x4x4-cell blocks; each body's key range
 * numbers its blocks super block by super block (2x2x2 blocks, row-major over
 * the body's super-block box, x fastest, then x fastest within the super
 * block), bodies in (scene, body) order.  Equal keys keep input order.  (The
 * contact step itself orders particles by block number only, keeping input
 * order within a block.)  keys_sorted and perm are device arrays of n_total
 * entries. */
apic_status apic_sort_keys(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                           int32_t n_scenes, int64_t n_total, const void *x,
                           const uint16_t *body_id, apic_precision prec,
                           uint32_t *keys_sorted, uint32_t *perm);

/* ------------------------------------------------------------------------
 * Resident time stepping.
 *
 * A sim owns device copies of a packed batch of scenes and advances them with
 * the explicit driver of Section 2.2 with tau = dt: each step predicts
 * Vbar = V + dt {a, 0} with the scene's mechanical acceleration a
 * (apic_scene.accel, constant; the scaled velocity gradient has no mechanical
 * rate), sets V <- S(Vbar) (the contact step above, with each scene's mu, N
 * and flags, normals from the body mass gradients) and then x <- x + dt v.  State stays in HBM between
 * steps, in the library's sorted order; apic_sim_read returns it in the
 * caller's original order.  Capacities are sized from the initial state with
 * headroom; a step that would exceed them is replayed after the plan grows,
 * so results never depend on the headroom.  Steps can be captured into HIP
 * graphs (use_graph = 1) and replayed with no host synchronisation.
 * ------------------------------------------------------------------------ */
typedef struct apic_sim apic_sim;

/* Copy the batch (same layout and rules as apic_contact_step_batched) into a
 * new sim.  dt (host, n_scenes entries) is each scene's time step. */
apic_status apic_sim_create(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                            int32_t n_scenes, int64_t n_total, const double *dt,
                            const void *x, const void *v, const void *C, const void *m,
                            const uint16_t *body_id, apic_precision prec, apic_sim **out);

/* Advance every scene by n_steps driver steps; synchronises `stream` at the
 * end to check for errors. */
apic_status apic_sim_step(apic_sim *sim, void *stream, int32_t n_steps, int32_t use_graph);

/* Copy the current state to caller arrays (device, caller order; any of the
 * pointers may be NULL). */
apic_status apic_sim_read(apic_sim *sim, void *stream, void *x, void *v, void *C);

/* Report of the last step per scene (host, n_scenes entries; may be NULL),
 * and the largest relative momentum drift of any step so far per scene:
 * max_drift[2*s] = max |dP|/P_scale, max_drift[2*s + 1] = max |dL|/L_scale
 * (host, 2*n_scenes entries; may be NULL).  Also returns the number of
 * completed steps. */
apic_status apic_sim_report(apic_sim *sim, apic_report *per_scene, double *max_drift,
                            int64_t *steps_done);

/* Kernel timing: when enabled, eager (non-graph) steps bracket each kernel
 * class with HIP events on the step's stream.  apic_sim_kernel_times
 * returns, per class (APIC_KC_*), the summed milliseconds and the number of
 * launches since the last call, and resets them. */
enum {
  APIC_KC_LAYOUT = 0,   /* cells, boxes, key domains, keys */
  APIC_KC_SORT = 1,     /* radix sort passes */
  APIC_KC_GATHER = 2,   /* permute state into sorted order, momentum before */
  APIC_KC_SEGMENTS = 3, /* segments, work items, node-block maps, grid clear */
  APIC_KC_MASS = 4,     /* grid mass and per-body mass */
  APIC_KC_P2G0 = 5,     /* contact normals and Vbar to grid */
  APIC_KC_GRIDVEL = 6,  /* (no kernels: grid velocities are formed as the rounds
                           load their tiles) */
  APIC_KC_ROUND1 = 7,   /* first series round (G2P + rule + P2G) */
  APIC_KC_ROUND = 8,    /* later series rounds (G2P + rule + P2G) */
  APIC_KC_FINAL = 9,    /* final G2P and output */
  APIC_KC_AFTER = 10,   /* momentum after the step, drift */
  APIC_KC_COUNT = 11
};
apic_status apic_sim_set_profiling(apic_sim *sim, int32_t enable);
apic_status apic_sim_kernel_times(apic_sim *sim, double *ms, int64_t *launches);

/* Sizes of the sim's current plan: out[0] particles, out[1] active shared
 * node blocks of the last step, out[2] active body node blocks, out[3]
 * segments, out[4] work items, out[5] sort key bits, out[6] device bytes held. */
apic_status apic_sim_info(apic_sim *sim, int64_t *out);

void apic_sim_destroy(apic_sim *sim);

/* Device bytes a context needs to step one scene of n particles on `grid`
 * (host, may be NULL): a dense grid bounds the node blocks by its dims, a
 * sparse one (or NULL) is estimated from n.  Used by admission control.
 * Pure host function; -1 for n < 0. */
int64_t apic_scene_footprint(int64_t n, const apic_grid *grid, apic_precision prec);

/* ------------------------------------------------------------------------
 * Launch tuning.
 *
 * The particle kernels (mass, normals, P2G and the fused rounds) run one
 * 64-lane wave per work item of up to 64 particles.  How many waves a launch
 * keeps per compute unit, how items are spread over the eight XCDs and how
 * many work items of one 2x2x2-block super block a workgroup merges in LDS
 * before its global atomics change speed but never results beyond
 * floating-point summation order.  A context keeps one tuning per
 * (precision, size bucket), the bucket being floor(log2(n_total)); calls and
 * sims created afterwards use the entry of their own bucket (a sim fixes its
 * tuning at creation).
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t item_waves_per_cu; /* persistent waves per compute unit for the
                                particle kernels, 1..64 */
  int32_t node_wg_per_cu;    /* 256-lane workgroups per compute unit for the
                                grid-node kernels, 1..64 */
  int32_t xcd_split;         /* 1: each XCD works through one contiguous eighth
                                of the (spatially sorted) items; 0: all
                                workgroups stride over all items */
  int32_t p2g_group;         /* 1, 4 or 8 work items of one super block per
                                workgroup, their LDS tiles summed before the
                                flush to the grid (FP64 uses at most 4) */
  int32_t p2g_pairs;         /* 1: paired scatter -- in work items whose cells
                                hold several particles, consecutive lanes of
                                one cell are paired and one lane of each pair
                                adds both particles' terms to the LDS tile,
                                halving the passes over the stencil; 0: one
                                pass per particle rank in its cell.  FP32-mixed
                                kernels only (the FP64 path ignores it) */
} apic_tuning;

/* Read or set the tuning a context uses for `prec` and the size bucket of n
 * (n >= 1).  apic_set_tuning rejects out-of-range fields with
 * APIC_E_INVALID. */
apic_status apic_get_tuning(apic_ctx *ctx, apic_precision prec, int64_t n, apic_tuning *out);
apic_status apic_set_tuning(apic_ctx *ctx, apic_precision prec, int64_t n,
                            const apic_tuning *tuning);

/* Autotuner: times the contact step of the given batch (same arguments and
 * rules as apic_contact_step_batched; x, v, C, m are only read -- the timed
 * steps write to internal copies of v and C) under each candidate tuning,
 * `reps` timed steps per candidate after one untimed step, scoring each by
 * the summed device time of its kernels (HIP events recorded with each
 * dispatch).  The fastest becomes the context's tuning for (prec, bucket of
 * n_total) and is returned in *best (host, optional); times_ms (host,
 * optional, max_candidates entries) receives each candidate's score and
 * candidates (host, optional) the candidates in the same order.  Returns the
 * number of candidates tried through *n_tried (optional). */
apic_status apic_autotune(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                          int32_t n_scenes, int64_t n_total, const void *x, const void *v,
                          const void *C, const void *m, const uint16_t *body_id,
                          apic_precision prec, int32_t reps, apic_tuning *best,
                          apic_tuning *candidates, double *times_ms, int32_t max_candidates,
                          int32_t *n_tried);

/* ------------------------------------------------------------------------
 * Serving loop (continuous batching).
 *
 * A server keeps the state of many independent requests resident in one
 * packed device arena and advances all of them together, one driver step per
 * tick: the contact step (as apic_contact_step_batched, every resident
 * request being one scene) and then x <- x + dt v, with each request's own
 * mu, N and dt.  Requests wait in FIFO order until the arena has room for
 * their particles, a scene slot is free and the summed apic_scene_footprint of
 * the resident requests stays within the server's budget; they join at the
 * next tick and leave once they have taken their steps, their final x, v, C
 * copied to the caller's output arrays.  A request's result does not depend
 * on which other requests share its ticks (up to floating-point summation
 * order).
 * ------------------------------------------------------------------------ */
typedef struct apic_server apic_server;

typedef struct {
  int32_t resident;   /* requests stepped by this tick */
  int32_t admitted;   /* requests that joined at this tick */
  int32_t completed;  /* requests that finished at this tick */
  int32_t queued;     /* requests still waiting after this tick */
  int32_t deferred;   /* queued requests held back at admission (no room, slot
                         or budget for the head of the queue) */
  int32_t failed;     /* requests retired by this tick with an error */
  int32_t replayed;   /* 1 if this tick's step replayed the graph captured for
                         an unchanged resident set, else 0 */
  int32_t reserved;
  int64_t particles;  /* particles stepped by this tick */
  int64_t footprint;  /* summed footprint of the requests stepped by this tick */
} apic_tick;

/* Create a server on ctx's device: an arena for max_particles resident
 * particles (device memory allocated here, 2 copies of x, v, C, m, body),
 * at most max_scenes resident requests, and budget_bytes bounding the summed
 * footprint of resident requests (0 = no bound). */
apic_status apic_server_create(apic_ctx *ctx, apic_precision prec, int64_t max_particles,
                               int32_t max_scenes, int64_t budget_bytes, apic_server **out);

/* Queue a request: one scene (scene->count = its n particles, offset
 * ignored; grid, mu, n_iter, n_bodies as for a batch) advanced `steps` >= 1
 * driver steps of `dt`.  x, v, C, m, body_id are device arrays of the request
 * in the library layout (stride n); they are read when the request is
 * admitted and must stay valid until then.  x_out, v_out, C_out (device,
 * stride n) receive the final state and may alias x, v, C.  Returns
 * APIC_E_BUDGET if the request can never be admitted (more particles than the
 * arena, or a footprint above the budget). */
apic_status apic_server_submit(apic_server *srv, int64_t tag, const apic_scene *scene, double dt,
                               int32_t steps, const void *x, const void *v, const void *C,
                               const void *m, const uint16_t *body_id, void *x_out, void *v_out,
                               void *C_out);

/* One tick on `stream`: admit what fits, step every resident request once
 * (each with its own mu, N, flags, dt and acceleration: Vbar = V + dt {a, 0},
 * then V <- S(Vbar), then x <- x + dt v), copy out and retire the requests
 * that have taken all their steps, and synchronise the stream.  A request
 * whose particles the device rejects (non-finite values, a body id beyond
 * its n_bodies, a stencil node outside its dense grid) is retired with that
 * status and the others are stepped without it, so one bad request never
 * stalls the rest.  info (host, optional) describes the tick; done_tags and
 * done_status (host, optional, max_done entries each) receive the tag and
 * status (APIC_OK when completed, else the error) of every request retired
 * by this tick (all of them are retired either way). */
apic_status apic_server_tick(apic_server *srv, void *stream, apic_tick *info, int64_t *done_tags,
                             int32_t *done_status, int32_t max_done);

/* Withdraw a request by tag: a queued one leaves the queue now, a resident
 * one leaves at the start of the next tick (its outputs are not written).
 * APIC_E_INVALID if no such request is queued or resident. */
apic_status apic_server_cancel(apic_server *srv, int64_t tag);

/* Release the server and its arena (queued requests are dropped). */
void apic_server_destroy(apic_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* APIC_CONTACT_H */
