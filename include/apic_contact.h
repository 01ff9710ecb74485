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
  APIC_E_BODY = -7          /* body id >= the scene's n_bodies */
} apic_status;

typedef enum { APIC_FP64 = 0, APIC_FP32_MIXED = 1 } apic_precision;

/* Background grid (Section 2, Appendix B): spacing h > 0, node j at
 * origin + h*j; dims = {0,0,0} for an unbounded sparse grid. */
typedef struct {
  double origin[3];
  double h;
  int32_t dims[3];
} apic_grid;

/* Momentum report of one step (all FP64).  L is taken about the grid origin
 * and includes the affine spin (h^2/2) (C_zy - C_yz, C_xz - C_zx, C_yx - C_xy)
 * that the APIC transfers conserve (Section 2.1.2); E = 1/2 sum m (|v|^2 +
 * (h^2/2)|C|_F^2).  P_scale = sum m |v|, L_scale = sum m (|x - o||v| +
 * (h^2/2)|C|_F) normalise drift when the totals vanish. */
typedef struct {
  double P_before[3], P_after[3];
  double L_before[3], L_after[3];
  double E_before, E_after;
  double P_scale, L_scale;
  int64_t n_particles;
  int64_t n_unconstrained; /* particles with a zero mass gradient */
  int64_t grid_blocks;     /* active 4x4x4 node blocks of the shared grid */
} apic_report;

/* One scene of a packed batch: its particles are [offset, offset + count) of
 * the packed arrays, its body ids are < n_bodies. */
typedef struct {
  int64_t offset, count;
  apic_grid grid;
  double mu;       /* Coulomb coefficient, >= 0 */
  int32_t n_iter;  /* augury iterations N >= 0 (N + 1 applications of H) */
  int32_t n_bodies;
} apic_scene;

typedef struct apic_ctx apic_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * workspace the context may hold (0 = no bound).  Returns APIC_E_DEVICE if
 * the device is not usable. */
apic_status apic_create(apic_ctx **out, int device, size_t hbm_budget_bytes);

/* Release the context and its workspace (synchronises its device). */
void apic_destroy(apic_ctx *ctx);

/* Human-readable name of a status code (static storage). */
const char *apic_status_string(apic_status s);

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

/* The contact step of many independent scenes in one set of launches over
 * packed arrays of n_total particles.  scenes (host, n_scenes entries) must
 * tile [0, n_total) in increasing offset order.  per_scene (host, optional,
 * n_scenes entries) receives each scene's report. */
apic_status apic_contact_step_batched(apic_ctx *ctx, void *stream,
                                      const apic_scene *scenes, int32_t n_scenes,
                                      int64_t n_total, const void *x, void *v,
                                      void *C, const void *m,
                                      const uint16_t *body_id, apic_precision prec,
                                      apic_report *per_scene);

/* Cell keys and the stable particle order of a batch (the layout step of the
 * contact step, exposed for verification): keys_sorted[i] is the 32-bit cell
 * key of the i-th particle in sorted order and perm[i] its input index.
 * key = (body block offset + local block, x fastest) * 64 + cell in block,
 * with cells floor((x - origin)/h) in FP64 and 4x4x4-cell blocks; each body's
 * block box is laid out in (scene, body) order.  Equal keys keep input
 * order.  keys_sorted and perm are device arrays of n_total entries. */
apic_status apic_sort_keys(apic_ctx *ctx, void *stream, const apic_scene *scenes,
                           int32_t n_scenes, int64_t n_total, const void *x,
                           const uint16_t *body_id, apic_precision prec,
                           uint32_t *keys_sorted, uint32_t *perm);

/* Device bytes a context needs to run one scene of n particles spread over
 * about `blocks_hint` 4x4x4 cell blocks (0 = estimate from n); used by
 * admission control.  Pure host function. */
int64_t apic_scene_footprint(int64_t n, int64_t blocks_hint, apic_precision prec);

#ifdef __cplusplus
}
#endif

#endif /* APIC_CONTACT_H */
