/*
 * apic_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, deliberately unoptimised FP64 CPU reference of the APIC
 * augury contact step of Tupek, Koester and Mosby, "A momentum preserving
 * frictional contact algorithm based on affine particle-in-cell grid
 * transfers" (arXiv 2108.02259).  It exists so that the GPU library can be
 * checked against something written directly from the paper.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * GPU library shares no code, header or table with it.
 *
 * Conventions (shared with the library's public interface, not its code):
 *   - arrays are structure-of-arrays, component-major: x[d*n + p];
 *   - C is the APIC affine matrix C_p = B_p D_p^{-1} (Section 2.1.2), stored
 *     row-major per particle: C[(3*a + b)*n + p] = C_ab (dv_a/dx_b);
 *   - grid node j sits at origin + h*j; dims[d] > 0 declares a dense grid whose
 *     stencil nodes must satisfy 0 <= j < dims[d], dims[d] == 0 is unbounded.
 *
 * Every floating-point quantity is double; accumulation runs in particle-index
 * order so the result is deterministic.
 *
 * Pins: every function is checked against closed forms, special cases,
 * brute force or library routines by the CPU tests (oracle pins and
 * variants).  Multi-step driving is pinned by invariants (exact translation,
 * and mirror symmetry, P and L of a symmetric collision at every step).
 * Parity unpinned: the driver's multi-step trajectories in general.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_E_INVALID (-1)
#define ORA_E_NOMEM (-2)
#define ORA_E_OUT_OF_GRID (-3)
#define ORA_E_KEY_OVERFLOW (-6)

#define ORA_KERNEL_QUAD 0   /* modified quadratic B-spline (Appendix B) */
#define ORA_KERNEL_LINEAR 1 /* linear hat functions (Section 3.1 analysis) */

#define ORA_TRANSFER_APIC 0 /* Section 2.1.2 */
#define ORA_TRANSFER_PIC 1  /* Section 2.1.1: no affine term, B not evolved */

#define ORA_RULE_COULOMB 0  /* Section 2.4: friction cone */
#define ORA_RULE_SEPARATE 1 /* Section 2.3: separation only */

typedef struct {
  int32_t dim;      /* 1 or 3 */
  int32_t kernel;   /* ORA_KERNEL_* */
  int32_t transfer; /* ORA_TRANSFER_* */
  int32_t rule;     /* ORA_RULE_* */
  double origin[3];
  double h;
  int32_t dims[3];
} ora_grid;

/* ------------------------------------------------------------------------ */
/* Shape functions                                                           */
/* ------------------------------------------------------------------------ */

/*
 * One-dimensional shape functions covering the point xi (in grid units),
 * Appendix B.  With i = floor(xi), the quadratic basis spans nodes i-1..i+2
 * and is assembled from the three parabolas a_i, b_i, c_i exactly as the
 * appendix defines them.  The two middle functions are (a+b)/4 and (b+c)/4:
 * with the printed factor 1/8 the four functions sum to (3a+2b+3c)/8, which is
 * not one, whereas the appendix requires partition of unity and linear
 * completeness; the factor 1/4 gives both, and gives D_p = h^2/2 I as the
 * appendix states.
 *
 * The linear option is the pair of hat functions used in the two-particle
 * analysis of Section 3.1 (nodes i and i+1).
 *
 * w[k] is the value at node first+k; dw[k] its derivative with respect to xi.
 * Returns the number of nodes (4 or 2).
 */
static int shape_1d(int kernel, double xi, int64_t *first, double w[4],
                    double dw[4]) {
  double i = floor(xi);
  if (kernel == ORA_KERNEL_QUAD) {
    double a = (i + 1.0 - xi) * (i + 1.0 - xi);
    double b = (-i + 1.0 + xi) * (i + 1.0 - xi) + (i + 2.0 - xi) * (xi - i);
    double c = (xi - i) * (xi - i);
    double da = -2.0 * (i + 1.0 - xi);
    double db = (i + 1.0 - xi) - (-i + 1.0 + xi) + (i + 2.0 - xi) - (xi - i);
    double dc = 2.0 * (xi - i);
    w[0] = a / 4.0;
    w[1] = (a + b) / 4.0;
    w[2] = (b + c) / 4.0;
    w[3] = c / 4.0;
    dw[0] = da / 4.0;
    dw[1] = (da + db) / 4.0;
    dw[2] = (db + dc) / 4.0;
    dw[3] = dc / 4.0;
    *first = (int64_t)i - 1;
    return 4;
  }
  double t = xi - i;
  w[0] = 1.0 - t;
  w[1] = t;
  dw[0] = -1.0;
  dw[1] = 1.0;
  *first = (int64_t)i;
  return 2;
}

/* Exported for the partition-of-unity / completeness pins. */
int ora_shape_1d(int32_t kernel, double xi, int64_t *first, double *w,
                 double *dw) {
  return shape_1d(kernel, xi, first, w, dw);
}

/*
 * The tensor-product stencil of one particle (Section 2, "standard outer
 * product of 1D spline spaces"): node indices, N_i(x_p), grad N_i(x_p) and
 * x_i - x_p.  Axes beyond `dim` carry a single node (index 0) with weight 1
 * and zero offset, so a 1-D problem uses the same code as a 3-D one.
 */
typedef struct {
  int count;
  int64_t node[64][3];
  double w[64];
  double grad[64][3];
  double dx[64][3];
} stencil;

static void make_stencil(const ora_grid *g, const double xp[3], stencil *s) {
  int64_t first[3] = {0, 0, 0};
  int cnt[3] = {1, 1, 1};
  double w[3][4] = {{1, 0, 0, 0}, {1, 0, 0, 0}, {1, 0, 0, 0}};
  double dw[3][4] = {{0}};
  for (int d = 0; d < g->dim; ++d) {
    double xi = (xp[d] - g->origin[d]) / g->h;
    cnt[d] = shape_1d(g->kernel, xi, &first[d], w[d], dw[d]);
  }
  s->count = 0;
  for (int c = 0; c < cnt[2]; ++c)
    for (int b = 0; b < cnt[1]; ++b)
      for (int a = 0; a < cnt[0]; ++a) {
        int k = s->count++;
        int off[3] = {a, b, c};
        double wk = w[0][a] * w[1][b] * w[2][c];
        s->w[k] = wk;
        s->grad[k][0] = dw[0][a] * w[1][b] * w[2][c] / g->h;
        s->grad[k][1] = w[0][a] * dw[1][b] * w[2][c] / g->h;
        s->grad[k][2] = w[0][a] * w[1][b] * dw[2][c] / g->h;
        for (int d = 0; d < 3; ++d) {
          s->node[k][d] = first[d] + off[d];
          if (d < g->dim) {
            double xi_node = g->origin[d] + g->h * (double)s->node[k][d];
            s->dx[k][d] = xi_node - xp[d];
          } else {
            s->dx[k][d] = 0.0;
            s->grad[k][d] = 0.0;
          }
        }
      }
}

/* ------------------------------------------------------------------------ */
/* A dense node array over a bounding box: the simplest correct grid.        */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t lo[3];
  int64_t ext[3];
  double *m; /* mass per node */
  double *q; /* momentum (3 per node), then velocity after normalisation */
} dgrid;

static int64_t dg_index(const dgrid *G, const int64_t j[3]) {
  return (j[0] - G->lo[0]) +
         G->ext[0] * ((j[1] - G->lo[1]) + G->ext[1] * (j[2] - G->lo[2]));
}

static void dg_free(dgrid *G) {
  free(G->m);
  free(G->q);
  G->m = G->q = NULL;
}

/* Allocate a zeroed node array over the box [lo, hi] (inclusive). */
static int dg_alloc_box(dgrid *G, const int64_t lo[3], const int64_t hi[3],
                        int with_q) {
  int64_t total = 1;
  for (int d = 0; d < 3; ++d) {
    G->lo[d] = lo[d];
    G->ext[d] = hi[d] >= lo[d] ? hi[d] - lo[d] + 1 : 1;
    total *= G->ext[d];
  }
  G->m = (double *)calloc((size_t)total, sizeof(double));
  G->q = with_q ? (double *)calloc((size_t)total * 3, sizeof(double)) : NULL;
  if (!G->m || (with_q && !G->q)) {
    dg_free(G);
    return ORA_E_NOMEM;
  }
  return ORA_OK;
}

static int64_t dg_total(const dgrid *G) { return G->ext[0] * G->ext[1] * G->ext[2]; }

static void dg_zero(dgrid *G) {
  int64_t total = dg_total(G);
  memset(G->m, 0, (size_t)total * sizeof(double));
  if (G->q) memset(G->q, 0, (size_t)total * 3 * sizeof(double));
}

static void particle_x(const ora_grid *g, int64_t n, const double *x,
                       int64_t p, double xp[3]) {
  xp[0] = x[p];
  xp[1] = g->dim > 1 ? x[n + p] : 0.0;
  xp[2] = g->dim > 1 ? x[2 * n + p] : 0.0;
}

/* First and last stencil node of particle p along each axis. */
static void node_range(const ora_grid *g, int64_t n, const double *x, int64_t p,
                       int64_t lo[3], int64_t hi[3]) {
  double xp[3], w[4], dw[4];
  particle_x(g, n, x, p, xp);
  for (int d = 0; d < 3; ++d) {
    lo[d] = hi[d] = 0;
    if (d >= g->dim) continue;
    int64_t first;
    int cnt = shape_1d(g->kernel, (xp[d] - g->origin[d]) / g->h, &first, w, dw);
    lo[d] = first;
    hi[d] = first + cnt - 1;
  }
}

/* Box of all stencil nodes of all particles. */
static int shared_grid(const ora_grid *g, int64_t n, const double *x, dgrid *G) {
  int64_t lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
  int64_t hi[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
  for (int64_t p = 0; p < n; ++p) {
    int64_t a[3], b[3];
    node_range(g, n, x, p, a, b);
    for (int d = 0; d < 3; ++d) {
      if (a[d] < lo[d]) lo[d] = a[d];
      if (b[d] > hi[d]) hi[d] = b[d];
    }
  }
  return dg_alloc_box(G, lo, hi, 1);
}

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra                                                */
/* ------------------------------------------------------------------------ */

/* Inverse of the leading dim x dim block of a 3x3 row-major matrix; the
 * remaining entries of the result are zero.  Returns 0 if singular. */
static int inverse_block(int dim, const double A[9], double R[9]) {
  memset(R, 0, 9 * sizeof(double));
  if (dim == 1) {
    if (A[0] == 0.0) return 0;
    R[0] = 1.0 / A[0];
    return 1;
  }
  double c00 = A[4] * A[8] - A[5] * A[7];
  double c01 = A[5] * A[6] - A[3] * A[8];
  double c02 = A[3] * A[7] - A[4] * A[6];
  double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  if (det == 0.0) return 0;
  R[0] = c00 / det;
  R[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  R[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  R[3] = c01 / det;
  R[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  R[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  R[6] = c02 / det;
  R[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  R[8] = (A[0] * A[4] - A[1] * A[3]) / det;
  return 1;
}

/*
 * D_p = sum_i N_i(x_p) (x_i - x_p) (x) (x_i - x_p)  (Section 2.1.2), taken
 * literally from its definition rather than from the closed form h^2/2 I.
 */
static void inertia_tensor(const ora_grid *g, const double xp[3], double D[9]) {
  stencil s;
  make_stencil(g, xp, &s);
  memset(D, 0, 9 * sizeof(double));
  for (int k = 0; k < s.count; ++k)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) D[3 * a + b] += s.w[k] * s.dx[k][a] * s.dx[k][b];
}

int ora_inertia(const ora_grid *g, const double *xp, double *D) {
  if (!g || !xp || !D) return ORA_E_INVALID;
  inertia_tensor(g, xp, D);
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Grid checks                                                               */
/* ------------------------------------------------------------------------ */

static int check_dense_bounds(const ora_grid *g, int64_t n, const double *x) {
  int dense = 0;
  for (int d = 0; d < g->dim; ++d) dense |= g->dims[d] > 0;
  if (!dense) return ORA_OK;
  stencil s;
  for (int64_t p = 0; p < n; ++p) {
    double xp[3];
    particle_x(g, n, x, p, xp);
    make_stencil(g, xp, &s);
    for (int k = 0; k < s.count; ++k)
      for (int d = 0; d < g->dim; ++d)
        if (s.node[k][d] < 0 || s.node[k][d] >= g->dims[d])
          return ORA_E_OUT_OF_GRID;
  }
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* The transformation operator H                                             */
/* ------------------------------------------------------------------------ */

/*
 * One application of the grid transfer operator, U -> H U, for a generalized
 * velocity U = {u, E} with E = B D^{-1}:
 *   mass to grid      m_i     = sum_p N_i(x_p) m_p                   (eq. massToGrid)
 *   momentum to grid  m_i v_i = sum_p N_i(x_p) m_p [u_p + E_p (x_i - x_p)]
 *                                                        (eq. particleToGrid)
 *   grid velocity     v_i = (m_i v_i) / m_i, and 0 where m_i = 0
 *   velocity back     u'_p = sum_i N_i(x_p) v_i            (eq. gridToParticle)
 *   gradient back     B'_p = sum_i N_i(x_p) v_i (x) (x_i - x_p)
 *                                                          (eq. scaledVelGrad)
 *                     E'_p = B'_p D_p^{-1}
 * For the PIC transfer (Section 2.1.1) the affine term is dropped from the
 * momentum sum and B is not part of the transferred state: Section 3.1 sets
 * B_p = 0 in the particle-to-grid sum and removes its evolution, and the PIC
 * augury of Section 2.2 is the method with no scaled velocity gradient term.
 * The operator therefore maps {u, E} to {u', E}: the affine part passes
 * through untouched (so G = H - I has a zero affine part and the series never
 * changes C).
 * Dinv holds D_p^{-1} per particle (9 per particle, row-major).
 */
static int apply_H(const ora_grid *g, int64_t n, const double *x,
                   const double *m, const double *Dinv, const double *u,
                   const double *E, double *uo, double *Eo, dgrid *Gp) {
  dgrid G = *Gp;
  dg_zero(&G);
  stencil s;
  int apic = g->transfer == ORA_TRANSFER_APIC;
  for (int64_t p = 0; p < n; ++p) {
    double xp[3];
    particle_x(g, n, x, p, xp);
    make_stencil(g, xp, &s);
    for (int k = 0; k < s.count; ++k) {
      int64_t idx = dg_index(&G, s.node[k]);
      double wm = s.w[k] * m[p];
      G.m[idx] += wm;
      for (int a = 0; a < 3; ++a) {
        double val = u[a * n + p];
        if (apic)
          for (int b = 0; b < 3; ++b) val += E[(3 * a + b) * n + p] * s.dx[k][b];
        G.q[3 * idx + a] += wm * val;
      }
    }
  }
  int64_t total = dg_total(&G);
  for (int64_t i = 0; i < total; ++i)
    for (int a = 0; a < 3; ++a)
      G.q[3 * i + a] = G.m[i] > 0.0 ? G.q[3 * i + a] / G.m[i] : 0.0;
  for (int64_t p = 0; p < n; ++p) {
    double xp[3];
    particle_x(g, n, x, p, xp);
    make_stencil(g, xp, &s);
    double vo[3] = {0, 0, 0};
    double Bo[9] = {0};
    for (int k = 0; k < s.count; ++k) {
      int64_t idx = dg_index(&G, s.node[k]);
      for (int a = 0; a < 3; ++a) {
        double vi = G.q[3 * idx + a];
        vo[a] += s.w[k] * vi;
        for (int b = 0; b < 3; ++b) Bo[3 * a + b] += s.w[k] * vi * s.dx[k][b];
      }
    }
    for (int a = 0; a < 3; ++a) uo[a * n + p] = vo[a];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double e = 0.0;
        if (apic)
          for (int c = 0; c < 3; ++c) e += Bo[3 * a + c] * Dinv[9 * p + 3 * c + b];
        else
          e = E[(3 * a + b) * n + p]; /* PIC: B is not evolved */
        Eo[(3 * a + b) * n + p] = e;
      }
  }
  return ORA_OK;
}

static int inverse_inertia_all(const ora_grid *g, int64_t n, const double *x,
                               double *Dinv) {
  for (int64_t p = 0; p < n; ++p) {
    double xp[3], D[9];
    particle_x(g, n, x, p, xp);
    inertia_tensor(g, xp, D);
    if (!inverse_block(g->dim, D, Dinv + 9 * p)) return ORA_E_INVALID;
  }
  return ORA_OK;
}

static int valid_grid(const ora_grid *g) {
  if (!g) return 0;
  if (g->dim != 1 && g->dim != 3) return 0;
  if (g->kernel != ORA_KERNEL_QUAD && g->kernel != ORA_KERNEL_LINEAR) return 0;
  if (g->transfer != ORA_TRANSFER_APIC && g->transfer != ORA_TRANSFER_PIC) return 0;
  if (g->rule != ORA_RULE_COULOMB && g->rule != ORA_RULE_SEPARATE) return 0;
  if (!(g->h > 0.0) || !isfinite(g->h)) return 0;
  for (int d = 0; d < 3; ++d)
    if (!isfinite(g->origin[d]) || g->dims[d] < 0) return 0;
  return 1;
}

/* Exported single application of H (linearity, brute-force matrix, pins). */
int ora_apply_H(const ora_grid *g, int64_t n, const double *x, const double *m,
                const double *u, const double *E, double *uo, double *Eo) {
  if (!valid_grid(g) || n < 0) return ORA_E_INVALID;
  if (n == 0) return ORA_OK;
  int rc = check_dense_bounds(g, n, x);
  if (rc) return rc;
  double *Dinv = (double *)malloc((size_t)n * 9 * sizeof(double));
  if (!Dinv) return ORA_E_NOMEM;
  dgrid G = {{0}, {0}, NULL, NULL};
  rc = inverse_inertia_all(g, n, x, Dinv);
  if (!rc) rc = shared_grid(g, n, x, &G);
  if (!rc) rc = apply_H(g, n, x, m, Dinv, u, E, uo, Eo, &G);
  dg_free(&G);
  free(Dinv);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Contact normals                                                           */
/* ------------------------------------------------------------------------ */

/*
 * Outward particle normals.  The paper area-weights finite-element boundary
 * face normals (Section 2.3); no mesh crosses this interface, so the normal
 * is taken from the particle's own body's grid mass field instead:
 *   m^b_i = sum_{q in body b} N_i(x_q) m_q,   g_p = sum_i m^{b(p)}_i grad N_i(x_p),
 *   n_p = -g_p / |g_p|   (mass decreases outward).
 * A particle with g_p == 0 has no normal and is reported unconstrained (flag 1).
 */
static int compute_normals(const ora_grid *g, int64_t n, const double *x,
                           const double *m, const uint16_t *body, double *nrm,
                           int32_t *uncon) {
  static const int NB = 65536;
  dgrid *bg = (dgrid *)calloc(NB, sizeof(dgrid));
  char *present = (char *)calloc(NB, 1);
  if (!bg || !present) {
    free(bg);
    free(present);
    return ORA_E_NOMEM;
  }
  int rc = ORA_OK;
  int64_t *lo = (int64_t *)malloc((size_t)NB * 3 * sizeof(int64_t));
  int64_t *hi = (int64_t *)malloc((size_t)NB * 3 * sizeof(int64_t));
  if (!lo || !hi) rc = ORA_E_NOMEM;
  for (int64_t k = 0; k < (int64_t)NB * 3 && !rc; ++k) {
    lo[k] = INT64_MAX;
    hi[k] = INT64_MIN;
  }
  for (int64_t p = 0; p < n && !rc; ++p) {
    int64_t a[3], b[3];
    int bb = body[p];
    present[bb] = 1;
    node_range(g, n, x, p, a, b);
    for (int d = 0; d < 3; ++d) {
      if (a[d] < lo[3 * bb + d]) lo[3 * bb + d] = a[d];
      if (b[d] > hi[3 * bb + d]) hi[3 * bb + d] = b[d];
    }
  }
  for (int b = 0; b < NB && !rc; ++b)
    if (present[b]) rc = dg_alloc_box(&bg[b], lo + 3 * b, hi + 3 * b, 0);
  free(lo);
  free(hi);
  stencil s;
  for (int64_t p = 0; p < n && !rc; ++p) {
    double xp[3];
    particle_x(g, n, x, p, xp);
    make_stencil(g, xp, &s);
    dgrid *G = &bg[body[p]];
    for (int k = 0; k < s.count; ++k) G->m[dg_index(G, s.node[k])] += s.w[k] * m[p];
  }
  for (int64_t p = 0; p < n && !rc; ++p) {
    double xp[3];
    particle_x(g, n, x, p, xp);
    make_stencil(g, xp, &s);
    dgrid *G = &bg[body[p]];
    double gp[3] = {0, 0, 0};
    for (int k = 0; k < s.count; ++k) {
      double mi = G->m[dg_index(G, s.node[k])];
      for (int d = 0; d < 3; ++d) gp[d] += mi * s.grad[k][d];
    }
    double len = sqrt(gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2]);
    if (len > 0.0) {
      for (int d = 0; d < 3; ++d) nrm[d * n + p] = -gp[d] / len;
      uncon[p] = 0;
    } else {
      for (int d = 0; d < 3; ++d) nrm[d * n + p] = 0.0;
      uncon[p] = 1;
    }
  }
  for (int b = 0; b < NB; ++b)
    if (present[b]) dg_free(&bg[b]);
  free(bg);
  free(present);
  return rc;
}

int ora_normals(const ora_grid *g, int64_t n, const double *x, const double *m,
                const uint16_t *body, double *nrm, int32_t *uncon) {
  if (!valid_grid(g) || n < 0) return ORA_E_INVALID;
  if (n == 0) return ORA_OK;
  return compute_normals(g, n, x, m, body, nrm, uncon);
}

/* ------------------------------------------------------------------------ */
/* The undesirable part of a velocity change                                 */
/* ------------------------------------------------------------------------ */

/*
 * Section 2.4 (Coulomb friction): for the proposed change d at a particle with
 * outward normal n,
 *   d_n = d . n;  d_t = d - d_n n  (the part in the tangent plane);
 *   s   = min(|d_t|, -mu d_n);
 *   undesirable = d - d_n n - s d_t/|d_t|   if d_n <= 0  (and 0 when d_t = 0),
 *               = d                          otherwise (the change pulls away).
 * The paper prints the tangential part as d n (x) n and the cone bound as
 * mu d_n; read with d_t in the tangent plane and -mu d_n, which is the only
 * reading under which the kept change d_n n + s d_t/|d_t| lies in the cone.
 *
 * Section 2.3 (separation only): undesirable = d if d_n > 0, else 0.
 */
static void undesirable_v(int rule, const double d[3], const double nrm[3],
                          double mu, double out[3]) {
  double dn = d[0] * nrm[0] + d[1] * nrm[1] + d[2] * nrm[2];
  if (dn > 0.0) {
    for (int a = 0; a < 3; ++a) out[a] = d[a];
    return;
  }
  if (rule == ORA_RULE_SEPARATE) {
    for (int a = 0; a < 3; ++a) out[a] = 0.0;
    return;
  }
  double dt[3];
  for (int a = 0; a < 3; ++a) dt[a] = d[a] - dn * nrm[a];
  double tau = sqrt(dt[0] * dt[0] + dt[1] * dt[1] + dt[2] * dt[2]);
  double s = fmin(tau, -mu * dn);
  for (int a = 0; a < 3; ++a) out[a] = tau > 0.0 ? dt[a] - s * dt[a] / tau : 0.0;
}

int ora_undesirable(int32_t rule, const double *d, const double *nrm, double mu,
                    double *out) {
  if (!d || !nrm || !out) return ORA_E_INVALID;
  undesirable_v(rule, d, nrm, mu, out);
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* The contact step                                                          */
/* ------------------------------------------------------------------------ */

/*
 * S: the predicted generalized velocity Vbar = {v, C} -> the preferred one
 * Vhat, by the augury-iteration series of Section 2.3 with one operator G for
 * every term:
 *   Vhat_0 = Vbar + G Vbar = H Vbar
 *   for m = 0 .. N-1:
 *     dV      = Vhat_m - Vbar             (always against the input field)
 *     W_{m+1} = {undesirable(dv), dC}     (Section 2.4: all of dB is undesirable;
 *                                          Section 2.3: both or neither)
 *     Vhat_{m+1} = Vhat_m + G W_{m+1} = Vhat_m + H W_{m+1} - W_{m+1}
 * Since C = B D^{-1} with D_p fixed within the step, dC = dB D^{-1} and W's
 * affine part can be carried as C.  Unconstrained particles (no normal) get
 * W = 0.  v and C are overwritten with Vhat.
 *
 * Normals: by default from the body mass fields (compute_normals).  When
 * nrm_in (3n) is given, those normals are used instead -- the paper's n_p is
 * an area-weighted outward normal of the finite-element boundary faces at the
 * node (Section 2.3), which only the caller's mesh knows; a particle whose
 * given normal is exactly zero is unconstrained.
 *
 * Optional outputs: nrm_out (3n) the normals, w1_out (12n) the first series
 * field W_1 (v part then C part), uncon_out (n) the unconstrained flags.
 */
int ora_contact_step(const ora_grid *g, int64_t n, const double *x, double *v,
                     double *C, const double *m, const uint16_t *body,
                     double mu, int32_t n_iter, const double *nrm_in,
                     double *nrm_out, double *w1_out, int32_t *uncon_out) {
  if (!valid_grid(g) || n < 0 || !(mu >= 0.0) || n_iter < 0) return ORA_E_INVALID;
  if (n == 0) return ORA_OK;
  if (!x || !v || !C || !m || !body) return ORA_E_INVALID;
  int rc = check_dense_bounds(g, n, x);
  if (rc) return rc;

  size_t N3 = (size_t)n * 3, N9 = (size_t)n * 9;
  double *Dinv = (double *)malloc(N9 * sizeof(double));
  double *nrm = (double *)malloc(N3 * sizeof(double));
  int32_t *uncon = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  double *vb = (double *)malloc(N3 * sizeof(double)); /* Vbar */
  double *Cb = (double *)malloc(N9 * sizeof(double));
  double *vh = (double *)malloc(N3 * sizeof(double)); /* Vhat */
  double *Ch = (double *)malloc(N9 * sizeof(double));
  double *wv = (double *)malloc(N3 * sizeof(double)); /* W */
  double *wC = (double *)malloc(N9 * sizeof(double));
  double *hv = (double *)malloc(N3 * sizeof(double)); /* H W */
  double *hC = (double *)malloc(N9 * sizeof(double));
  dgrid G = {{0}, {0}, NULL, NULL};
  if (!Dinv || !nrm || !uncon || !vb || !Cb || !vh || !Ch || !wv || !wC || !hv ||
      !hC) {
    rc = ORA_E_NOMEM;
    goto done;
  }
  rc = inverse_inertia_all(g, n, x, Dinv);
  if (rc) goto done;
  if (nrm_in) {
    for (int64_t p = 0; p < n; ++p) {
      int zero = 1;
      for (int d = 0; d < 3; ++d) {
        nrm[d * n + p] = nrm_in[d * n + p];
        zero &= nrm_in[d * n + p] == 0.0;
      }
      uncon[p] = zero;
    }
  } else {
    rc = compute_normals(g, n, x, m, body, nrm, uncon);
    if (rc) goto done;
  }
  rc = shared_grid(g, n, x, &G);
  if (rc) goto done;

  memcpy(vb, v, N3 * sizeof(double));
  memcpy(Cb, C, N9 * sizeof(double));
  rc = apply_H(g, n, x, m, Dinv, vb, Cb, vh, Ch, &G);
  if (rc) goto done;

  for (int32_t it = 0; it < n_iter; ++it) {
    for (int64_t p = 0; p < n; ++p) {
      double d[3], nn[3], wu[3];
      for (int a = 0; a < 3; ++a) {
        d[a] = vh[a * n + p] - vb[a * n + p];
        nn[a] = nrm[a * n + p];
      }
      if (uncon[p]) {
        for (int a = 0; a < 3; ++a) wv[a * n + p] = 0.0;
        for (int k = 0; k < 9; ++k) wC[k * n + p] = 0.0;
        continue;
      }
      undesirable_v(g->rule, d, nn, mu, wu);
      int keep_affine = 1;
      if (g->rule == ORA_RULE_SEPARATE) {
        double dn = d[0] * nn[0] + d[1] * nn[1] + d[2] * nn[2];
        keep_affine = dn > 0.0;
      }
      for (int a = 0; a < 3; ++a) wv[a * n + p] = wu[a];
      for (int k = 0; k < 9; ++k)
        wC[k * n + p] = keep_affine ? Ch[k * n + p] - Cb[k * n + p] : 0.0;
    }
    if (it == 0 && w1_out) {
      memcpy(w1_out, wv, N3 * sizeof(double));
      memcpy(w1_out + N3, wC, N9 * sizeof(double));
    }
    rc = apply_H(g, n, x, m, Dinv, wv, wC, hv, hC, &G);
    if (rc) goto done;
    for (size_t k = 0; k < N3; ++k) vh[k] += hv[k] - wv[k];
    for (size_t k = 0; k < N9; ++k) Ch[k] += hC[k] - wC[k];
  }
  memcpy(v, vh, N3 * sizeof(double));
  memcpy(C, Ch, N9 * sizeof(double));
  if (nrm_out) memcpy(nrm_out, nrm, N3 * sizeof(double));
  if (uncon_out) memcpy(uncon_out, uncon, (size_t)n * sizeof(int32_t));

done:
  dg_free(&G);
  free(Dinv);
  free(nrm);
  free(uncon);
  free(vb);
  free(Cb);
  free(vh);
  free(Ch);
  free(wv);
  free(wC);
  free(hv);
  free(hC);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Momentum, angular momentum and kinetic energy                             */
/* ------------------------------------------------------------------------ */

/*
 * Invariants of H for the quadratic basis (D_p = h^2/2 I):
 *   P = sum m v
 *   L = sum m [ (x - xref) x v + spin ],  spin_k = eps_kab (C D)_ba
 *     = (h^2/2) (C_zy - C_yz, C_xz - C_zx, C_yx - C_xy)
 *   E = 1/2 sum m ( |v|^2 + (h^2/2) |C|_F^2 )
 * The spin term is the angular momentum the affine mode carries onto the grid
 * (sum_i N_i dx_i x (C dx_i)); without it L is not conserved.
 * out[0..2] P, out[3..5] L, out[6] E, out[7] sum m|v|, out[8] the L scale
 * sum m (|x - xref| |v| + (h^2/2) |C|_F).
 */
int ora_momentum(int64_t n, const double *x, const double *v, const double *C,
                 const double *m, double h, const double *xref, double *out) {
  if (n < 0 || !out) return ORA_E_INVALID;
  memset(out, 0, 9 * sizeof(double));
  double k = 0.5 * h * h;
  for (int64_t p = 0; p < n; ++p) {
    double r[3], vv[3], Cp[9];
    for (int a = 0; a < 3; ++a) {
      r[a] = x[a * n + p] - xref[a];
      vv[a] = v[a * n + p];
    }
    for (int a = 0; a < 9; ++a) Cp[a] = C[a * n + p];
    double mp = m[p];
    out[0] += mp * vv[0];
    out[1] += mp * vv[1];
    out[2] += mp * vv[2];
    out[3] += mp * (r[1] * vv[2] - r[2] * vv[1] + k * (Cp[7] - Cp[5]));
    out[4] += mp * (r[2] * vv[0] - r[0] * vv[2] + k * (Cp[2] - Cp[6]));
    out[5] += mp * (r[0] * vv[1] - r[1] * vv[0] + k * (Cp[3] - Cp[1]));
    double v2 = vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2];
    double c2 = 0.0;
    for (int a = 0; a < 9; ++a) c2 += Cp[a] * Cp[a];
    out[6] += 0.5 * mp * (v2 + k * c2);
    double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    out[7] += mp * sqrt(v2);
    out[8] += mp * (rn * sqrt(v2) + k * sqrt(c2));
  }
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Cell keys and the particle order                                          */
/* ------------------------------------------------------------------------ */

/*
 * The particle ordering the GPU library must reproduce bit for bit.  The paper
 * fixes only the base node x_i = h floor(x/h) (Appendix B); the order is this
 * library's own definition:
 *   cell     c_d = floor((x_d - origin_d) / h)   (FP64 division)
 *   block    B_d = floor(c_d / 4)                (4x4x4 cells per block)
 *   pair     S_d = floor(B_d / 2)                (2x2x2 blocks per super block)
 *   body     gb  = body_base[scene] + body_id    (global body number)
 *   each body gets the box [Smin, Smax] of its super blocks, holding
 *   8 * es_x * es_y * es_z block numbers (es = Smax - Smin + 1); the boxes are
 *   laid end to end in global-body order (offset_gb = sum of earlier sizes);
 *   block number = offset_gb
 *                  + 8 ((Sx-Sminx) + es_x ((Sy-Sminy) + es_y (Sz-Sminz)))
 *                  + (Bx mod 2) + 2 (By mod 2) + 4 (Bz mod 2)
 *   key = block number * 64 + (cx mod 4) + 4 (cy mod 4) + 16 (cz mod 4)
 * and the permutation sorts keys ascending, equal keys by input index.  The
 * blocks of one super block of one body are thus consecutive in key order.
 * Keys must fit 32 bits (ORA_E_KEY_OVERFLOW otherwise).
 */
typedef struct {
  uint32_t key;
  uint32_t idx;
} keyidx;

static int cmp_keyidx(const void *A, const void *B) {
  const keyidx *a = (const keyidx *)A, *b = (const keyidx *)B;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

static int64_t floor_div4(int64_t c) { return c >= 0 ? c / 4 : -((-c + 3) / 4); }
static int64_t mod4(int64_t c) { return c - 4 * floor_div4(c); }
static int64_t floor_div2(int64_t c) { return c >= 0 ? c / 2 : -((-c + 1) / 2); }
static int64_t mod2(int64_t c) { return c - 2 * floor_div2(c); }

int ora_cell_keys(int32_t n_scenes, const ora_grid *grids, const int64_t *offsets,
                  const int64_t *counts, const int32_t *body_base,
                  int32_t n_bodies_total, const double *x, int64_t n,
                  const uint16_t *body, uint32_t *keys, uint32_t *perm) {
  if (n_scenes < 0 || n < 0 || n_bodies_total < 0) return ORA_E_INVALID;
  if (n == 0) return ORA_OK;
  int64_t *cell = (int64_t *)malloc((size_t)n * 3 * sizeof(int64_t));
  int64_t *gbody = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int64_t *bmin = (int64_t *)malloc((size_t)n_bodies_total * 3 * sizeof(int64_t));
  int64_t *bmax = (int64_t *)malloc((size_t)n_bodies_total * 3 * sizeof(int64_t));
  int64_t *boff = (int64_t *)malloc((size_t)(n_bodies_total + 1) * sizeof(int64_t));
  keyidx *ki = (keyidx *)malloc((size_t)n * sizeof(keyidx));
  int rc = ORA_OK;
  if (!cell || !gbody || !bmin || !bmax || !boff || !ki) {
    rc = ORA_E_NOMEM;
    goto done;
  }
  for (int64_t b = 0; b < n_bodies_total; ++b)
    for (int d = 0; d < 3; ++d) {
      bmin[3 * b + d] = INT64_MAX;
      bmax[3 * b + d] = INT64_MIN;
    }
  for (int32_t s = 0; s < n_scenes; ++s) {
    const ora_grid *g = &grids[s];
    for (int64_t p = offsets[s]; p < offsets[s] + counts[s]; ++p) {
      int64_t gb = (int64_t)body_base[s] + body[p];
      if (gb >= n_bodies_total) {
        rc = ORA_E_INVALID;
        goto done;
      }
      gbody[p] = gb;
      for (int d = 0; d < 3; ++d) {
        double xi = (x[d * n + p] - g->origin[d]) / g->h;
        double f = floor(xi);
        if (!(f >= -2147483648.0 && f <= 2147483647.0)) {
          rc = ORA_E_OUT_OF_GRID;
          goto done;
        }
        cell[3 * p + d] = (int64_t)f;
        int64_t B = floor_div4(cell[3 * p + d]);
        if (B < bmin[3 * gb + d]) bmin[3 * gb + d] = B;
        if (B > bmax[3 * gb + d]) bmax[3 * gb + d] = B;
      }
    }
  }
  boff[0] = 0;
  for (int64_t b = 0; b < n_bodies_total; ++b) {
    int64_t vol = 0;
    if (bmin[3 * b] <= bmax[3 * b]) {
      vol = 8;
      for (int d = 0; d < 3; ++d)
        vol *= floor_div2(bmax[3 * b + d]) - floor_div2(bmin[3 * b + d]) + 1;
    }
    boff[b + 1] = boff[b] + vol;
  }
  if (boff[n_bodies_total] > ((int64_t)1 << 26)) {
    rc = ORA_E_KEY_OVERFLOW;
    goto done;
  }
  for (int32_t s = 0; s < n_scenes; ++s)
    for (int64_t p = offsets[s]; p < offsets[s] + counts[s]; ++p) {
      int64_t gb = gbody[p];
      int64_t S[3], es[3], sub = 0;
      for (int d = 0; d < 3; ++d) {
        const int64_t B = floor_div4(cell[3 * p + d]);
        const int64_t smin = floor_div2(bmin[3 * gb + d]);
        S[d] = floor_div2(B) - smin;
        es[d] = floor_div2(bmax[3 * gb + d]) - smin + 1;
        sub += mod2(B) << d;
      }
      int64_t lin = boff[gb] + 8 * (S[0] + es[0] * (S[1] + es[1] * S[2])) + sub;
      int64_t cib = mod4(cell[3 * p]) + 4 * mod4(cell[3 * p + 1]) + 16 * mod4(cell[3 * p + 2]);
      ki[p].key = (uint32_t)(lin * 64 + cib);
      ki[p].idx = (uint32_t)p;
    }
  for (int64_t p = 0; p < n; ++p) keys[p] = ki[p].key;
  qsort(ki, (size_t)n, sizeof(keyidx), cmp_keyidx);
  for (int64_t p = 0; p < n; ++p) perm[p] = ki[p].idx;

done:
  free(cell);
  free(gbody);
  free(bmin);
  free(bmax);
  free(boff);
  free(ki);
  return rc;
}
