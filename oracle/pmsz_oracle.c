/*
 * pmsz_oracle.c -- plain CPU oracle for the pMSz topology correction.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * helper with the GPU library: every definition below is written out again
 * from the paper, in the plainest form that still finishes at test sizes.
 *
 * What it computes (pMSz, arXiv 2601.01787):
 *   - the piecewise-linear scalar field on a Freudenthal-triangulated grid and
 *     its extrema (Sec. III-A);
 *   - for every vertex i the steepest-ascent neighbour n_max(i) and the
 *     steepest-descent neighbour n_min(i), as argmax/argmin of the values over
 *     the neighbourhood (Sec. IV-A, definition of n_min / n_max);
 *   - the iterative, decrease-only correction (Sec. III-B Eq. 1, Sec. IV-A
 *     descending and ascending rules, Sec. III-B FPmax rule) until every
 *     vertex's directions match those of the original field;
 *   - ascending / descending segmentation labels by following the steepest
 *     directions to the extremum they end at (Sec. III-A, integral lines);
 *   - the evaluation counts: wrongly labelled points, false maxima / minima
 *     (Sec. V-D);
 *   - the correction of one block of a decomposed domain (Sec. IV-B): the
 *     same loop with the comparisons restricted to the block's core, the
 *     outer ghost layer only providing neighbour values and receiving flags.
 *
 * Readings of points the paper leaves open (all written out in the design doc):
 *   - neighbourhood N*(i) = {i} + the Freudenthal (Kuhn) neighbours, 14 in 3D
 *     and 6 in 2D; no periodic wrap;
 *   - order: a beats b iff h_a > h_b, or h_a == h_b and index a > index b;
 *     n_max is the maximum of N*(i) in that order, n_min the minimum, so a
 *     vertex is a maximum iff n_max(i) == i;
 *   - edit size (delta in Eq. 1, left open by the paper): halve the gap to the
 *     lower bound, i.e. g <- lb + (g - lb)/2, and take lb itself when rounding
 *     would not decrease g;
 *   - Jacobi order: the flag set is computed from g^k alone, then every flagged
 *     vertex gets exactly one edit;
 *   - bounds are exact: lb = RU(f - xi_T), ub = RD(f + xi_T) in the field's
 *     type T, xi_T <= xi.
 *
 * Arithmetic: IEEE-754 binary32 / binary64, round to nearest even, built with
 * -ffp-contract=off and without fast-math, so that no product is fused.
 *
 * Pins (see tests/test_oracle_*.py): explicit-simplex adjacency and closed-form
 * edge counts, path-walking labels on every ordering of a 3x3 grid, exact
 * rational checks of the bounds and the edit, hand examples with dyadic values
 * mirroring the paper's worked cases, and the invariants of Sec. III-B / IV-C.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_F32 = 0, ORC_F64 = 1 };
enum {
  ORC_OK = 0,
  ORC_INVALID = 1,
  ORC_NONFINITE = 2,
  ORC_INPUT_BOUND = 3,
  ORC_NOT_CONVERGED = 4,
  ORC_STALLED = 5,
  ORC_OOM = 6
};

typedef struct {
  int ndim;
  int64_t nx, ny, nz;
} grid_t;

typedef struct {
  int64_t iterations;
  int64_t steps_applied;
  int64_t flagged_final;
  int64_t stalled_flags;
  int64_t mismatch_initial;
  int32_t status;
  int32_t pad;
} orc_stats;

typedef struct {
  int64_t bound_violations;
  int64_t asc_mismatch, desc_mismatch;
  int64_t false_max, false_min, missed_max, missed_min;
  int64_t wrong_max_label, wrong_min_label, wrong_label;
  int64_t vertices_edited;
  double max_abs_err;
} orc_report;

/* ------------------------------------------------------------------------- */
/* Grid and neighbourhood (Sec. III-A: PL field on a triangulated grid).      */
/* ------------------------------------------------------------------------- */

static int grid_ok(const grid_t* G) {
  if (G->ndim != 2 && G->ndim != 3) return 0;
  if (G->nx < 1 || G->ny < 1 || G->nz < 1) return 0;
  if (G->ndim == 2 && G->nz != 1) return 0;
  /* vertex ids are int32 in the label arrays */
  if (G->nx > INT32_MAX || G->ny > INT32_MAX || G->nz > INT32_MAX) return 0;
  if (G->nx * G->ny > INT32_MAX / G->nz) return 0;
  return 1;
}

static int64_t nverts(const grid_t* G) { return G->nx * G->ny * G->nz; }

/* Direction code -> lattice offset.  Code 0 is the vertex itself.  Codes 1..7
 * are the offsets +(bx, by, bz) with (bx, by, bz) the bits of the code (bit 0
 * = x, bit 1 = y, bit 2 = z); codes 9..15 are the negated offsets of code-8.
 * Every offset is a 0/1 vector or its negative: these are the edges of the
 * Kuhn split of each cube into six tetrahedra around its main diagonal (in 2D,
 * the split of each square along (0,0)-(1,1)).  In 2D, codes using the z bit
 * do not exist.  Returns 0 for a code that is not a neighbour in this ndim. */
static int code_offset(int ndim, int code, int* dx, int* dy, int* dz) {
  if (code == 0) { *dx = *dy = *dz = 0; return 1; }
  if (code == 8 || code < 0 || code > 15) return 0;
  int m = code & 7;
  int s = (code & 8) ? -1 : 1;
  if (ndim == 2 && (m & 4)) return 0;
  *dx = s * (m & 1);
  *dy = s * ((m >> 1) & 1);
  *dz = s * ((m >> 2) & 1);
  return 1;
}

/* Neighbour of vertex (x,y,z) along `code`, or -1 when outside the box. */
static int64_t neighbour(const grid_t* G, int64_t x, int64_t y, int64_t z, int code) {
  int dx, dy, dz;
  if (!code_offset(G->ndim, code, &dx, &dy, &dz)) return -1;
  int64_t X = x + dx, Y = y + dy, Z = z + dz;
  if (X < 0 || X >= G->nx || Y < 0 || Y >= G->ny || Z < 0 || Z >= G->nz) return -1;
  return X + G->nx * (Y + G->ny * Z);
}

static double val(const void* h, int dtype, int64_t i) {
  /* float -> double is exact, so comparisons on the widened value are the
   * comparisons of the original binary32 values. */
  return dtype == ORC_F32 ? (double)((const float*)h)[i] : ((const double*)h)[i];
}

/* n_max(i) and n_min(i) over N*(i) (Sec. IV-A), ties broken by vertex index:
 * the larger index wins for the maximum, the smaller for the minimum.  The
 * result is the code of the winning neighbour (0 = i itself). */
static void steepest(const grid_t* G, const void* h, int dtype, int64_t i, int* cmax,
                     int* cmin) {
  int64_t x = i % G->nx, y = (i / G->nx) % G->ny, z = i / (G->nx * G->ny);
  int64_t bmax = i, bmin = i;
  double vmax = val(h, dtype, i), vmin = vmax;
  int kmax = 0, kmin = 0;
  for (int c = 1; c < 16; ++c) {
    int64_t j = neighbour(G, x, y, z, c);
    if (j < 0) continue;
    double v = val(h, dtype, j);
    if (v > vmax || (v == vmax && j > bmax)) { vmax = v; bmax = j; kmax = c; }
    if (v < vmin || (v == vmin && j < bmin)) { vmin = v; bmin = j; kmin = c; }
  }
  *cmax = kmax;
  *cmin = kmin;
}

static int64_t follow(const grid_t* G, int64_t i, int code) {
  int64_t x = i % G->nx, y = (i / G->nx) % G->ny, z = i / (G->nx * G->ny);
  return neighbour(G, x, y, z, code);
}

/* ------------------------------------------------------------------------- */
/* Error bound (Sec. III-B problem statement, Eq. 1): |f - g| <= xi.          */
/* ------------------------------------------------------------------------- */

/* xi in the field's type, never above xi: for binary32 the nearest float,
 * stepped once toward zero when rounding went up. */
static double xi_in_type(int dtype, double xi) {
  if (dtype == ORC_F64) return xi;
  float x = (float)xi;
  if ((double)x > xi) x = nextafterf(x, 0.0f);
  return (double)x;
}

/* Exact sum error by Knuth's TwoSum: a + b == s + e exactly. */
static void two_sum_f(float a, float b, float* s, float* e) {
  float S = a + b, bp = S - a, ap = S - bp;
  *s = S;
  *e = (a - ap) + (b - bp);
}
static void two_sum_d(double a, double b, double* s, double* e) {
  double S = a + b, bp = S - a, ap = S - bp;
  *s = S;
  *e = (a - ap) + (b - bp);
}

/* lb = smallest value of T >= f - xi_T ; ub = largest value of T <= f + xi_T */
static float lower_f(float f, float xi) {
  float s, e;
  two_sum_f(f, -xi, &s, &e);
  if (isinf(s)) return -FLT_MAX;
  if (e > 0) s = nextafterf(s, INFINITY);
  return s;
}
static float upper_f(float f, float xi) {
  float s, e;
  two_sum_f(f, xi, &s, &e);
  if (isinf(s)) return FLT_MAX;
  if (e < 0) s = nextafterf(s, -INFINITY);
  return s;
}
static double lower_d(double f, double xi) {
  double s, e;
  two_sum_d(f, -xi, &s, &e);
  if (isinf(s)) return -DBL_MAX;
  if (e > 0) s = nextafter(s, INFINITY);
  return s;
}
static double upper_d(double f, double xi) {
  double s, e;
  two_sum_d(f, xi, &s, &e);
  if (isinf(s)) return DBL_MAX;
  if (e < 0) s = nextafter(s, -INFINITY);
  return s;
}

/* One edit of Eq. 1 with delta = half of the remaining gap to the lower bound:
 * h = g - lb, m = lb + h/2, result m if that is below g, else lb itself. */
static float edit_f(float g, float lb) {
  float h = g - lb;
  float m = lb + 0.5f * h;
  return (m < g) ? m : lb;
}
static double edit_d(double g, double lb) {
  double h = g - lb;
  double m = lb + 0.5 * h;
  return (m < g) ? m : lb;
}

/* ------------------------------------------------------------------------- */
/* Exported entry points.                                                     */
/* ------------------------------------------------------------------------- */

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

double orc_xi_t(int dtype, double xi) { return xi_in_type(dtype, xi); }

/* Lower and upper bounds per element, in the field's type. */
void orc_bounds(int dtype, const void* f, int64_t n, double xi, void* lb, void* ub) {
  double xt = xi_in_type(dtype, xi);
  for (int64_t i = 0; i < n; ++i) {
    if (dtype == ORC_F32) {
      float fi = ((const float*)f)[i];
      ((float*)lb)[i] = lower_f(fi, (float)xt);
      ((float*)ub)[i] = upper_f(fi, (float)xt);
    } else {
      double fi = ((const double*)f)[i];
      ((double*)lb)[i] = lower_d(fi, xt);
      ((double*)ub)[i] = upper_d(fi, xt);
    }
  }
}

/* The single edit rule, exposed so that tests can pin it against rationals. */
void orc_edit(int dtype, const void* g, const void* lb, int64_t n, void* out) {
  for (int64_t i = 0; i < n; ++i) {
    if (dtype == ORC_F32)
      ((float*)out)[i] = edit_f(((const float*)g)[i], ((const float*)lb)[i]);
    else
      ((double*)out)[i] = edit_d(((const double*)g)[i], ((const double*)lb)[i]);
  }
}

/* Directions of a field: low nibble = code of n_max(i), high nibble = code of
 * n_min(i), both over N*(i). */
int orc_directions(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* h,
                   uint8_t* dirs) {
  grid_t G = {ndim, nx, ny, nz};
  if (!grid_ok(&G)) return ORC_INVALID;
  int64_t n = nverts(&G);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int a, d;
    steepest(&G, h, dtype, i, &a, &d);
    dirs[i] = (uint8_t)(a | (d << 4));
  }
  return ORC_OK;
}

/* Directions at selected vertices only (for sampled checks of large fields). */
int orc_directions_at(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* h,
                      const int64_t* idx, int64_t m, uint8_t* out) {
  grid_t G = {ndim, nx, ny, nz};
  if (!grid_ok(&G)) return ORC_INVALID;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    int a, d;
    steepest(&G, h, dtype, idx[k], &a, &d);
    out[k] = (uint8_t)(a | (d << 4));
  }
  return ORC_OK;
}

/* Validation of the inputs (problem statement of Sec. III-B): finite values and
 * |f - fhat| <= xi in the exact sense lb <= fhat <= ub. */
int orc_validate(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* f,
                 const void* fhat, double xi) {
  grid_t G = {ndim, nx, ny, nz};
  if (!grid_ok(&G) || (dtype != ORC_F32 && dtype != ORC_F64)) return ORC_INVALID;
  if (!isfinite(xi) || xi < 0) return ORC_INVALID;
  int64_t n = nverts(&G);
  double xt = xi_in_type(dtype, xi);
  int64_t nonfinite = 0, outside = 0;
#pragma omp parallel for reduction(+ : nonfinite, outside)
  for (int64_t i = 0; i < n; ++i) {
    if (dtype == ORC_F32) {
      float a = ((const float*)f)[i], b = ((const float*)fhat)[i];
      if (!isfinite(a) || !isfinite(b)) { nonfinite++; continue; }
      if (b < lower_f(a, (float)xt) || b > upper_f(a, (float)xt)) outside++;
    } else {
      double a = ((const double*)f)[i], b = ((const double*)fhat)[i];
      if (!isfinite(a) || !isfinite(b)) { nonfinite++; continue; }
      if (b < lower_d(a, xt) || b > upper_d(a, xt)) outside++;
    }
  }
  if (nonfinite) return ORC_NONFINITE;
  if (outside) return ORC_INPUT_BOUND;
  return ORC_OK;
}

/* The flag set of one iteration, from g alone (Sec. IV-A):
 *   - ascending rule / FPmax: if n_max under g differs from n_max under f,
 *     flag the vertex that is now the steepest-ascent neighbour (the spurious
 *     maximum; for a false maximum that is i itself);
 *   - descending rule: if n_min under g differs from n_min under f, flag the
 *     original steepest-descent neighbour so that it is lowered below the
 *     rival.
 * flags[t] = 1 for every flagged t.  Returns the number of mismatching
 * (vertex, direction) pairs. */
/* Is vertex i inside the box core = {x0, x1, y0, y1, z0, z1} (half-open)? */
static int in_box(const grid_t* G, int64_t i, const int64_t* core) {
  int64_t x = i % G->nx, y = (i / G->nx) % G->ny, z = i / (G->nx * G->ny);
  return x >= core[0] && x < core[1] && y >= core[2] && y < core[3] && z >= core[4] &&
         z < core[5];
}

/* orc_flags with the comparisons restricted to the vertices of `core` (the
 * targets they flag may lie anywhere). */
static int64_t flags_core(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype,
                          const void* g, const uint8_t* dirs_f, uint8_t* flags,
                          const int64_t* core) {
  grid_t G = {ndim, nx, ny, nz};
  int64_t n = nverts(&G);
  int32_t* ag = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* dg = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!ag || !dg) { free(ag); free(dg); return -1; }
  /* phase 1: directions of g^k for every vertex */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int a, d;
    steepest(&G, g, dtype, i, &a, &d);
    ag[i] = (int32_t)follow(&G, i, a);
    dg[i] = (int32_t)follow(&G, i, d);
  }
  /* phase 2: collect the targets */
  memset(flags, 0, (size_t)n);
  int64_t mism = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!in_box(&G, i, core)) continue;
    int64_t af = follow(&G, i, dirs_f[i] & 15);
    int64_t df = follow(&G, i, dirs_f[i] >> 4);
    if (ag[i] != af) { flags[ag[i]] = 1; mism++; }
    if (dg[i] != df) { flags[df] = 1; mism++; }
  }
  free(ag);
  free(dg);
  return mism;
}

int64_t orc_flags(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* g,
                  const uint8_t* dirs_f, uint8_t* flags) {
  const int64_t all[6] = {0, nx, 0, ny, 0, nz};
  return flags_core(ndim, nx, ny, nz, dtype, g, dirs_f, flags, all);
}

/* Targeted edit (the variant of Sec. IV-A's worked examples, where a spurious
 * maximum is lowered to its rival's value "or slightly below" instead of by a
 * fixed step).  Every flag carries a proposed value for its target: the
 * largest value at which the target no longer beats its rival in the (value,
 * index) order --
 *   ascending rule  (n_max under g is t, under f it is c != t): rival c;
 *   descending rule (n_min under f is t, under g it is r != t): rival r;
 *   proposal = g[rival] when t < rival (the tie then goes to the rival), else
 *   the next value below g[rival]; a zero proposal is +0.
 * prop[t] receives the smallest proposal for t (+inf where none); flags and
 * the return value are those of orc_flags. */
static double next_below(int dtype, double v) {
  return dtype == ORC_F32 ? (double)nextafterf((float)v, -INFINITY) : nextafter(v, -INFINITY);
}

static int64_t flags_targeted_core(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype,
                                   const void* g, const uint8_t* dirs_f, uint8_t* flags,
                                   double* prop, const int64_t* core) {
  grid_t G = {ndim, nx, ny, nz};
  int64_t n = nverts(&G);
  int32_t* ag = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* dg = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!ag || !dg) { free(ag); free(dg); return -1; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int a, d;
    steepest(&G, g, dtype, i, &a, &d);
    ag[i] = (int32_t)follow(&G, i, a);
    dg[i] = (int32_t)follow(&G, i, d);
  }
  memset(flags, 0, (size_t)n);
  for (int64_t t = 0; t < n; ++t) prop[t] = INFINITY;
  int64_t mism = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!in_box(&G, i, core)) continue;
    int64_t af = follow(&G, i, dirs_f[i] & 15);
    int64_t df = follow(&G, i, dirs_f[i] >> 4);
    int64_t t = -1, rival = -1;
    for (int rule = 0; rule < 2; ++rule) {
      if (rule == 0) {
        if (ag[i] == af) continue;
        t = ag[i];
        rival = af;
      } else {
        if (dg[i] == df) continue;
        t = df;
        rival = dg[i];
      }
      mism++;
      flags[t] = 1;
      double rv = val(g, dtype, rival);
      double p = t < rival ? rv : next_below(dtype, rv);
      if (p == 0.0) p = 0.0; /* +0 */
      if (p < prop[t]) prop[t] = p;
    }
  }
  free(ag);
  free(dg);
  return mism;
}

int64_t orc_flags_targeted(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype,
                           const void* g, const uint8_t* dirs_f, uint8_t* flags, double* prop) {
  const int64_t all[6] = {0, nx, 0, ny, 0, nz};
  return flags_targeted_core(ndim, nx, ny, nz, dtype, g, dirs_f, flags, prop, all);
}

/* The correction loop.  g holds fhat on entry and the last iterate on exit.
 *   k = 0
 *   repeat: F = flags(g^k)
 *           F empty                   -> OK, iterations = k
 *           every t in F has g_t = lb -> STALLED (no edit can act)
 *           k == max_iters            -> NOT_CONVERGED
 *           g_t <- edit(g_t) for t in F, simultaneously; k += 1
 * dirs_f may be NULL (then computed here).  Only the vertices of `core`
 * ({x0, x1, y0, y1, z0, z1}, half-open) are compared; the whole grid for a
 * single field, a block's core for a decomposed domain. */
int orc_correct_core(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* f,
                     void* g, double xi, const uint8_t* dirs_f_in, int64_t max_iters,
                     int mode, const int64_t* core, orc_stats* st) {
  memset(st, 0, sizeof(*st));
  int s = orc_validate(ndim, nx, ny, nz, dtype, f, g, xi);
  if (s == ORC_OK && max_iters < 0) s = ORC_INVALID;
  if (s != ORC_OK) { st->status = s; return s; }
  grid_t G = {ndim, nx, ny, nz};
  int64_t n = nverts(&G);
  double xt = xi_in_type(dtype, xi);
  uint8_t* dirs_f = (uint8_t*)dirs_f_in;
  uint8_t* own = NULL;
  if (!dirs_f) {
    own = (uint8_t*)malloc((size_t)n);
    if (!own) { st->status = ORC_OOM; return ORC_OOM; }
    orc_directions(ndim, nx, ny, nz, dtype, f, own);
    dirs_f = own;
  }
  uint8_t* flags = (uint8_t*)malloc((size_t)n);
  double* prop = mode ? (double*)malloc(sizeof(double) * (size_t)n) : NULL;
  if (!flags || (mode && !prop)) {
    free(flags);
    free(prop);
    free(own);
    st->status = ORC_OOM;
    return ORC_OOM;
  }
  int64_t k = 0;
  int status;
  for (;;) {
    int64_t mism = mode ? flags_targeted_core(ndim, nx, ny, nz, dtype, g, dirs_f, flags, prop,
                                              core)
                        : flags_core(ndim, nx, ny, nz, dtype, g, dirs_f, flags, core);
    if (mism < 0) { status = ORC_OOM; break; }
    if (k == 0) st->mismatch_initial = mism;
    int64_t nflag = 0, at_lb = 0;
#pragma omp parallel for reduction(+ : nflag, at_lb)
    for (int64_t t = 0; t < n; ++t) {
      if (!flags[t]) continue;
      nflag++;
      if (dtype == ORC_F32) {
        float lb = lower_f(((const float*)f)[t], (float)xt);
        if (!(((float*)g)[t] > lb)) at_lb++;
      } else {
        double lb = lower_d(((const double*)f)[t], xt);
        if (!(((double*)g)[t] > lb)) at_lb++;
      }
    }
    st->flagged_final = nflag;
    st->stalled_flags = at_lb;
    if (nflag == 0) { status = ORC_OK; break; }
    if (at_lb == nflag) { status = ORC_STALLED; break; }
    if (k == max_iters) { status = ORC_NOT_CONVERGED; break; }
    int64_t changed = 0;
#pragma omp parallel for reduction(+ : changed)
    for (int64_t t = 0; t < n; ++t) {
      if (!flags[t]) continue;
      if (dtype == ORC_F32) {
        float* gt = (float*)g + t;
        float lb = lower_f(((const float*)f)[t], (float)xt);
        float nv = mode ? ((float)prop[t] > lb ? (float)prop[t] : lb) : edit_f(*gt, lb);
        if (nv != *gt) changed++;
        *gt = nv;
      } else {
        double* gt = (double*)g + t;
        double lb = lower_d(((const double*)f)[t], xt);
        double nv = mode ? (prop[t] > lb ? prop[t] : lb) : edit_d(*gt, lb);
        if (nv != *gt) changed++;
        *gt = nv;
      }
    }
    st->steps_applied += changed;
    k++;
  }
  st->iterations = k;
  st->status = status;
  free(flags);
  free(prop);
  free(own);
  return status;
}

int orc_correct_mode(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* f,
                     void* g, double xi, const uint8_t* dirs_f_in, int64_t max_iters,
                     int mode, orc_stats* st) {
  const int64_t all[6] = {0, nx, 0, ny, 0, nz};
  return orc_correct_core(ndim, nx, ny, nz, dtype, f, g, xi, dirs_f_in, max_iters, mode, all,
                          st);
}

/* The correction with the halving edit of Eq. 1 (mode 0). */
int orc_correct(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* f,
                void* g, double xi, const uint8_t* dirs_f_in, int64_t max_iters,
                orc_stats* st) {
  return orc_correct_mode(ndim, nx, ny, nz, dtype, f, g, xi, dirs_f_in, max_iters, 0, st);
}

/* Label of vertex i: walk the steepest direction (low nibble = ascending, high
 * nibble = descending) until a vertex points at itself; that extremum's index
 * is the label (Sec. III-A, integral lines and segmentations). */
static int64_t walk(const grid_t* G, const uint8_t* dirs, int64_t i, int shift) {
  for (;;) {
    int c = (dirs[i] >> shift) & 15;
    if (c == 0) return i;
    i = follow(G, i, c);
  }
}

int orc_labels(int ndim, int64_t nx, int64_t ny, int64_t nz, const uint8_t* dirs,
               int32_t* max_label, int32_t* min_label) {
  grid_t G = {ndim, nx, ny, nz};
  if (!grid_ok(&G)) return ORC_INVALID;
  int64_t n = nverts(&G);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    if (max_label) max_label[i] = (int32_t)walk(&G, dirs, i, 0);
    if (min_label) min_label[i] = (int32_t)walk(&G, dirs, i, 4);
  }
  return ORC_OK;
}

/* Labels at selected vertices, with the directions computed on the fly from
 * the field while walking (no full direction array needed). */
int orc_labels_at(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* h,
                  const int64_t* idx, int64_t m, int32_t* max_label, int32_t* min_label) {
  grid_t G = {ndim, nx, ny, nz};
  if (!grid_ok(&G)) return ORC_INVALID;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < m; ++k) {
    int a, d;
    int64_t i = idx[k];
    for (;;) {
      steepest(&G, h, dtype, i, &a, &d);
      if (a == 0) break;
      i = follow(&G, i, a);
    }
    max_label[k] = (int32_t)i;
    i = idx[k];
    for (;;) {
      steepest(&G, h, dtype, i, &a, &d);
      if (d == 0) break;
      i = follow(&G, i, d);
    }
    min_label[k] = (int32_t)i;
  }
  return ORC_OK;
}

/* Evaluation counts of Sec. V-D, recomputed from (f, g) from scratch. */
int orc_verify(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* f,
               const void* g, const void* fhat, double xi, orc_report* r) {
  memset(r, 0, sizeof(*r));
  grid_t G = {ndim, nx, ny, nz};
  if (!grid_ok(&G) || !isfinite(xi) || xi < 0) return ORC_INVALID;
  int64_t n = nverts(&G);
  double xt = xi_in_type(dtype, xi);
  uint8_t* df = (uint8_t*)malloc((size_t)n);
  uint8_t* dg = (uint8_t*)malloc((size_t)n);
  int32_t* lf = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n);
  int32_t* lg = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n);
  if (!df || !dg || !lf || !lg) {
    free(df); free(dg); free(lf); free(lg);
    return ORC_OOM;
  }
  orc_directions(ndim, nx, ny, nz, dtype, f, df);
  orc_directions(ndim, nx, ny, nz, dtype, g, dg);
  orc_labels(ndim, nx, ny, nz, df, lf, lf + n);
  orc_labels(ndim, nx, ny, nz, dg, lg, lg + n);
  int64_t bv = 0, am = 0, dm = 0, fmax = 0, fmin = 0, mmax = 0, mmin = 0, wl = 0, wu = 0,
          wb = 0, ed = 0;
  double err = 0.0;
#pragma omp parallel for reduction(+ : bv, am, dm, fmax, fmin, mmax, mmin, wl, wu, wb, ed) \
    reduction(max : err)
  for (int64_t i = 0; i < n; ++i) {
    double fi = val(f, dtype, i), gi = val(g, dtype, i);
    int inside;
    if (dtype == ORC_F32) {
      float a = (float)fi, b = (float)gi;
      inside = isfinite(b) && b >= lower_f(a, (float)xt) && b <= upper_f(a, (float)xt);
    } else {
      inside = isfinite(gi) && gi >= lower_d(fi, xt) && gi <= upper_d(fi, xt);
    }
    if (!inside) bv++;
    double e = fabs(gi - fi);
    if (e > err || isnan(e)) err = isnan(e) ? INFINITY : e;
    int af = df[i] & 15, ag = dg[i] & 15, nf = df[i] >> 4, ng = dg[i] >> 4;
    if (af != ag) am++;
    if (nf != ng) dm++;
    if (ag == 0 && af != 0) fmax++;
    if (af == 0 && ag != 0) mmax++;
    if (ng == 0 && nf != 0) fmin++;
    if (nf == 0 && ng != 0) mmin++;
    int w1 = lf[i] != lg[i], w2 = lf[n + i] != lg[n + i];
    wu += w1;
    wl += w2;
    wb += (w1 || w2);
    if (fhat && val(fhat, dtype, i) != gi) ed++;
  }
  r->bound_violations = bv;
  r->asc_mismatch = am;
  r->desc_mismatch = dm;
  r->false_max = fmax;
  r->false_min = fmin;
  r->missed_max = mmax;
  r->missed_min = mmin;
  r->wrong_max_label = wu;
  r->wrong_min_label = wl;
  r->wrong_label = wb;
  r->vertices_edited = fhat ? ed : -1;
  r->max_abs_err = err;
  free(df); free(dg); free(lf); free(lg);
  return ORC_OK;
}
