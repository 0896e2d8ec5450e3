/* Driver for the sanitizer check of the CPU oracle: runs every entry point on
 * small seeded fields (2D and 3D, binary32 and binary64, halving and targeted
 * edits, a core box) so that AddressSanitizer / UndefinedBehaviorSanitizer
 * builds of the oracle exercise their code.  Exit status 0 when every call
 * returned and the corrections converged. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t iterations, steps_applied, flagged_final, stalled_flags, mismatch_initial;
  int32_t status, pad;
} orc_stats;
typedef struct {
  int64_t c[11];
  double max_abs_err;
} orc_report;

double orc_xi_t(int dtype, double xi);
void orc_bounds(int dtype, const void* f, int64_t n, double xi, void* lb, void* ub);
int orc_directions(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* h,
                   uint8_t* dirs);
int orc_correct_mode(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* f,
                     void* g, double xi, const uint8_t* dirs_f, int64_t max_iters, int mode,
                     orc_stats* st);
int orc_correct_core(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* f,
                     void* g, double xi, const uint8_t* dirs_f, int64_t max_iters, int mode,
                     const int64_t* core, orc_stats* st);
int orc_labels(int ndim, int64_t nx, int64_t ny, int64_t nz, const uint8_t* dirs,
               int32_t* max_label, int32_t* min_label);
int orc_verify(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, const void* f,
               const void* g, const void* fhat, double xi, orc_report* r);

static uint64_t rng = 88172645463325252ull;
static double uni(void) {  /* xorshift64 */
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int run(int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, int mode) {
  const int64_t n = nx * ny * nz;
  const size_t s = dtype ? 8 : 4;
  const double xi = 0.05;
  void* f = malloc(n * s);
  void* fh = malloc(n * s);
  void* g = malloc(n * s);
  void* lb = malloc(n * s);
  void* ub = malloc(n * s);
  uint8_t* d = malloc(n);
  int32_t* mx = malloc(n * 4);
  int32_t* mn = malloc(n * 4);
  for (int64_t i = 0; i < n; ++i) {
    const double v = uni();
    if (dtype) ((double*)f)[i] = v; else ((float*)f)[i] = (float)v;
  }
  orc_bounds(dtype, f, n, xi, lb, ub);
  for (int64_t i = 0; i < n; ++i) {
    const double t = uni();
    if (dtype) {
      const double l = ((double*)lb)[i], u = ((double*)ub)[i];
      ((double*)fh)[i] = l + t * (u - l);
    } else {
      const float l = ((float*)lb)[i], u = ((float*)ub)[i];
      float v = (float)((double)l + t * ((double)u - l));
      if (v < l) v = l;
      if (v > u) v = u;
      ((float*)fh)[i] = v;
    }
  }
  int bad = 0;
  orc_stats st;
  orc_report rep;
  bad |= orc_directions(ndim, nx, ny, nz, dtype, f, d) != 0;
  memcpy(g, fh, n * s);
  bad |= orc_correct_mode(ndim, nx, ny, nz, dtype, f, g, xi, d, 1 << 20, mode, &st) != 0;
  bad |= orc_labels(ndim, nx, ny, nz, d, mx, mn) != 0;
  bad |= orc_verify(ndim, nx, ny, nz, dtype, f, g, fh, xi, &rep) != 0;
  const int64_t core[6] = {nx > 2 ? 1 : 0, nx > 2 ? nx - 1 : nx, ny > 2 ? 1 : 0,
                           ny > 2 ? ny - 1 : ny, 0, nz};
  memcpy(g, fh, n * s);
  bad |= orc_correct_core(ndim, nx, ny, nz, dtype, f, g, xi, NULL, 1 << 20, mode, core, &st) != 0;
  free(f); free(fh); free(g); free(lb); free(ub); free(d); free(mx); free(mn);
  return bad;
}

int main(void) {
  int bad = 0;
  for (int dtype = 0; dtype < 2; ++dtype)
    for (int mode = 0; mode < 2; ++mode) {
      bad |= run(2, 37, 23, 1, dtype, mode);
      bad |= run(3, 9, 7, 11, dtype, mode);
      bad |= run(3, 1, 5, 6, dtype, mode);
    }
  printf(bad ? "FAILED\n" : "ok\n");
  return bad;
}
