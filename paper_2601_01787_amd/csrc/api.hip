// api.hip -- the C ABI of libpmsz: argument checks, workspace layout, the
// host side of the correction loop, labels and verification.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "launch.hpp"

using namespace pmsz;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(PMSZ_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int check_grid(const pmsz_grid* g) {
  if (!g) return fail(PMSZ_ERR_INVALID_ARG, "grid is NULL");
  if (g->ndim != 2 && g->ndim != 3)
    return fail(PMSZ_ERR_INVALID_ARG, "ndim must be 2 or 3 (got %d)", g->ndim);
  if (g->dtype != PMSZ_F32 && g->dtype != PMSZ_F64)
    return fail(PMSZ_ERR_INVALID_ARG, "dtype must be PMSZ_F32 or PMSZ_F64 (got %d)", g->dtype);
  if (g->nx < 1 || g->ny < 1 || g->nz < 1)
    return fail(PMSZ_ERR_INVALID_ARG, "extents must be >= 1");
  if (g->ndim == 2 && g->nz != 1) return fail(PMSZ_ERR_INVALID_ARG, "a 2D grid needs nz == 1");
  const int64_t lim = 2147483647LL;
  if (g->nx > lim || g->ny > lim || g->nz > lim || g->nx * g->ny > lim / g->nz)
    return fail(PMSZ_ERR_INVALID_ARG, "nx*ny*nz must be below 2^31");
  return PMSZ_OK;
}

// xi in the field type, never above xi.
double xi_in_type(int dtype, double xi) {
  if (dtype == PMSZ_F64) return xi;
  float x = (float)xi;
  if ((double)x > xi) x = nextafterf(x, 0.0f);
  return (double)x;
}

struct CorrectLayout {
  size_t ctl, bm, dirs, total;
};
CorrectLayout correct_layout(const Geo& G) {
  CorrectLayout L;
  L.ctl = 0;
  L.bm = align_up(sizeof(Ctl));
  L.dirs = L.bm + align_up((size_t)bitmap_words(G.n) * 4);
  L.total = L.dirs + align_up((size_t)G.n);
  return L;
}

struct VerifyLayout {
  size_t counts, df, dg, lfx, lfn, lgx, lgn, flag, total;
};
VerifyLayout verify_layout(const Geo& G) {
  VerifyLayout L;
  const size_t n = (size_t)G.n;
  L.counts = 0;
  L.df = align_up(sizeof(VerifyCounts));
  L.dg = L.df + align_up(n);
  L.lfx = L.dg + align_up(n);
  L.lfn = L.lfx + align_up(4 * n);
  L.lgx = L.lfn + align_up(4 * n);
  L.lgn = L.lgx + align_up(4 * n);
  L.flag = L.lgn + align_up(4 * n);
  L.total = L.flag + kAlign;
  return L;
}

// Per-thread pinned slots for reading the control block back while the next
// rounds are already queued.
struct HostSlots {
  Ctl* pinned = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int ok = 0;
  ~HostSlots() {
    if (pinned) (void)hipHostFree(pinned);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};
thread_local HostSlots t_slots;

int host_slots(HostSlots** out) {
  HostSlots& s = t_slots;
  if (!s.ok) {
    HIP_TRY(hipHostMalloc((void**)&s.pinned, 2 * sizeof(Ctl), hipHostMallocDefault));
    for (auto& e : s.ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    s.ok = 1;
  }
  *out = &s;
  return PMSZ_OK;
}

int rounds_per_poll() {
  static int v = [] {
    const char* e = getenv("PMSZ_ROUNDS_PER_POLL");
    int r = e ? atoi(e) : 4;
    return r < 1 ? 1 : (r > 64 ? 64 : r);
  }();
  return v;
}

int label_pass(int32_t* lab, int64_t n, unsigned int* flag, hipStream_t s) {
  unsigned int h = 1;
  for (int round = 0; round < 64 && h; ++round) {
    HIP_TRY(hipMemsetAsync(flag, 0, sizeof(unsigned int), s));
    HIP_TRY(launch_labels_jump(lab, n, flag, s));
    HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (h) return fail(PMSZ_ERR_DEVICE, "label propagation did not settle");
  return PMSZ_OK;
}

int labels_impl(const Geo& G, const uint8_t* dirs, int32_t* lmax, int32_t* lmin,
                unsigned int* flag, hipStream_t s) {
  HIP_TRY(launch_labels_init(dirs, G, lmax, lmin, s));
  if (lmax) {
    int r = label_pass(lmax, G.n, flag, s);
    if (r) return r;
  }
  if (lmin) {
    int r = label_pass(lmin, G.n, flag, s);
    if (r) return r;
  }
  return PMSZ_OK;
}

}  // namespace

extern "C" {

const char* pmsz_status_string(int status) {
  switch (status) {
    case PMSZ_OK: return "OK";
    case PMSZ_ERR_INVALID_ARG: return "INVALID_ARG";
    case PMSZ_ERR_NONFINITE: return "NONFINITE";
    case PMSZ_ERR_INPUT_BOUND: return "INPUT_BOUND";
    case PMSZ_ERR_NOT_CONVERGED: return "NOT_CONVERGED";
    case PMSZ_ERR_STALLED: return "STALLED";
    case PMSZ_ERR_OOM: return "OOM";
    case PMSZ_ERR_DEVICE: return "DEVICE";
    default: return "UNKNOWN";
  }
}

const char* pmsz_last_error(void) { return g_last_error.c_str(); }

int pmsz_workspace_size(const pmsz_grid* grid, int op, size_t* bytes) {
  int r = check_grid(grid);
  if (r) return r;
  if (!bytes) return fail(PMSZ_ERR_INVALID_ARG, "bytes is NULL");
  const Geo G = make_geo(*grid);
  switch (op) {
    case PMSZ_WS_CORRECT: *bytes = correct_layout(G).total; break;
    case PMSZ_WS_VERIFY: *bytes = verify_layout(G).total; break;
    case PMSZ_WS_LABELS: *bytes = kAlign; break;
    default: return fail(PMSZ_ERR_INVALID_ARG, "unknown workspace kind %d", op);
  }
  return PMSZ_OK;
}

int pmsz_directions(const pmsz_grid* grid, const void* field, uint8_t* dirs, void* stream) {
  int r = check_grid(grid);
  if (r) return r;
  if (!field || !dirs) return fail(PMSZ_ERR_INVALID_ARG, "NULL array");
  const Geo G = make_geo(*grid);
  HIP_TRY(launch_dirs(grid->dtype, field, G, dirs, (hipStream_t)stream));
  return PMSZ_OK;
}

int pmsz_correct(const pmsz_grid* grid, const void* f, void* g, double xi,
                 const uint8_t* dirs_f, void* ws, size_t ws_bytes, int64_t max_iters,
                 pmsz_stats* stats, void* stream) {
  int r = check_grid(grid);
  if (r) return r;
  if (!f || !g || !ws || !stats) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (!isfinite(xi) || xi < 0) return fail(PMSZ_ERR_INVALID_ARG, "xi must be finite and >= 0");
  if (max_iters < 0) return fail(PMSZ_ERR_INVALID_ARG, "max_iters must be >= 0");
  if ((uintptr_t)ws % kAlign) return fail(PMSZ_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  const Geo G = make_geo(*grid);
  const CorrectLayout L = correct_layout(G);
  if (ws_bytes < L.total)
    return fail(PMSZ_ERR_OOM, "workspace %zu bytes, need %zu", ws_bytes, L.total);
  memset(stats, 0, sizeof(*stats));
  HostSlots* hs;
  if ((r = host_slots(&hs))) return r;

  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  Ctl* ctl = (Ctl*)(base + L.ctl);
  uint32_t* bm = (uint32_t*)(base + L.bm);
  const double xt = xi_in_type(grid->dtype, xi);
  const int dt = grid->dtype;

  HIP_TRY(launch_init(ctl, bm, bitmap_words(G.n), s));
  if (!dirs_f) {
    uint8_t* d = (uint8_t*)(base + L.dirs);
    HIP_TRY(launch_dirs(dt, f, G, d, s));
    dirs_f = d;
  }
  HIP_TRY(launch_validate(dt, f, g, G.n, xt, ctl, s));

  // Rounds are queued in groups; the control block of group j is read while
  // group j+1 runs.  Rounds queued after the run ended return at once.
  // Every round either ends the run or applies one edit round, so a run that
  // is not done after R rounds must report k == R; anything else means the
  // control block is broken and the loop stops instead of spinning.
  const int K = rounds_per_poll();
  int slot = 0, have_prev = 0;
  long long queued = 0, queued_at[2] = {0, 0};
  const Ctl* fin = nullptr;
  for (;;) {
    for (int k = 0; k < K; ++k) {
      HIP_TRY(launch_detect(dt, g, G, dirs_f, bm, ctl, s));
      HIP_TRY(launch_apply(dt, f, g, G, bm, xt, ctl, max_iters, s));
    }
    queued += K;
    queued_at[slot] = queued;
    HIP_TRY(hipMemcpyAsync(&hs->pinned[slot], ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(hs->ev[slot], s));
    if (have_prev) {
      const int p = slot ^ 1;
      HIP_TRY(hipEventSynchronize(hs->ev[p]));
      if (hs->pinned[p].done) {
        fin = &hs->pinned[p];
        break;
      }
      if ((long long)hs->pinned[p].k != queued_at[p]) {
        (void)hipStreamSynchronize(s);
        return fail(PMSZ_ERR_DEVICE, "control block inconsistent: k=%llu after %lld rounds",
                    hs->pinned[p].k, queued_at[p]);
      }
    }
    have_prev = 1;
    slot ^= 1;
  }
  HIP_TRY(hipStreamSynchronize(s));
  stats->iterations = (int64_t)fin->k;
  stats->steps_applied = (int64_t)fin->steps;
  stats->flagged_final = (int64_t)fin->flagged_final;
  stats->stalled_flags = (int64_t)fin->stalled_final;
  stats->mismatch_initial = (int64_t)fin->mism0;
  stats->status = fin->status;
  if (fin->status == PMSZ_ERR_NONFINITE || fin->status == PMSZ_ERR_INPUT_BOUND) {
    stats->iterations = 0;
    stats->steps_applied = 0;
    stats->flagged_final = 0;
    stats->stalled_flags = 0;
    stats->mismatch_initial = 0;
    return fail(fin->status, "%s: %llu non-finite, %llu outside the bound",
                pmsz_status_string(fin->status), fin->bad_nonfinite, fin->bad_bound);
  }
  if (fin->status != PMSZ_OK)
    return fail(fin->status, "%s after %lld rounds", pmsz_status_string(fin->status),
                (long long)fin->k);
  return PMSZ_OK;
}

int pmsz_labels(const pmsz_grid* grid, const uint8_t* dirs, int32_t* max_label,
                int32_t* min_label, void* ws, size_t ws_bytes, void* stream) {
  int r = check_grid(grid);
  if (r) return r;
  if (!dirs || !ws) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (ws_bytes < kAlign) return fail(PMSZ_ERR_OOM, "labels workspace needs %zu bytes", kAlign);
  const Geo G = make_geo(*grid);
  return labels_impl(G, dirs, max_label, min_label, (unsigned int*)ws, (hipStream_t)stream);
}

int pmsz_verify(const pmsz_grid* grid, const void* f, const void* g, const void* fhat,
                double xi, void* ws, size_t ws_bytes, pmsz_report* report, void* stream) {
  int r = check_grid(grid);
  if (r) return r;
  if (!f || !g || !ws || !report) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (!isfinite(xi) || xi < 0) return fail(PMSZ_ERR_INVALID_ARG, "xi must be finite and >= 0");
  if ((uintptr_t)ws % kAlign) return fail(PMSZ_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  const Geo G = make_geo(*grid);
  const VerifyLayout L = verify_layout(G);
  if (ws_bytes < L.total)
    return fail(PMSZ_ERR_OOM, "workspace %zu bytes, need %zu", ws_bytes, L.total);
  hipStream_t s = (hipStream_t)stream;
  char* b = (char*)ws;
  VerifyCounts* vc = (VerifyCounts*)(b + L.counts);
  uint8_t* df = (uint8_t*)(b + L.df);
  uint8_t* dg = (uint8_t*)(b + L.dg);
  int32_t *lfx = (int32_t*)(b + L.lfx), *lfn = (int32_t*)(b + L.lfn);
  int32_t *lgx = (int32_t*)(b + L.lgx), *lgn = (int32_t*)(b + L.lgn);
  unsigned int* flag = (unsigned int*)(b + L.flag);
  HIP_TRY(hipMemsetAsync(vc, 0, sizeof(VerifyCounts), s));
  HIP_TRY(launch_dirs(grid->dtype, f, G, df, s));
  HIP_TRY(launch_dirs(grid->dtype, g, G, dg, s));
  if ((r = labels_impl(G, df, lfx, lfn, flag, s))) return r;
  if ((r = labels_impl(G, dg, lgx, lgn, flag, s))) return r;
  HIP_TRY(launch_verify(grid->dtype, f, g, fhat, G.n, xi_in_type(grid->dtype, xi), df, dg, lfx,
                        lfn, lgx, lgn, vc, s));
  VerifyCounts h;
  HIP_TRY(hipMemcpyAsync(&h, vc, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  report->bound_violations = (int64_t)h.c[0];
  report->asc_mismatch = (int64_t)h.c[1];
  report->desc_mismatch = (int64_t)h.c[2];
  report->false_max = (int64_t)h.c[3];
  report->false_min = (int64_t)h.c[4];
  report->missed_max = (int64_t)h.c[5];
  report->missed_min = (int64_t)h.c[6];
  report->wrong_max_label = (int64_t)h.c[7];
  report->wrong_min_label = (int64_t)h.c[8];
  report->wrong_label = (int64_t)h.c[9];
  report->vertices_edited = fhat ? (int64_t)h.c[10] : -1;
  double e;
  memcpy(&e, &h.max_err_bits, sizeof(e));
  report->max_abs_err = e;
  return PMSZ_OK;
}

int pmsz_batched_workspace_size(int32_t n, const pmsz_field* fields, size_t* bytes) {
  if (n < 0 || (n > 0 && !fields) || !bytes) return fail(PMSZ_ERR_INVALID_ARG, "bad batch");
  size_t tot = 0;
  for (int32_t i = 0; i < n; ++i) {
    int r = check_grid(&fields[i].grid);
    if (r) return r;
    tot = std::max(tot, correct_layout(make_geo(fields[i].grid)).total);
  }
  *bytes = tot;
  return PMSZ_OK;
}

int pmsz_correct_batched(int32_t n, const pmsz_field* fields, void* ws, size_t ws_bytes,
                         int64_t max_iters, pmsz_stats* stats, void* stream) {
  size_t need;
  int r = pmsz_batched_workspace_size(n, fields, &need);
  if (r) return r;
  if (!stats || (n > 0 && !ws)) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (ws_bytes < need) return fail(PMSZ_ERR_OOM, "workspace %zu bytes, need %zu", ws_bytes, need);
  int first = PMSZ_OK;
  for (int32_t i = 0; i < n; ++i) {
    r = pmsz_correct(&fields[i].grid, fields[i].f, fields[i].g, fields[i].xi, nullptr, ws,
                     ws_bytes, max_iters, &stats[i], stream);
    if (r == PMSZ_ERR_INVALID_ARG || r == PMSZ_ERR_DEVICE || r == PMSZ_ERR_OOM) return r;
    if (r != PMSZ_OK && first == PMSZ_OK) first = r;
  }
  return first;
}

}  // extern "C"
