// api.hip -- the C ABI of libpmsz: argument checks, workspace layout, the
// host side of the correction loop, labels and verification.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include <unordered_map>
#include <vector>

#include "engine.hpp"
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

// Status of a HIP call, for code that releases resources before returning.
inline int hip_check(hipError_t e) {
  return e == hipSuccess ? PMSZ_OK
                         : fail(PMSZ_ERR_DEVICE, "HIP call failed: %s", hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr int64_t DEFAULT_TUNE_ITERS = int64_t(1) << 40;  // tuning runs go to convergence
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
  // 3D tiles address six rows of a plane from one base with 32-bit offsets
  const int64_t size = g->dtype == PMSZ_F64 ? 8 : 4;
  if (g->ndim == 3 && (5 * g->nx + 65) * size > 4294967295LL)
    return fail(PMSZ_ERR_INVALID_ARG, "3D grids need nx below %lld for this value type",
                (long long)((4294967295LL / size - 65) / 5 + 1));
  return PMSZ_OK;
}

// xi in the field type, never above xi.
double xi_in_type(int dtype, double xi) {
  if (dtype == PMSZ_F64) return xi;
  float x = (float)xi;
  if ((double)x > xi) x = nextafterf(x, 0.0f);
  return (double)x;
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
  L.total = L.flag + align_up(kLabelsWsBytes);
  return L;
}

// ---------------------------------------------------------------------------
// Workspace plan of the correction engine for n fields:
//   [EngineCtl][FieldDesc x n][FieldIter x n]
//   [field 0: state, activity, bitmap] ... [field n-1: ...]
//   [directions of field 0] ... [directions of field n-1]
// Every region starts on a 256-byte boundary; everything before the direction
// bytes is cleared by one kernel before the launch.
// ---------------------------------------------------------------------------
// A plan's per-field arrays: one field is held inline, so that planning a
// single field (the allocation-free entry point) touches no heap.
template <class T>
struct PlanVec {
  T one{};
  std::vector<T> many;
  size_t n = 0;
  void resize(size_t k) {
    n = k;
    if (k > 1) many.resize(k);
  }
  size_t size() const { return n; }
  T* data() { return n > 1 ? many.data() : &one; }
  T& operator[](size_t i) { return data()[i]; }
};

struct BatchPlan {
  size_t ctl = 0, desc = 0, out = 0, trace = 0, fields = 0, dirs = 0, prop = 0, total = 0;
  int64_t total_tiles = 0, total_segs = 0;
  int edit_mode = 0;  // 0 halving, 1 targeted (proposal arrays after dirs)
  PlanVec<FieldDesc> fd;
  PlanVec<size_t> field_off, dirs_off, prop_off;
};

// Tile height policy per (ndim, dtype): the tuned tiles-per-field target
// (0 = the default).  Read when a field is planned, so a field keeps the
// geometry it was planned with.
std::mutex g_tiles_mu;
int32_t g_tiles_target[2][2] = {{0, 0}, {0, 0}};

// The tune cache: a JSON object in the file the environment variable
// PMSZ_TUNE_CACHE names, whose keys "2d_f32", "2d_f64", "3d_f32" and
// "3d_f64" hold tiles-per-field targets (0: the default).  Read once, before
// the first target is read or set in the process; rewritten whole by
// pmsz_tune_tiles.  A missing or malformed file leaves the defaults.
const char* const kTuneKeys[2][2] = {{"2d_f32", "2d_f64"}, {"3d_f32", "3d_f64"}};
std::once_flag g_tune_cache_once;

void read_tune_cache() {
  const char* path = getenv("PMSZ_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* fp = fopen(path, "rb");
  if (!fp) return;
  char buf[4096];
  const size_t n = fread(buf, 1, sizeof(buf) - 1, fp);
  fclose(fp);
  buf[n] = 0;
  std::lock_guard<std::mutex> lk(g_tiles_mu);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      char key[16];
      snprintf(key, sizeof(key), "\"%s\"", kTuneKeys[a][b]);
      const char* at = strstr(buf, key);
      if (!at) continue;
      at += strlen(key);
      while (*at == ' ' || *at == '\t' || *at == '\n' || *at == '\r') ++at;
      if (*at != ':') continue;
      char* end = nullptr;
      const long v = strtol(at + 1, &end, 10);
      if (end != at + 1 && v >= 0 && v <= (1L << 30)) g_tiles_target[a][b] = (int32_t)v;
    }
}

void ensure_tune_cache() { std::call_once(g_tune_cache_once, read_tune_cache); }

// Writes every target to the cache file (when PMSZ_TUNE_CACHE is set), through
// a temporary file and a rename.
int write_tune_cache() {
  const char* path = getenv("PMSZ_TUNE_CACHE");
  if (!path || !*path) return PMSZ_OK;
  int32_t t[2][2];
  {
    std::lock_guard<std::mutex> lk(g_tiles_mu);
    memcpy(t, g_tiles_target, sizeof(t));
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fp = fopen(tmp.c_str(), "wb");
  if (!fp) return fail(PMSZ_ERR_INVALID_ARG, "tune cache %s: cannot write", path);
  const int w = fprintf(fp, "{\"2d_f32\": %d, \"2d_f64\": %d, \"3d_f32\": %d, \"3d_f64\": %d}\n",
                        t[0][0], t[0][1], t[1][0], t[1][1]);
  const bool ok = w > 0 && fclose(fp) == 0;
  if (!ok || rename(tmp.c_str(), path) != 0)
    return fail(PMSZ_ERR_INVALID_ARG, "tune cache %s: cannot write", path);
  return PMSZ_OK;
}

// The set or tuned target, 0 when there is none (the default rule).
int32_t tiles_target(int ndim, int dtype) {
  ensure_tune_cache();
  std::lock_guard<std::mutex> lk(g_tiles_mu);
  return g_tiles_target[ndim == 3][dtype == PMSZ_F64];
}

// Descriptor of one field with everything but its device pointers.  target:
// tiles per field (0: the set or tuned target, else the default for a batch
// of nf fields).
int describe_field(const pmsz_field& fld, int64_t max_iters, int dirs_given, FieldDesc& d,
                   int32_t target = 0, int64_t nf = 1) {
  const pmsz_grid& g = fld.grid;
  int r = check_grid(&g);
  if (r) return r;
  if (!isfinite(fld.xi) || fld.xi < 0) return fail(PMSZ_ERR_INVALID_ARG, "xi must be finite and >= 0");
  memset(&d, 0, sizeof(d));
  d.f = fld.f;
  d.g = fld.g;
  if (target <= 0) target = tiles_target(g.ndim, g.dtype);
  if (target <= 0) target = default_tiles_target(nf);
  d.geo = make_tile_geo(g.ndim, g.nx, g.ny, g.nz, engine_chunk(g.ndim, g.nx, g.ny, g.nz, target));
  d.xi_t = xi_in_type(g.dtype, fld.xi);
  d.max_iters = max_iters;
  d.words = bitmap_words(d.geo.n);
  d.dirs_given = dirs_given;
  return PMSZ_OK;
}

int plan_batch(int32_t n, const pmsz_field* fields, const uint8_t* const* dirs_given,
               int64_t max_iters, BatchPlan& P, int edit_mode = 0, int32_t target = 0) {
  P.fd.resize(n);
  P.field_off.resize(n);
  P.dirs_off.resize(n);
  P.prop_off.resize(n);
  P.edit_mode = edit_mode;
  size_t fbytes = 0, dbytes = 0, pbytes = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (fields[i].grid.dtype != fields[0].grid.dtype)
      return fail(PMSZ_ERR_INVALID_ARG, "all fields of a batch must share one dtype");
    FieldDesc& d = P.fd[i];
    int r = describe_field(fields[i], max_iters, (dirs_given && dirs_given[i]) ? 1 : 0, d, target,
                           n);
    if (r) return r;
    d.tile_base = P.total_tiles;
    d.seg_base = P.total_segs;
    P.total_tiles += tile_count(d.geo);
    P.total_segs += (d.words + kSegWords - 1) / kSegWords;
    const FieldLayout L = field_layout(d.geo, true);
    P.field_off[i] = fbytes;
    fbytes += L.total;
    P.dirs_off[i] = dbytes;
    if (!d.dirs_given) dbytes += align_up((size_t)d.geo.n);
    P.prop_off[i] = pbytes;
    const size_t vsize = fields[i].grid.dtype == PMSZ_F64 ? 8 : 4;
    if (edit_mode) pbytes += align_up((size_t)d.geo.n * vsize);
  }
  P.ctl = 0;
  P.desc = align_up(sizeof(EngineCtl));
  P.out = P.desc + align_up(sizeof(FieldDesc) * (size_t)n);
  P.trace = P.out + align_up(sizeof(FieldIter) * (size_t)n);
  P.fields = P.trace + align_up(kTraceBytes);
  P.dirs = P.fields + fbytes;
  P.prop = P.dirs + dbytes;
  P.total = P.prop + pbytes;
  return PMSZ_OK;
}

// Host resources kept for reuse across calls: pinned staging buffers and HIP
// events, per thread.  None is released by a destructor: a thread-local
// destructor runs at thread or process exit, possibly after the HIP runtime
// has been torn down (profilers and torch finalise it from their own exit
// handlers), and a HIP call then faults inside exit().  Every resource is
// listed in a process-wide registry instead, and pmsz_release() frees them
// all while the runtime is still up; a thread whose resources were released
// (the registry's generation moved on) allocates new ones on its next call.
struct HostRes {
  std::mutex mu;
  std::vector<void*> pinned;
  std::vector<hipEvent_t> events;
  uint64_t gen = 1;
};
HostRes& host_res() {
  static HostRes* r = new HostRes();  // never destroyed
  return *r;
}
uint64_t res_gen() {
  std::lock_guard<std::mutex> lk(host_res().mu);
  return host_res().gen;
}

// Pinned staging for descriptors going up and states coming back; the calls
// that use it synchronise before returning, so one buffer per thread serves.
struct Staging {
  void* p = nullptr;
  size_t cap = 0;
  uint64_t gen = 0;
};
thread_local Staging t_stage;

int staging(Staging& s, size_t bytes, void** out) {
  if (s.gen != res_gen()) {  // released since it was allocated (or never allocated)
    s.p = nullptr;
    s.cap = 0;
  }
  if (s.cap < bytes) {
    HostRes& R = host_res();
    if (s.p) {
      std::lock_guard<std::mutex> lk(R.mu);
      R.pinned.erase(std::remove(R.pinned.begin(), R.pinned.end(), s.p), R.pinned.end());
      (void)hipHostFree(s.p);
    }
    s.p = nullptr;
    s.cap = 0;
    HIP_TRY(hipHostMalloc(&s.p, bytes, hipHostMallocDefault));
    std::lock_guard<std::mutex> lk(R.mu);
    R.pinned.push_back(s.p);
    s.cap = bytes;
    s.gen = R.gen;
  }
  *out = s.p;
  return PMSZ_OK;
}

// Frees a staging buffer now (unless pmsz_release already did).
void release_staging(Staging& s) {
  HostRes& R = host_res();
  std::lock_guard<std::mutex> lk(R.mu);
  if (s.p && s.gen == R.gen) {
    R.pinned.erase(std::remove(R.pinned.begin(), R.pinned.end(), s.p), R.pinned.end());
    (void)hipHostFree(s.p);
  }
  s.p = nullptr;
  s.cap = 0;
}

// Events around the engine launch and the figures of the last run.
struct Timing {
  // directions, first sweep, first engine launch, second sweep, second
  // engine launch, end (the sweeps and the first launch only when split);
  // then around each later sweep and engine launch (large tile rounds)
  hipEvent_t ev[9] = {};
  uint64_t gen = 0;
  pmsz_timing last;
  pmsz_round rounds[kTraceRounds];
  int64_t nrounds = 0;
  pmsz_labels_info labels;
};
thread_local Timing t_timing;

// The thread's timing events, created on first use (and after a release).
int timing_events(Timing& tm) {
  HostRes& R = host_res();
  if (tm.gen == res_gen() && tm.ev[0]) return PMSZ_OK;
  for (auto& e : tm.ev) {
    e = nullptr;
    HIP_TRY(hipEventCreate(&e));
    std::lock_guard<std::mutex> lk(R.mu);
    R.events.push_back(e);
    tm.gen = R.gen;
  }
  return PMSZ_OK;
}

void fill_stats(const FieldIter& it, pmsz_stats& o) {
  memset(&o, 0, sizeof(o));
  o.iterations = (int64_t)it.k;
  o.steps_applied = (int64_t)it.steps;
  o.flagged_final = (int64_t)it.flagged_final;
  o.stalled_flags = (int64_t)it.stalled_final;
  o.mismatch_initial = (int64_t)it.mism0;
  o.status = it.status;
  if (it.status == PMSZ_ERR_NONFINITE || it.status == PMSZ_ERR_INPUT_BOUND) {
    o.iterations = 0;
    o.steps_applied = 0;
  }
}

// Bytes of host staging run_batch needs for n fields (descriptors up; control
// block, states and round trace down, the last two as laid out in the
// workspace, so that one copy brings both).
size_t batch_stage_bytes(int32_t n) {
  const size_t up = sizeof(FieldDesc) * (size_t)n;
  const size_t down = kCtlHostBytes + align_up(sizeof(FieldIter) * (size_t)n) + kTraceBytes;
  return up > down ? up : down;
}

// Run the engine to completion on a planned batch; fills stats[n].  stage:
// host staging of batch_stage_bytes(n) bytes, or NULL for this thread's
// pinned buffer.  timed: record HIP events and the round trace into this
// thread's timing record (the allocation-free path records neither).
int run_batch(int dtype, BatchPlan& P, const uint8_t* const* dirs_given, void* ws,
              pmsz_stats* stats, hipStream_t s, void* stage = nullptr, bool timed = true) {
  const int32_t n = (int32_t)P.fd.size();
  char* base = (char*)ws;
  for (int32_t i = 0; i < n; ++i) {
    FieldDesc& d = P.fd[i];
    const FieldLayout L = field_layout(d.geo, true);
    char* fb = base + P.fields + P.field_off[i];
    d.st = (FieldState*)(fb + L.state);
    d.act = (uint8_t*)(fb + L.act);
    d.bm = (uint32_t*)(fb + L.bm);
    d.list = (uint32_t*)(fb + L.list);
    d.marks = (uint8_t*)(fb + L.marks);
    d.list_cap = list_capacity(d.geo);
    d.dirs = d.dirs_given ? (uint8_t*)dirs_given[i] : (uint8_t*)(base + P.dirs + P.dirs_off[i]);
    d.prop = P.edit_mode ? (void*)(base + P.prop + P.prop_off[i]) : nullptr;
  }
  const size_t up = sizeof(FieldDesc) * (size_t)n;
  int r = PMSZ_OK;
  if (!stage && (r = staging(t_stage, batch_stage_bytes(n), &stage))) return r;
  memcpy(stage, P.fd.data(), up);
  EngineCtl* ctl = (EngineCtl*)(base + P.ctl);
  FieldIter* out = (FieldIter*)(base + P.out);
  HIP_TRY(engine_zero(base, P.dirs, s));
  // proposal keys start unset (all ones)
  if (P.edit_mode) HIP_TRY(engine_fill(base + P.prop, P.total - P.prop, 0xFFFFFFFFu, s));
  HIP_TRY(hipMemcpyAsync(base + P.desc, stage, up, hipMemcpyHostToDevice, s));
  EngineArgs a;
  a.tiles_swept = 0;
  a.stop_on_done = 0;
  a.stop_host = nullptr;
  a.split_tiles = 0;
  a.tail_ok = n <= 256 ? 1 : 0;
  a.fd = (const FieldDesc*)(base + P.desc);
  a.out = out;
  a.nf = n;
  a.has_fresh = 1;
  a.ctl = ctl;
  a.total_tiles = P.total_tiles;
  a.total_segs = P.total_segs;
  a.max_rounds = -1;
  a.trace = timed ? (unsigned long long*)(base + P.trace) : nullptr;
  Timing& tm = t_timing;
  if (timed && (r = timing_events(tm))) return r;
  int grid = 0;
  bool need_dirs = false;
  int64_t voxels = 0;
  int dims = 0;
  for (int32_t i = 0; i < n; ++i) {
    need_dirs |= !P.fd[i].dirs_given;
    voxels += P.fd[i].geo.n;
    dims |= P.fd[i].geo.ndim == 3 ? 4 : 2;
  }
  // Directions of f, then the correction loop.  Large batches run the tile
  // detection of rounds 0 and 1 (full sweeps: every tile in round 0, nearly
  // every one in round 1) as plain kernels at the march's own occupancy,
  // each followed by an engine launch that starts with that round's apply;
  // small ones keep the whole loop in one launch (the extra launches would
  // cost more than they save).
  const bool split = voxels >= kSplitVoxels;
  if (timed) HIP_TRY(hipEventRecord(tm.ev[0], s));
  if (need_dirs) HIP_TRY(engine_dirs(dtype, a.fd, n, P.total_tiles, s));
  if (timed) HIP_TRY(hipEventRecord(tm.ev[1], s));
  if (split) {
    a.tiles_swept = 1;
    a.max_rounds = 1;
    HIP_TRY(engine_sweep(dtype, KIND_FIRST_GIVEN, P.edit_mode != 0, dims, a, s));
    if (timed) HIP_TRY(hipEventRecord(tm.ev[2], s));
    // round 0's apply pass as a plain kernel; the engine starts at round 1
    HIP_TRY(engine_apply_first(dtype, a, s));
    if (timed) HIP_TRY(hipEventRecord(tm.ev[3], s));
    a.has_fresh = 0;
    a.max_rounds = -1;
    HIP_TRY(engine_sweep(dtype, KIND_NEXT, P.edit_mode != 0, dims, a, s));
    if (timed) HIP_TRY(hipEventRecord(tm.ev[4], s));
  }
  // A large batch's later launches end before any round in which a field of
  // kSplitVoxels vertices or more sweeps tiles; the host then runs that
  // round's tile detection as a sweep kernel and launches the engine again.
  a.split_tiles = split ? 1 : 0;
  // (the workspace, barrier state included, was cleared at the start)
  HIP_TRY(engine_launch(dtype, a, s, &grid, false));
  if (a.tail_ok) HIP_TRY(engine_tail(dtype, a, s));
  if (timed) HIP_TRY(hipEventRecord(tm.ev[5], s));
  const EngineCtl* hc = (const EngineCtl*)stage;
  // staging: [control block][states, padded as in the workspace][trace]
  const FieldIter* hs = (const FieldIter*)((char*)stage + kCtlHostBytes);
  const unsigned long long* tr =
      (const unsigned long long*)((char*)stage + kCtlHostBytes + (P.trace - P.out));
  // the sweeps of those later tile rounds: ms by round (timed runs), count
  float late_ms[kTraceRounds] = {};
  int64_t late = 0;
  unsigned long long late_round = 0;
  float late_sweep_ms = 0.f, late_engine_ms = 0.f;
  int32_t tail_rounds = 0, handbacks = 0;
  for (;;) {
    // the staging buffer is reused for the results: the upload above is
    // stream-ordered before this copy, so it has been consumed
    HIP_TRY(hipMemcpyAsync(stage, ctl, kCtlHostBytes, hipMemcpyDeviceToHost, s));
    // the states, and the trace right after them in the workspace
    HIP_TRY(hipMemcpyAsync((char*)stage + kCtlHostBytes, out,
                           timed ? (P.trace - P.out) + kTraceBytes : sizeof(FieldIter) * (size_t)n,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hc->error) return fail(PMSZ_ERR_DEVICE, "grid barrier timed out in the correction engine");
    if (hc->handoff == kHandToEngine || hc->handoff == kTailDone) {
      tail_rounds += (int32_t)hc->rounds;
      handbacks += hc->handoff == kHandToEngine ? 1 : 0;
    }
    if (late > 0 && timed) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, tm.ev[6], tm.ev[7]));
      if (late_round < (unsigned long long)kTraceRounds) late_ms[late_round] += ms;
      late_sweep_ms += ms;
      HIP_TRY(hipEventElapsedTime(&ms, tm.ev[7], tm.ev[8]));
      late_engine_ms += ms;
    }
    bool running = false;
    for (int32_t i = 0; i < n && !running; ++i) running = !hs[i].done;
    if (!running) break;
    // the launches ended before a round with tile sweeps: a large one (split
    // batches), or one after the tail (k_tail handed the loop back)
    if (!split && hc->handoff != kHandToEngine) break;
    ++late;
    late_round = hc->epoch;
    a.tiles_swept = 1;
    a.has_fresh = 0;
    a.max_rounds = -1;
    if (timed) HIP_TRY(hipEventRecord(tm.ev[6], s));
    HIP_TRY(engine_sweep(dtype, KIND_NEXT, P.edit_mode != 0, dims, a, s));
    if (timed) HIP_TRY(hipEventRecord(tm.ev[7], s));
    HIP_TRY(engine_launch(dtype, a, s, &grid));
    if (a.tail_ok) HIP_TRY(engine_tail(dtype, a, s));
    if (timed) HIP_TRY(hipEventRecord(tm.ev[8], s));
  }
  if (!timed) {
    int first = PMSZ_OK;
    for (int32_t i = 0; i < n; ++i) {
      if (!hs[i].done) return fail(PMSZ_ERR_DEVICE, "field %d did not finish", i);
      fill_stats(hs[i], stats[i]);
      if (hs[i].status != PMSZ_OK && first == PMSZ_OK) first = hs[i].status;
    }
    if (first != PMSZ_OK) return fail(first, "%s", pmsz_status_string(first));
    return PMSZ_OK;
  }
  float el[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  HIP_TRY(hipEventElapsedTime(&el[0], tm.ev[0], tm.ev[1]));
  if (split) {
    for (int k = 1; k < 5; ++k) HIP_TRY(hipEventElapsedTime(&el[k], tm.ev[k], tm.ev[k + 1]));
  } else {
    HIP_TRY(hipEventElapsedTime(&el[4], tm.ev[1], tm.ev[5]));
  }
  memset(&tm.last, 0, sizeof(tm.last));
  tm.last.dirs_ms = el[0];
  tm.last.sweep_ms = el[1] + el[3] + late_sweep_ms;
  tm.last.sweeps = split ? 2 + late : 0;
  tm.last.tail_rounds = tail_rounds;
  tm.last.handbacks = handbacks;
  tm.last.engine_ms = el[2] + el[4] + late_engine_ms;
  tm.last.rounds = (int64_t)hc->epoch;  // the workspace starts every call at round 0
  tm.last.tiles = P.total_tiles;
  tm.last.grid = grid;
  {
    const int64_t R = hc->epoch < (unsigned long long)kTraceRounds ? (int64_t)hc->epoch
                                                                      : kTraceRounds;
    tm.nrounds = R;
    for (int64_t r = 0; r < R; ++r) {
      const unsigned long long* t = tr + kTraceSlots * r;
      const double start = (double)(r == 0 ? tr[kTraceRounds * kTraceSlots] : t[0]);
      pmsz_round& o = tm.rounds[r];
      o.detect_ms = ((double)t[1] - start) * 1e-5;  // 100 MHz ticks -> ms
      o.apply_ms = (double)(t[2] - t[1]) * 1e-5;
      o.swept = (int64_t)t[3];
      o.flagged = (int64_t)t[4];
      o.edits = (int64_t)t[5];
      o.sparse = (int64_t)t[6];
      if (split && r < 2) o.detect_ms += (double)el[r == 0 ? 1 : 3];  // the sweep kernel
      o.detect_ms += (double)late_ms[r];  // a later round's sweep kernel
      if (r == 0) {
        tm.last.first_round_ms = o.detect_ms + o.apply_ms;
      } else {
        tm.last.detect_ms += o.detect_ms;
        tm.last.apply_ms += o.apply_ms;
      }
    }
  }
  int first = PMSZ_OK;
  for (int32_t i = 0; i < n; ++i) {
    if (!hs[i].done) return fail(PMSZ_ERR_DEVICE, "field %d did not finish", i);
    fill_stats(hs[i], stats[i]);
    tm.last.swept += (int64_t)hs[i].swept;
    tm.last.edits += (int64_t)hs[i].steps;
    tm.last.voxels += P.fd[i].geo.n;
    if (hs[i].status != PMSZ_OK && first == PMSZ_OK) first = hs[i].status;
  }
  if (first != PMSZ_OK) return fail(first, "%s", pmsz_status_string(first));
  return PMSZ_OK;
}



// ---------------------------------------------------------------------------
// Decomposed domain (Sec. IV-B), emulated on one GPU.  Workspace:
//   [block table][exchange counter][per block: copy of f, copy of g,
//   direction bytes of the copy of f][engine workspace of the R block fields]
// The direction bytes of the copies are computed once and given to every
// phase's engine launch.
// ---------------------------------------------------------------------------
struct BlocksPlan {
  int32_t nb[3] = {1, 1, 1};
  int64_t R = 0;
  std::vector<int64_t> org, ext, core;  // 3R, 3R, 6R
  std::vector<size_t> off_f, off_g, off_d;
  size_t tab = 0, ctr = 0, hold = 0, planes_off = 0, batch = 0, total = 0;
  std::vector<int32_t> holders;  // per axis and coordinate: up to 3 blocks, -1 padded
  std::vector<int32_t> planes;   // (axis, coordinate) of every shared layer
  int64_t max_plane = 0;         // vertices of the largest such layer
  std::vector<pmsz_field> fields;
  std::vector<const uint8_t*> dirs;
  BatchPlan P;
};

int plan_blocks(const pmsz_grid& grid, const int32_t* blocks, double xi, int64_t cap,
                uintptr_t base, BlocksPlan& B) {
  const int64_t n[3] = {grid.nx, grid.ny, grid.nz};
  for (int a = 0; a < 3; ++a) {
    B.nb[a] = blocks[a];
    if (blocks[a] < 1 || blocks[a] > n[a])
      return fail(PMSZ_ERR_INVALID_ARG, "blocks[%d] = %d must lie in [1, %lld]", a, blocks[a],
                  (long long)n[a]);
  }
  B.R = (int64_t)B.nb[0] * B.nb[1] * B.nb[2];
  if (B.R > 65536) return fail(PMSZ_ERR_INVALID_ARG, "at most 65536 blocks");
  const size_t vs = grid.dtype == PMSZ_F64 ? 8 : 4;
  B.org.resize(3 * B.R);
  B.ext.resize(3 * B.R);
  B.core.resize(6 * B.R);
  B.off_f.resize(B.R);
  B.off_g.resize(B.R);
  B.off_d.resize(B.R);
  B.fields.resize(B.R);
  B.dirs.resize(B.R);
  B.tab = 0;
  B.ctr = align_up(sizeof(BlockCopy) * (size_t)B.R);
  B.hold = B.ctr + align_up(sizeof(unsigned long long));
  // holders of every coordinate along each axis, x then y then z
  B.holders.assign(3 * (size_t)(n[0] + n[1] + n[2]), -1);
  {
    size_t base_i = 0;
    for (int a = 0; a < 3; ++a) {
      const int64_t b = B.nb[a];
      for (int64_t k = 0; k < b; ++k) {
        const int64_t s0 = k * n[a] / b, s1 = (k + 1) * n[a] / b;
        const int64_t lo = s0 > 0 ? s0 - 1 : 0, hi = s1 < n[a] ? s1 + 1 : n[a];
        for (int64_t c = lo; c < hi; ++c) {
          int32_t* h = &B.holders[base_i + 3 * (size_t)c];
          int j = 0;
          while (j < 3 && h[j] >= 0) ++j;
          if (j < 3) h[j] = (int32_t)k;  // blocks visited in ascending order
        }
      }
      base_i += 3 * (size_t)n[a];
    }
    // layers held by more than one block along their axis
    base_i = 0;
    B.planes.clear();
    B.max_plane = 0;
    for (int a = 0; a < 3; ++a) {
      for (int64_t c = 0; c < n[a]; ++c)
        if (B.holders[base_i + 3 * (size_t)c + 1] >= 0) {
          B.planes.push_back(a);
          B.planes.push_back((int32_t)c);
          B.max_plane = std::max(B.max_plane, n[0] * n[1] * n[2] / n[a]);
        }
      base_i += 3 * (size_t)n[a];
    }
  }
  B.planes_off = B.hold + align_up(B.holders.size() * sizeof(int32_t));
  size_t at = B.planes_off + align_up((B.planes.size() + 2) * sizeof(int32_t));
  for (int64_t id = 0; id < B.R; ++id) {
    const int64_t k[3] = {id % B.nb[0], (id / B.nb[0]) % B.nb[1], id / ((int64_t)B.nb[0] * B.nb[1])};
    int64_t cells = 1;
    for (int a = 0; a < 3; ++a) {
      const int64_t b = B.nb[a], s0 = k[a] * n[a] / b, s1 = (k[a] + 1) * n[a] / b;
      const int64_t lo = s0 > 0 ? s0 - 1 : 0, hi = s1 < n[a] ? s1 + 1 : n[a];
      B.org[3 * id + a] = lo;
      B.ext[3 * id + a] = hi - lo;
      B.core[6 * id + 2 * a] = s0 - lo;
      B.core[6 * id + 2 * a + 1] = s1 - lo;
      cells *= hi - lo;
    }
    B.off_f[id] = at;
    at += align_up((size_t)cells * vs);
    B.off_g[id] = at;
    at += align_up((size_t)cells * vs);
    B.off_d[id] = at;
    at += align_up((size_t)cells);
    pmsz_field& fl = B.fields[id];
    fl.grid = grid;
    fl.grid.nx = B.ext[3 * id];
    fl.grid.ny = B.ext[3 * id + 1];
    fl.grid.nz = B.ext[3 * id + 2];
    fl.f = (const void*)(base + B.off_f[id]);
    fl.g = (void*)(base + B.off_g[id]);
    fl.xi = xi;
    B.dirs[id] = (const uint8_t*)(base + B.off_d[id]);
  }
  B.batch = at;
  int r = plan_batch((int32_t)B.R, B.fields.data(), B.dirs.data(), cap, B.P);
  if (r) return r;
  for (int64_t id = 0; id < B.R; ++id) {
    TileGeo& G = B.P.fd[id].geo;
    G.cx0 = (int32_t)B.core[6 * id];
    G.cx1 = (int32_t)B.core[6 * id + 1];
    G.cy0 = (int32_t)B.core[6 * id + 2];
    G.cy1 = (int32_t)B.core[6 * id + 3];
    G.cz0 = (int32_t)B.core[6 * id + 4];
    G.cz1 = (int32_t)B.core[6 * id + 5];
  }
  B.total = B.batch + B.P.total;
  return PMSZ_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Serving sessions: fields are admitted and retired between engine launches;
// each launch (a step) runs up to max_rounds rounds of every unfinished field.
// ---------------------------------------------------------------------------
struct pmsz_session {
  int dtype = 0;
  int32_t cap = 0;
  char* ws = nullptr;  // device: [EngineCtl][FieldDesc x cap][FieldIter x cap]
  size_t desc_off = 0, out_off = 0;
  Staging up, down;
  hipEvent_t ev = nullptr;
  hipStream_t stream = nullptr;
  bool pending = false;
  unsigned long long epoch = 0;
  int32_t next_handle = 1;
  struct Entry {
    FieldDesc d;
    int done = 0;
    int started = 0;  // its first round (directions of f, validation) has run
    pmsz_stats st;
  };
  std::unordered_map<int32_t, Entry> fields;
  std::vector<int32_t> order;  // insertion order of live handles
  std::vector<int32_t> stepped;  // handles of the last step, in descriptor order
  std::vector<int32_t> finished;  // handles that finished in the last synced step
  unsigned* stop_word = nullptr;  // pinned host word the engine polls (stop requests)
  pmsz_timing last;
};

namespace {

static size_t session_ctl_bytes(int32_t cap) {
  return align_up(sizeof(EngineCtl)) + align_up(sizeof(FieldDesc) * (size_t)cap) +
         align_up(sizeof(FieldIter) * (size_t)cap);
}

// Pointer jumping to the fixed point on the device: passes are queued a
// batch at a time (each returns at once when its predecessor changed
// nothing) and only the batch's changed flags are read back.  *passes
// receives the passes that ran, the last being the one that found nothing to
// change.  Direction bytes that do not form a forest (possible only for
// caller-supplied bytes) either never settle (PMSZ_ERR_INVALID_ARG here) or
// are counted in *bad by the passes (see k_labels_jump).
int label_pass(int32_t* lab, int64_t n, const uint8_t* dirs, int shift, unsigned int* flags,
               unsigned long long* bad, hipStream_t s, int64_t* passes) {
  HIP_TRY(engine_zero(flags, 4 * kLabelMaxPasses, s));
  unsigned int h[kLabelBatch];
  for (int b = 0; b < kLabelMaxPasses; b += kLabelBatch) {
    for (int p = b; p < b + kLabelBatch; ++p)
      HIP_TRY(launch_labels_jump(lab, n, dirs, shift, flags, bad, p, s));
    HIP_TRY(hipMemcpyAsync(h, flags + b, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int p = 0; p < kLabelBatch; ++p)
      if (!h[p]) {
        *passes = b + p + 1;
        return PMSZ_OK;
      }
  }
  return fail(PMSZ_ERR_INVALID_ARG,
              "label propagation did not settle in %d passes: the direction bytes do not form "
              "a forest", kLabelMaxPasses);
}

// ws: kLabelsWsBytes of device workspace.  Invalid direction codes are
// reported as PMSZ_ERR_INVALID_ARG (the label arrays are then unspecified).
int labels_impl(const Geo& G, const uint8_t* dirs, int32_t* lmax, int32_t* lmin, void* ws,
                hipStream_t s) {
  unsigned long long* bad = (unsigned long long*)ws;
  unsigned int* flags = (unsigned int*)((char*)ws + 256);
  Timing& tm = t_timing;
  int r = timing_events(tm);
  if (r) return r;
  memset(&tm.labels, 0, sizeof(tm.labels));
  HIP_TRY(engine_zero(bad, 8, s));
  HIP_TRY(hipEventRecord(tm.ev[0], s));
  HIP_TRY(launch_labels_init(dirs, G, lmax, lmin, bad, s));
  if (lmax && (r = label_pass(lmax, G.n, dirs, 0, flags, bad, s, &tm.labels.passes_max)))
    return r;
  if (lmin && (r = label_pass(lmin, G.n, dirs, 4, flags, bad, s, &tm.labels.passes_min)))
    return r;
  HIP_TRY(hipEventRecord(tm.ev[1], s));
  unsigned long long nbad = 0;
  HIP_TRY(hipMemcpyAsync(&nbad, bad, sizeof(nbad), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (nbad)
    return fail(PMSZ_ERR_INVALID_ARG, "%llu direction bytes hold a code that is not a neighbour "
                "of their vertex, or lie on a cycle of pointers", nbad);
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, tm.ev[0], tm.ev[1]));
  tm.labels.ms = ms;
  tm.labels.vertices = G.n;
  return PMSZ_OK;
}

// Rejects caller-supplied direction bytes with a code that is not valid for
// its vertex, before anything reads them as offsets.  scratch: 8 device bytes.
int check_dirs(const Geo& G, const uint8_t* dirs, void* scratch, hipStream_t s) {
  unsigned long long* bad = (unsigned long long*)scratch;
  HIP_TRY(engine_zero(bad, 8, s));
  HIP_TRY(launch_check_dirs(dirs, G, bad, s));
  unsigned long long nbad = 0;
  HIP_TRY(hipMemcpyAsync(&nbad, bad, sizeof(nbad), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (nbad)
    return fail(PMSZ_ERR_INVALID_ARG, "dirs_f: %llu direction bytes hold a code that is not a "
                "neighbour of their vertex", nbad);
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

int pmsz_last_timing(pmsz_timing* out) {
  if (!out) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  *out = t_timing.last;
  return PMSZ_OK;
}

int pmsz_last_rounds(pmsz_round* out, int64_t cap, int64_t* n) {
  if (!n || (cap > 0 && !out)) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  const int64_t m = t_timing.nrounds < cap ? t_timing.nrounds : (cap > 0 ? cap : 0);
  for (int64_t r = 0; r < m; ++r) out[r] = t_timing.rounds[r];
  *n = t_timing.nrounds;
  return PMSZ_OK;
}

int pmsz_last_labels(pmsz_labels_info* out) {
  if (!out) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  *out = t_timing.labels;
  return PMSZ_OK;
}

int pmsz_release(void) {
  HostRes& R = host_res();
  std::lock_guard<std::mutex> lk(R.mu);
  for (void* p : R.pinned) (void)hipHostFree(p);
  for (hipEvent_t e : R.events) (void)hipEventDestroy(e);
  R.pinned.clear();
  R.events.clear();
  ++R.gen;
  return PMSZ_OK;
}

int pmsz_workspace_size(const pmsz_grid* grid, int op, size_t* bytes) {
  int r = check_grid(grid);
  if (r) return r;
  if (!bytes) return fail(PMSZ_ERR_INVALID_ARG, "bytes is NULL");
  const Geo G = make_geo(*grid);
  switch (op) {
    case PMSZ_WS_CORRECT:
    case PMSZ_WS_CORRECT_TARGETED: {
      pmsz_field one;
      memset(&one, 0, sizeof(one));
      one.grid = *grid;
      BatchPlan P;
      if ((r = plan_batch(1, &one, nullptr, 0, P, op == PMSZ_WS_CORRECT_TARGETED))) return r;
      *bytes = P.total;
      break;
    }
    case PMSZ_WS_VERIFY: *bytes = verify_layout(G).total; break;
    case PMSZ_WS_LABELS: *bytes = kLabelsWsBytes; break;
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
  return pmsz_correct_mode(grid, f, g, xi, dirs_f, PMSZ_EDIT_HALVING, ws, ws_bytes, max_iters,
                           stats, stream);
}

int pmsz_correct_mode(const pmsz_grid* grid, const void* f, void* g, double xi,
                      const uint8_t* dirs_f, int edit_mode, void* ws, size_t ws_bytes,
                      int64_t max_iters, pmsz_stats* stats, void* stream) {
  if (edit_mode != PMSZ_EDIT_HALVING && edit_mode != PMSZ_EDIT_TARGETED)
    return fail(PMSZ_ERR_INVALID_ARG, "unknown edit mode %d", edit_mode);
  int r = check_grid(grid);
  if (r) return r;
  if (!f || !g || !ws || !stats) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (!isfinite(xi) || xi < 0) return fail(PMSZ_ERR_INVALID_ARG, "xi must be finite and >= 0");
  if (max_iters < 0) return fail(PMSZ_ERR_INVALID_ARG, "max_iters must be >= 0");
  if ((uintptr_t)ws % kAlign) return fail(PMSZ_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  pmsz_field one;
  one.grid = *grid;
  one.f = f;
  one.g = g;
  one.xi = xi;
  const uint8_t* given[1] = {dirs_f};
  BatchPlan P;
  if ((r = plan_batch(1, &one, given, max_iters, P, edit_mode))) return r;
  if (ws_bytes < P.total) return fail(PMSZ_ERR_OOM, "workspace %zu bytes, need %zu", ws_bytes, P.total);
  memset(stats, 0, sizeof(*stats));
  // caller-supplied directions become neighbour offsets: check them first
  if (dirs_f && (r = check_dirs(make_geo(*grid), dirs_f, ws, (hipStream_t)stream))) {
    stats->status = r;
    return r;
  }
  return run_batch(grid->dtype, P, given, ws, stats, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Allocation-free correction.  The workspace is a file-scope device array
// (each device that runs the library holds its own copy until the process
// ends).  In host code the array's name is only a host-side stand-in: its
// device address is looked up once per device with hipGetSymbolAddress, with
// that device current, and only that address is ever handed to kernels.
// ---------------------------------------------------------------------------
}  // extern "C"

constexpr size_t kScratchBytes = PMSZ_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kMaxDevices];  // device address of `scratch`, per device

// Address of the current device's scratch array; the stream must belong to
// that device.
int scratch_address(hipStream_t s, void** out) {
  int dev = -1;
  hipDevice_t sdev = -1;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipStreamGetDevice(s, &sdev));
  if (sdev != dev)
    return fail(PMSZ_ERR_INVALID_ARG, "the stream belongs to device %d, the current device is %d",
                (int)sdev, dev);
  if (dev < 0 || dev >= kMaxDevices)
    return fail(PMSZ_ERR_INVALID_ARG, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || (uintptr_t)p % kAlign)
      return fail(PMSZ_ERR_DEVICE, "scratch array of device %d has no aligned address", dev);
    g_scratch_at[dev] = p;
  }
  *out = g_scratch_at[dev];
  return PMSZ_OK;
}

// Host staging of one field's run (descriptor up; control block, round trace
// and state down), on the caller's stack.
constexpr size_t kOneFieldStage =
    std::max(sizeof(FieldDesc), kCtlHostBytes + kTraceBytes + sizeof(FieldIter));

}  // namespace

extern "C" {

int pmsz_correct_noalloc(const pmsz_grid* grid, const void* f, void* g, double xi,
                         const uint8_t* dirs_f, int64_t max_iters, pmsz_stats* stats,
                         void* stream) {
  int r = check_grid(grid);
  if (r) return r;
  if (!f || !g || !stats) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (!isfinite(xi) || xi < 0) return fail(PMSZ_ERR_INVALID_ARG, "xi must be finite and >= 0");
  if (max_iters < 0) return fail(PMSZ_ERR_INVALID_ARG, "max_iters must be >= 0");
  const hipStream_t s = (hipStream_t)stream;
  pmsz_field one;
  one.grid = *grid;
  one.f = f;
  one.g = g;
  one.xi = xi;
  const uint8_t* given[1] = {dirs_f};
  BatchPlan P;
  if ((r = plan_batch(1, &one, given, max_iters, P, PMSZ_EDIT_HALVING))) return r;
  if (P.total > kScratchBytes)
    return fail(PMSZ_ERR_OOM,
                "this field needs %zu bytes of workspace; the allocation-free correction has %zu "
                "(use pmsz_correct with a workspace)", P.total, kScratchBytes);
  void* ws = nullptr;
  if ((r = scratch_address(s, &ws))) return r;
  memset(stats, 0, sizeof(*stats));
  if (dirs_f && (r = check_dirs(make_geo(*grid), dirs_f, ws, s))) {
    stats->status = r;
    return r;
  }
  alignas(64) unsigned char stage[kOneFieldStage];
  return run_batch(grid->dtype, P, given, ws, stats, s, stage, false);
}

int pmsz_probe_read(const void* p, int64_t bytes, int32_t pattern, uint64_t* sum, void* stream) {
  if (!p || !sum) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (bytes < 0 || (pattern == 0 && bytes % 4) || (pattern != 0 && pattern != 1))
    return fail(PMSZ_ERR_INVALID_ARG, "bytes must be >= 0 (a multiple of 4 for pattern 0); "
                "pattern 0 or 1");
  if ((uintptr_t)p % 4) return fail(PMSZ_ERR_INVALID_ARG, "p must be 4-byte aligned");
  const hipStream_t s = (hipStream_t)stream;
  unsigned long long* d = nullptr;
  HIP_TRY(hipMallocAsync((void**)&d, sizeof(*d), s));
  int r = hip_check(engine_zero(d, 8, s));
  if (!r) r = hip_check(launch_probe_read(p, bytes, pattern, d, s));
  unsigned long long h = 0;
  if (!r) r = hip_check(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s));
  const int r2 = hip_check(hipFreeAsync(d, s));
  if (!r) r = r2;
  if (!r) r = hip_check(hipStreamSynchronize(s));
  if (r) return r;
  *sum = h;
  return PMSZ_OK;
}

int pmsz_edits_workspace_size(const pmsz_grid* grid, int64_t max_edits, size_t* bytes) {
  int r = check_grid(grid);
  if (r) return r;
  if (!bytes) return fail(PMSZ_ERR_INVALID_ARG, "bytes is NULL");
  if (max_edits < 0) return fail(PMSZ_ERR_INVALID_ARG, "max_edits must be >= 0");
  const Geo G = make_geo(*grid);
  *bytes = edits_workspace_bytes(G.n, max_edits < G.n ? max_edits : G.n);
  return PMSZ_OK;
}

int pmsz_edits_max_bytes(int64_t n_edits, size_t* bytes) {
  if (!bytes || n_edits < 0) return fail(PMSZ_ERR_INVALID_ARG, "bad argument");
  *bytes = edits_stream_bytes(n_edits);
  return PMSZ_OK;
}

int pmsz_encode_edits(const pmsz_grid* grid, const void* fhat, const void* g, int64_t max_edits,
                      void* ws, size_t ws_bytes, uint8_t* out, size_t out_cap, int64_t* n_edits,
                      int64_t* n_bytes, void* stream) {
  int r = check_grid(grid);
  if (r) return r;
  if (!fhat || !g || !ws || !out || !n_edits || !n_bytes)
    return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (max_edits < 0) return fail(PMSZ_ERR_INVALID_ARG, "max_edits must be >= 0");
  if ((uintptr_t)ws % kAlign || (uintptr_t)out % 8)
    return fail(PMSZ_ERR_INVALID_ARG, "workspace must be 256-byte and out 8-byte aligned");
  const Geo G = make_geo(*grid);
  const int64_t cap = max_edits < G.n ? max_edits : G.n;
  const size_t need = edits_workspace_bytes(G.n, cap);
  if (ws_bytes < need) return fail(PMSZ_ERR_OOM, "workspace %zu bytes, need %zu", ws_bytes, need);
  *n_edits = *n_bytes = 0;
  hipError_t he = hipSuccess;
  const int res = edits_encode(grid->dtype, fhat, g, G.n, cap, ws, out, out_cap, n_edits, n_bytes,
                               &he, (hipStream_t)stream);
  if (res < 0) return fail(PMSZ_ERR_DEVICE, "edit encoding: %s", hipGetErrorString(he));
  if (res == 1)
    return fail(PMSZ_ERR_OOM, "%lld edits exceed max_edits %lld", (long long)*n_edits,
                (long long)cap);
  if (res == 2)
    return fail(PMSZ_ERR_OOM, "stream needs %lld bytes, out holds %zu", (long long)*n_bytes,
                out_cap);
  return PMSZ_OK;
}

int pmsz_decode_edits(const pmsz_grid* grid, const uint8_t* in, size_t n_bytes, void* g,
                      void* ws, size_t ws_bytes, void* stream) {
  int r = check_grid(grid);
  if (r) return r;
  if (!in || !g || !ws) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (ws_bytes < kAlign || (uintptr_t)ws % kAlign || (uintptr_t)in % 8)
    return fail(PMSZ_ERR_INVALID_ARG, "need a 256-byte aligned workspace of 256 bytes and an "
                                      "8-byte aligned stream");
  if (n_bytes < 40) return fail(PMSZ_ERR_INVALID_ARG, "stream shorter than its header");
  hipStream_t s = (hipStream_t)stream;
  unsigned char h[40];
  HIP_TRY(hipMemcpyAsync(h, in, 40, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  unsigned long long nv, ne, nb;
  uint32_t chunk, chunks;
  memcpy(&nv, h + 8, 8);
  memcpy(&ne, h + 16, 8);
  memcpy(&nb, h + 24, 8);
  memcpy(&chunk, h + 32, 4);
  memcpy(&chunks, h + 36, 4);
  const Geo G = make_geo(*grid);
  const int dt = grid->dtype == PMSZ_F64 ? 1 : 0;
  if (memcmp(h, "PMSE", 4) || h[4] != 1 || h[5] != dt || nv != (unsigned long long)G.n ||
      chunk != 4096 || chunks != (ne + 4095) / 4096 || ne > nv ||
      40 + 16 * (unsigned long long)chunks + nb > n_bytes)
    return fail(PMSZ_ERR_INVALID_ARG, "not an edit stream of this grid and type");
  int* err = (int*)ws;
  HIP_TRY(engine_zero(err, 256, s));
  HIP_TRY(edits_decode(grid->dtype, in + 40, in + 40 + 16 * (size_t)chunks, (int64_t)nb,
                       (int64_t)ne, G.n, g, err, s));
  int herr = 0;
  HIP_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (herr) return fail(PMSZ_ERR_INVALID_ARG, "malformed edit stream payload");
  return PMSZ_OK;
}

int pmsz_labels(const pmsz_grid* grid, const uint8_t* dirs, int32_t* max_label,
                int32_t* min_label, void* ws, size_t ws_bytes, void* stream) {
  int r = check_grid(grid);
  if (r) return r;
  if (!dirs || !ws) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if ((uintptr_t)ws % kAlign) return fail(PMSZ_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < kLabelsWsBytes)
    return fail(PMSZ_ERR_OOM, "labels workspace needs %zu bytes", kLabelsWsBytes);
  const Geo G = make_geo(*grid);
  return labels_impl(G, dirs, max_label, min_label, ws, (hipStream_t)stream);
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
  void* lws = b + L.flag;
  HIP_TRY(engine_zero(vc, sizeof(VerifyCounts), s));
  HIP_TRY(launch_dirs(grid->dtype, f, G, df, s));
  HIP_TRY(launch_dirs(grid->dtype, g, G, dg, s));
  if ((r = labels_impl(G, df, lfx, lfn, lws, s))) return r;
  if ((r = labels_impl(G, dg, lgx, lgn, lws, s))) return r;
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
  BatchPlan P;
  int r = plan_batch(n, fields, nullptr, 0, P);
  if (r) return r;
  *bytes = P.total;
  return PMSZ_OK;
}

int pmsz_correct_batched(int32_t n, const pmsz_field* fields, void* ws, size_t ws_bytes,
                         int64_t max_iters, pmsz_stats* stats, void* stream) {
  if (n < 0 || (n > 0 && (!fields || !stats || !ws)))
    return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (max_iters < 0) return fail(PMSZ_ERR_INVALID_ARG, "max_iters must be >= 0");
  if (n == 0) return PMSZ_OK;
  if ((uintptr_t)ws % kAlign) return fail(PMSZ_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  for (int32_t i = 0; i < n; ++i)
    if (!fields[i].f || !fields[i].g) return fail(PMSZ_ERR_INVALID_ARG, "field %d: NULL array", i);
  BatchPlan P;
  int r = plan_batch(n, fields, nullptr, max_iters, P);
  if (r) return r;
  if (ws_bytes < P.total) return fail(PMSZ_ERR_OOM, "workspace %zu bytes, need %zu", ws_bytes, P.total);
  return run_batch(fields[0].grid.dtype, P, nullptr, ws, stats, (hipStream_t)stream);
}


int pmsz_set_tiles_target(int32_t ndim, int32_t dtype, int32_t target) {
  if ((ndim != 2 && ndim != 3) || (dtype != PMSZ_F32 && dtype != PMSZ_F64) || target < 0)
    return fail(PMSZ_ERR_INVALID_ARG, "bad ndim, dtype or target");
  ensure_tune_cache();  // an explicit setting overrides the cache
  std::lock_guard<std::mutex> lk(g_tiles_mu);
  g_tiles_target[ndim == 3][dtype == PMSZ_F64] = target;
  return PMSZ_OK;
}

int pmsz_get_tiles_target(int32_t ndim, int32_t dtype, int32_t* target) {
  if ((ndim != 2 && ndim != 3) || (dtype != PMSZ_F32 && dtype != PMSZ_F64) || !target)
    return fail(PMSZ_ERR_INVALID_ARG, "bad ndim, dtype or NULL target");
  *target = tiles_target(ndim, dtype);
  return PMSZ_OK;
}

namespace {
// Scratch copies of the fields' fhat for the tuner, then the batch workspace.
int tune_layout(int32_t n, const pmsz_field* fields, std::vector<size_t>& off, size_t* total) {
  if (n < 1 || !fields) return fail(PMSZ_ERR_INVALID_ARG, "empty batch");
  off.resize(n);
  size_t at = 0;
  for (int32_t i = 0; i < n; ++i) {
    int r = check_grid(&fields[i].grid);
    if (r) return r;
    if (fields[i].grid.ndim != fields[0].grid.ndim || fields[i].grid.dtype != fields[0].grid.dtype)
      return fail(PMSZ_ERR_INVALID_ARG, "tuned fields must share ndim and dtype");
    const size_t vs = fields[i].grid.dtype == PMSZ_F64 ? 8 : 4;
    off[i] = at;
    at += align_up((size_t)(fields[i].grid.nx * fields[i].grid.ny * fields[i].grid.nz) * vs);
  }
  BatchPlan P;
  int r = plan_batch(n, fields, nullptr, 0, P);
  if (r) return r;
  *total = at + P.total;
  return PMSZ_OK;
}
}  // namespace

int pmsz_tune_workspace_size(int32_t n, const pmsz_field* fields, size_t* bytes) {
  if (!bytes) return fail(PMSZ_ERR_INVALID_ARG, "bytes is NULL");
  std::vector<size_t> off;
  return tune_layout(n, fields, off, bytes);
}

int pmsz_tune_tiles(int32_t n, const pmsz_field* fields, const int32_t* candidates,
                    int32_t n_candidates, int32_t reps, void* ws, size_t ws_bytes, double* ms,
                    int32_t* best, void* stream) {
  if (!fields || !candidates || n_candidates < 1 || reps < 1 || !ws || !best)
    return fail(PMSZ_ERR_INVALID_ARG, "NULL argument or empty candidate list");
  if ((uintptr_t)ws % kAlign) return fail(PMSZ_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  for (int32_t c = 0; c < n_candidates; ++c)
    if (candidates[c] < 1) return fail(PMSZ_ERR_INVALID_ARG, "candidate targets must be >= 1");
  for (int32_t i = 0; i < n; ++i)
    if (!fields[i].f || !fields[i].g) return fail(PMSZ_ERR_INVALID_ARG, "field %d: NULL array", i);
  std::vector<size_t> off;
  size_t total = 0;
  int r = tune_layout(n, fields, off, &total);
  if (r) return r;
  if (ws_bytes < total) return fail(PMSZ_ERR_OOM, "workspace %zu bytes, need %zu", ws_bytes, total);
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  std::vector<pmsz_field> scratch(fields, fields + n);
  for (int32_t i = 0; i < n; ++i) scratch[i].g = base + off[i];
  std::vector<pmsz_stats> st((size_t)n);
  const size_t vs = fields[0].grid.dtype == PMSZ_F64 ? 8 : 4;
  double best_ms = 0.0;
  int32_t best_t = 0;
  for (int32_t c = 0; c < n_candidates; ++c) {
    BatchPlan P;
    if ((r = plan_batch(n, scratch.data(), nullptr, DEFAULT_TUNE_ITERS, P, 0, candidates[c])))
      return r;
    double t_min = 0.0;
    for (int32_t k = 0; k < reps; ++k) {
      for (int32_t i = 0; i < n; ++i) {
        const pmsz_grid& g = fields[i].grid;
        HIP_TRY(hipMemcpyAsync(scratch[i].g, fields[i].g, (size_t)(g.nx * g.ny * g.nz) * vs,
                               hipMemcpyDeviceToDevice, s));
      }
      r = run_batch(fields[0].grid.dtype, P, nullptr, base + (total - P.total), st.data(), s);
      if (r != PMSZ_OK && r != PMSZ_ERR_NOT_CONVERGED && r != PMSZ_ERR_STALLED) return r;
      const double t = t_timing.last.dirs_ms + t_timing.last.sweep_ms + t_timing.last.engine_ms;
      if (k == 0 || t < t_min) t_min = t;
    }
    if (ms) ms[c] = t_min;
    if (c == 0 || t_min < best_ms) {
      best_ms = t_min;
      best_t = candidates[c];
    }
  }
  *best = best_t;
  if ((r = pmsz_set_tiles_target(fields[0].grid.ndim, fields[0].grid.dtype, best_t))) return r;
  return write_tune_cache();
}

int pmsz_blocks_workspace_size(const pmsz_grid* grid, const int32_t* blocks, size_t* bytes) {
  int r = check_grid(grid);
  if (r) return r;
  if (!blocks || !bytes) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  BlocksPlan B;
  if ((r = plan_blocks(*grid, blocks, 0.0, 0, (uintptr_t)kAlign, B))) return r;
  *bytes = B.total;
  return PMSZ_OK;
}

int pmsz_correct_blocks(const pmsz_grid* grid, const void* f, void* g, double xi,
                        const int32_t* blocks, int32_t per_round, int64_t max_phases,
                        int64_t max_iters, void* ws, size_t ws_bytes, pmsz_blocks_stats* stats,
                        void* stream) {
  int r = check_grid(grid);
  if (r) return r;
  if (!f || !g || !blocks || !ws || !stats) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (!isfinite(xi) || xi < 0) return fail(PMSZ_ERR_INVALID_ARG, "xi must be finite and >= 0");
  if (max_phases < 1) return fail(PMSZ_ERR_INVALID_ARG, "max_phases must be >= 1");
  if (max_iters < 0) return fail(PMSZ_ERR_INVALID_ARG, "max_iters must be >= 0");
  if ((uintptr_t)ws % kAlign) return fail(PMSZ_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  memset(stats, 0, sizeof(*stats));
  BlocksPlan B;
  const int64_t cap = per_round ? 1 : max_iters;
  if ((r = plan_blocks(*grid, blocks, xi, cap, (uintptr_t)ws, B))) return r;
  if (ws_bytes < B.total) return fail(PMSZ_ERR_OOM, "workspace %zu bytes, need %zu", ws_bytes, B.total);
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  const Geo G = make_geo(*grid);
  // block table for the exchange
  {
    std::vector<BlockCopy> tab((size_t)B.R);
    for (int64_t id = 0; id < B.R; ++id) {
      tab[id].ox = B.org[3 * id];
      tab[id].oy = B.org[3 * id + 1];
      tab[id].oz = B.org[3 * id + 2];
      tab[id].lnx = B.ext[3 * id];
      tab[id].lny = B.ext[3 * id + 1];
      tab[id].g = base + B.off_g[id];
    }
    void* stage;
    const size_t tb = sizeof(BlockCopy) * tab.size(), hb = sizeof(int32_t) * B.holders.size(),
                 pb = sizeof(int32_t) * B.planes.size();
    if ((r = staging(t_stage, tb + hb + pb, &stage))) return r;
    memcpy(stage, tab.data(), tb);
    memcpy((char*)stage + tb, B.holders.data(), hb);
    if (pb) memcpy((char*)stage + tb + hb, B.planes.data(), pb);
    HIP_TRY(hipMemcpyAsync(base + B.tab, stage, tb, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(base + B.hold, (char*)stage + tb, hb, hipMemcpyHostToDevice, s));
    if (pb)
      HIP_TRY(hipMemcpyAsync(base + B.planes_off, (char*)stage + tb + hb, pb,
                             hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // the staging buffer is reused below
  }
  // copies of f and fhat, and the directions of each copy of f
  for (int64_t id = 0; id < B.R; ++id) {
    HIP_TRY(blocks_gather(grid->dtype, f, G, &B.org[3 * id], &B.ext[3 * id], base + B.off_f[id], s));
    HIP_TRY(blocks_gather(grid->dtype, g, G, &B.org[3 * id], &B.ext[3 * id], base + B.off_g[id], s));
    HIP_TRY(launch_dirs(grid->dtype, base + B.off_f[id], make_geo(B.fields[id].grid),
                        (uint8_t*)(base + B.off_d[id]), s));
  }
  hipEvent_t ev[2];
  HIP_TRY(hipEventCreate(&ev[0]));
  HIP_TRY(hipEventCreate(&ev[1]));
  std::vector<pmsz_stats> st((size_t)B.R);
  unsigned long long* ctr = (unsigned long long*)(base + B.ctr);
  int status = PMSZ_OK;
  r = PMSZ_OK;
  for (;;) {
    if (stats->phases == max_phases) {
      status = PMSZ_ERR_NOT_CONVERGED;
      break;
    }
    // local correction of every block: the blocks are the fields of one
    // engine launch, each comparing its core only
    r = run_batch(grid->dtype, B.P, B.dirs.data(), base + B.batch, st.data(), s);
    if (r != PMSZ_OK && r != PMSZ_ERR_NOT_CONVERGED && r != PMSZ_ERR_STALLED) break;
    r = PMSZ_OK;
    // a block whose copy failed validation (first phase only): g untouched
    for (int64_t id = 0; id < B.R && r == PMSZ_OK; ++id)
      if (st[id].status == PMSZ_ERR_NONFINITE || st[id].status == PMSZ_ERR_INPUT_BOUND)
        r = fail(st[id].status, "block %lld: %s", (long long)id,
                 pmsz_status_string(st[id].status));
    if (r != PMSZ_OK) break;
    stats->compute_ms += t_timing.last.dirs_ms + t_timing.last.sweep_ms + t_timing.last.engine_ms;
    // ghost-layer exchange
    unsigned long long lowered = 0;
    if ((r = hip_check(engine_fill(ctr, sizeof(unsigned long long), 0u, s)))) break;
    if ((r = hip_check(hipEventRecord(ev[0], s)))) break;
    // owners' cores into g, then the shared vertices take their minimum
    for (int64_t id = 0; id < B.R && r == PMSZ_OK; ++id)
      r = hip_check(blocks_scatter_core(grid->dtype, base + B.off_g[id], &B.ext[3 * id],
                                        &B.core[6 * id], &B.org[3 * id], g, G, s));
    if (r != PMSZ_OK) break;
    if ((r = hip_check(blocks_exchange(grid->dtype, g, G, B.nb,
                                       (const BlockCopy*)(base + B.tab),
                                       (const int32_t*)(base + B.hold),
                                       (const int32_t*)(base + B.planes_off),
                                       (int32_t)(B.planes.size() / 2), B.max_plane, ctr, s))))
      break;
    if ((r = hip_check(hipEventRecord(ev[1], s)))) break;
    if ((r = hip_check(hipMemcpyAsync(&lowered, ctr, sizeof(lowered), hipMemcpyDeviceToHost, s))))
      break;
    if ((r = hip_check(hipStreamSynchronize(s)))) break;
    float ms = 0.f;
    if ((r = hip_check(hipEventElapsedTime(&ms, ev[0], ev[1])))) break;
    stats->exchange_ms += ms;
    int64_t steps = 0, most = 0;
    bool all_ok = true, any_stalled = false;
    for (int64_t id = 0; id < B.R; ++id) {
      steps += st[id].steps_applied;
      stats->local_rounds += st[id].iterations;
      most = std::max(most, st[id].iterations);
      all_ok &= st[id].status == PMSZ_OK;
      any_stalled |= st[id].status == PMSZ_ERR_STALLED;
    }
    stats->phases += 1;
    stats->critical_rounds += most;
    stats->lowered += (int64_t)lowered;
    stats->steps_applied += steps;
    if (all_ok && lowered == 0) break;
    if (steps == 0 && lowered == 0) {
      status = any_stalled ? PMSZ_ERR_STALLED : PMSZ_ERR_NOT_CONVERGED;
      break;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (r != PMSZ_OK) {
    stats->status = r;
    return r;
  }
  stats->status = status;
  if (status != PMSZ_OK) return fail(status, "%s", pmsz_status_string(status));
  return PMSZ_OK;
}

int pmsz_session_workspace_size(int32_t max_fields, size_t* bytes) {
  if (max_fields < 1 || !bytes) return fail(PMSZ_ERR_INVALID_ARG, "max_fields must be >= 1");
  *bytes = session_ctl_bytes(max_fields);
  return PMSZ_OK;
}

int pmsz_field_workspace_size(const pmsz_grid* grid, size_t* bytes) {
  int r = check_grid(grid);
  if (r) return r;
  if (!bytes) return fail(PMSZ_ERR_INVALID_ARG, "bytes is NULL");
  const TileGeo G = make_tile_geo(grid->ndim, grid->nx, grid->ny, grid->nz,
                                  engine_chunk(grid->ndim, grid->nx, grid->ny, grid->nz,
                                               default_tiles_target(1)));
  *bytes = field_layout(G, false).total;
  return PMSZ_OK;
}

int pmsz_session_create(int32_t dtype, int32_t max_fields, void* ws, size_t ws_bytes,
                        void* stream, pmsz_session** out) {
  if (!out || !ws || max_fields < 1 || (dtype != PMSZ_F32 && dtype != PMSZ_F64))
    return fail(PMSZ_ERR_INVALID_ARG, "bad session arguments");
  if ((uintptr_t)ws % kAlign) return fail(PMSZ_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < session_ctl_bytes(max_fields))
    return fail(PMSZ_ERR_OOM, "session workspace %zu bytes, need %zu", ws_bytes,
                session_ctl_bytes(max_fields));
  pmsz_session* S = new pmsz_session();
  S->dtype = dtype;
  S->cap = max_fields;
  S->ws = (char*)ws;
  S->desc_off = align_up(sizeof(EngineCtl));
  S->out_off = S->desc_off + align_up(sizeof(FieldDesc) * (size_t)max_fields);
  S->stream = (hipStream_t)stream;
  hipError_t e = hipEventCreateWithFlags(&S->ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&S->stop_word, 64, hipHostMallocDefault);
  if (e == hipSuccess) {
    __atomic_store_n(S->stop_word, 0u, __ATOMIC_RELAXED);
    e = engine_zero(S->ws, align_up(sizeof(EngineCtl)), S->stream);
  }
  if (e != hipSuccess) {
    if (S->ev) (void)hipEventDestroy(S->ev);
    if (S->stop_word) (void)hipHostFree(S->stop_word);
    delete S;
    return fail(PMSZ_ERR_DEVICE, "session setup failed: %s", hipGetErrorString(e));
  }
  memset(&S->last, 0, sizeof(S->last));
  *out = S;
  return PMSZ_OK;
}

int pmsz_session_add(pmsz_session* S, const pmsz_field* field, int64_t max_iters, void* field_ws,
                     size_t field_ws_bytes, int32_t* handle) {
  if (!S || !field || !field_ws || !handle) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  if (S->pending) return fail(PMSZ_ERR_INVALID_ARG, "a step is in flight: sync first");
  if (field->grid.dtype != S->dtype) return fail(PMSZ_ERR_INVALID_ARG, "dtype differs from session");
  if (!field->f || !field->g) return fail(PMSZ_ERR_INVALID_ARG, "NULL array");
  if (max_iters < 0) return fail(PMSZ_ERR_INVALID_ARG, "max_iters must be >= 0");
  if ((int32_t)S->order.size() >= S->cap) return fail(PMSZ_ERR_OOM, "session is full");
  if ((uintptr_t)field_ws % kAlign) return fail(PMSZ_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  pmsz_session::Entry e;
  int r = describe_field(*field, max_iters, 0, e.d);
  if (r) return r;
  const FieldLayout L = field_layout(e.d.geo, false);
  if (field_ws_bytes < L.total)
    return fail(PMSZ_ERR_OOM, "field workspace %zu bytes, need %zu", field_ws_bytes, L.total);
  char* fb = (char*)field_ws;
  e.d.st = (FieldState*)(fb + L.state);
  e.d.act = (uint8_t*)(fb + L.act);
  e.d.bm = (uint32_t*)(fb + L.bm);
  e.d.list = (uint32_t*)(fb + L.list);
  e.d.marks = (uint8_t*)(fb + L.marks);
  e.d.list_cap = list_capacity(e.d.geo);
  e.d.dirs = (uint8_t*)(fb + L.dirs);
  HIP_TRY(engine_zero(fb, L.dirs, S->stream));
  // directions of f now, at the stencil's own occupancy; the engine then
  // starts the field from them
  HIP_TRY(launch_dirs(field->grid.dtype, field->f, make_geo(field->grid), e.d.dirs, S->stream));
  e.d.dirs_given = 1;
  memset(&e.st, 0, sizeof(e.st));
  const int32_t h = S->next_handle++;
  S->fields[h] = e;
  S->order.push_back(h);
  *handle = h;
  return PMSZ_OK;
}

int pmsz_session_step(pmsz_session* S, int64_t max_rounds) {
  if (max_rounds < 1) return fail(PMSZ_ERR_INVALID_ARG, "max_rounds must be >= 1");
  return pmsz_session_step_ex(S, max_rounds, 0);
}

int pmsz_session_request_stop(pmsz_session* S) {
  if (!S) return fail(PMSZ_ERR_INVALID_ARG, "NULL session");
  __atomic_store_n(S->stop_word, kStopNow, __ATOMIC_RELEASE);
  return PMSZ_OK;
}

int pmsz_session_request_stop_when_done(pmsz_session* S) {
  if (!S) return fail(PMSZ_ERR_INVALID_ARG, "NULL session");
  unsigned expect = 0u;  // a stop already requested stands
  __atomic_compare_exchange_n(S->stop_word, &expect, kStopWhenDone, false, __ATOMIC_RELEASE,
                              __ATOMIC_RELAXED);
  return PMSZ_OK;
}

int pmsz_session_query(pmsz_session* S, int32_t* running) {
  if (!S || !running) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  *running = 0;
  if (!S->pending) return PMSZ_OK;
  const hipError_t e = hipEventQuery(S->ev);
  if (e == hipErrorNotReady) {
    *running = 1;
    return PMSZ_OK;
  }
  HIP_TRY(e);
  return PMSZ_OK;
}

int pmsz_session_finished(pmsz_session* S, int32_t cap, int32_t* handles, pmsz_stats* stats,
                          int32_t* n) {
  if (!S || !n || (cap > 0 && !handles)) return fail(PMSZ_ERR_INVALID_ARG, "NULL argument");
  const int32_t k = (int32_t)S->finished.size();
  *n = k;
  for (int32_t i = 0; i < k && i < cap; ++i) {
    handles[i] = S->finished[i];
    if (stats) stats[i] = S->fields[S->finished[i]].st;
  }
  return PMSZ_OK;
}

int pmsz_session_step_ex(pmsz_session* S, int64_t max_rounds, int32_t flags) {
  if (!S) return fail(PMSZ_ERR_INVALID_ARG, "NULL session");
  if (S->pending) return fail(PMSZ_ERR_INVALID_ARG, "a step is in flight: sync first");
  if (flags & ~PMSZ_STEP_STOP_ON_DONE) return fail(PMSZ_ERR_INVALID_ARG, "unknown step flags");
  if (max_rounds < 1) max_rounds = -1;  // until every field is done or a stop
  S->stepped.clear();
  std::vector<FieldDesc> fd;
  int64_t tiles = 0, segs = 0;
  int fresh = 0;
  for (int32_t h : S->order) {
    pmsz_session::Entry& e = S->fields[h];
    if (e.done) continue;
    FieldDesc d = e.d;
    d.tile_base = tiles;
    d.seg_base = segs;
    tiles += tile_count(d.geo);
    segs += (d.words + kSegWords - 1) / kSegWords;
    fd.push_back(d);
    S->stepped.push_back(h);
    fresh |= !e.started;
  }
  if (fd.empty()) return PMSZ_OK;
  const int32_t n = (int32_t)fd.size();
  void *up, *down;
  int r = staging(S->up, sizeof(FieldDesc) * (size_t)n, &up);
  if (r) return r;
  r = staging(S->down, kCtlHostBytes + sizeof(FieldIter) * (size_t)n, &down);
  if (r) return r;
  memcpy(up, fd.data(), sizeof(FieldDesc) * (size_t)n);
  HIP_TRY(hipMemcpyAsync(S->ws + S->desc_off, up, sizeof(FieldDesc) * (size_t)n,
                         hipMemcpyHostToDevice, S->stream));
  EngineArgs a;
  a.tiles_swept = 0;
  a.stop_on_done = 0;
  a.stop_host = nullptr;
  a.split_tiles = 0;
  a.fd = (const FieldDesc*)(S->ws + S->desc_off);
  a.out = (FieldIter*)(S->ws + S->out_off);
  a.nf = n;
  a.has_fresh = fresh;
  a.ctl = (EngineCtl*)S->ws;
  a.total_tiles = tiles;
  a.total_segs = segs;
  a.max_rounds = max_rounds;
  a.trace = nullptr;
  a.stop_on_done = (flags & PMSZ_STEP_STOP_ON_DONE) ? 1 : 0;
  a.stop_host = S->stop_word;
  // the step's last launch may hand its last rounds to the tail kernel when
  // the step has no round budget (the tail reads the stop words too)
  a.tail_ok = 0;
  const int32_t tail_ok = (max_rounds < 0 && n <= 256) ? 1 : 0;
  // a stop requested before this launch is spent (the host's store is
  // ordered before the launch that reads the word)
  __atomic_store_n(S->stop_word, 0u, __ATOMIC_RELEASE);
  // Fields starting in this step with kSplitVoxels vertices or more in all:
  // the tile detection of the step's first two rounds runs as plain kernels
  // between engine launches, as in run_batch.  The first round's sweeps
  // cover both the starting fields and the running fields in tile rounds
  // (each sweep takes only the fields of its kind); a field that finishes
  // in the first launch ends the step after the next round.
  int64_t fresh_voxels = 0;
  int dims = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (!S->fields[S->stepped[i]].started) fresh_voxels += fd[i].geo.n;
    dims |= fd[i].geo.ndim == 3 ? 4 : 2;
  }
  int grid = 0;
  if (fresh_voxels >= kSplitVoxels) {
    a.tiles_swept = 1;
    a.max_rounds = 1;
    HIP_TRY(engine_sweep(S->dtype, KIND_FIRST_GIVEN, false, dims, a, S->stream));
    HIP_TRY(engine_sweep(S->dtype, KIND_NEXT, false, dims, a, S->stream));
    HIP_TRY(engine_launch(S->dtype, a, S->stream, &grid));
    a.has_fresh = 0;
    a.max_rounds = max_rounds < 0 ? -1 : max_rounds - 1;
    if (a.max_rounds != 0) {
      HIP_TRY(engine_sweep(S->dtype, KIND_NEXT, false, dims, a, S->stream));
      a.tail_ok = tail_ok;
      HIP_TRY(engine_launch(S->dtype, a, S->stream, &grid));
      if (a.tail_ok) HIP_TRY(engine_tail(S->dtype, a, S->stream));
    }
  } else {
    a.tail_ok = tail_ok;
    HIP_TRY(engine_launch(S->dtype, a, S->stream, &grid));
    if (a.tail_ok) HIP_TRY(engine_tail(S->dtype, a, S->stream));
  }
  HIP_TRY(hipMemcpyAsync(down, S->ws, kCtlHostBytes, hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipMemcpyAsync((char*)down + kCtlHostBytes, a.out, sizeof(FieldIter) * (size_t)n,
                         hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipEventRecord(S->ev, S->stream));
  S->last.tiles = tiles;
  S->last.grid = grid;
  S->pending = true;
  return PMSZ_OK;
}

int pmsz_session_sync(pmsz_session* S, int32_t* n_done) {
  if (!S) return fail(PMSZ_ERR_INVALID_ARG, "NULL session");
  int32_t finished = 0;
  if (S->pending) {
    HIP_TRY(hipEventSynchronize(S->ev));
    S->pending = false;
    const EngineCtl* hc = (const EngineCtl*)S->down.p;
    const FieldIter* hs = (const FieldIter*)((char*)S->down.p + kCtlHostBytes);
    if (hc->error) return fail(PMSZ_ERR_DEVICE, "grid barrier timed out in the correction engine");
    S->epoch = hc->epoch;
    S->last.rounds = (int64_t)hc->rounds;
    S->finished.clear();
    for (size_t i = 0; i < S->stepped.size(); ++i) {
      pmsz_session::Entry& e = S->fields[S->stepped[i]];
      fill_stats(hs[i], e.st);
      if (!hs[i].done) e.st.status = PMSZ_OK;
      e.started = hs[i].started;
      if (hs[i].done && !e.done) {
        e.done = 1;
        ++finished;
        S->finished.push_back(S->stepped[i]);
      }
    }
  }
  if (n_done) *n_done = finished;
  return PMSZ_OK;
}

int pmsz_session_result(pmsz_session* S, int32_t handle, pmsz_stats* stats, int32_t* done) {
  if (!S) return fail(PMSZ_ERR_INVALID_ARG, "NULL session");
  auto it = S->fields.find(handle);
  if (it == S->fields.end()) return fail(PMSZ_ERR_INVALID_ARG, "unknown handle %d", handle);
  if (stats) *stats = it->second.st;
  if (done) *done = it->second.done;
  return PMSZ_OK;
}

int pmsz_session_remove(pmsz_session* S, int32_t handle) {
  if (!S) return fail(PMSZ_ERR_INVALID_ARG, "NULL session");
  if (S->pending) return fail(PMSZ_ERR_INVALID_ARG, "a step is in flight: sync first");
  auto it = S->fields.find(handle);
  if (it == S->fields.end()) return fail(PMSZ_ERR_INVALID_ARG, "unknown handle %d", handle);
  S->fields.erase(it);
  for (size_t i = 0; i < S->order.size(); ++i)
    if (S->order[i] == handle) {
      S->order.erase(S->order.begin() + (long)i);
      break;
    }
  return PMSZ_OK;
}

int pmsz_session_destroy(pmsz_session* S) {
  if (!S) return PMSZ_OK;
  if (S->pending) (void)hipEventSynchronize(S->ev);
  if (S->ev) (void)hipEventDestroy(S->ev);
  if (S->stop_word) (void)hipHostFree(S->stop_word);
  release_staging(S->up);
  release_staging(S->down);
  delete S;
  return PMSZ_OK;
}

}  // extern "C"
