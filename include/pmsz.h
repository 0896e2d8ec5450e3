/*
 * pmsz.h -- C ABI of libpmsz, the gfx950 (MI355X) implementation of the
 * pMSz correction of piecewise-linear Morse-Smale segmentations (PLMSS) in
 * lossy-compressed scalar fields (Li et al., pMSz, arXiv 2601.01787).
 *
 * Problem (Sec. III-B, problem statement): given an original field f, a
 * decompressed field fhat with |f - fhat| <= xi everywhere, produce
 * g = fhat + delta with |f - g| <= xi whose extrema and PLMSS equal those of f.
 * pMSz reaches this with the relaxed sufficient condition of Sec. IV-A: every
 * vertex keeps the steepest-ascent and steepest-descent neighbour it has in f
 * (extrema included), enforced by decrease-only edits (Eq. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid.  Values are stored densely, x fastest: index = x + nx*(y + ny*z).  A 2D
 *   grid has ndim = 2 and nz = 1.  The mesh is the Freudenthal (Kuhn)
 *   triangulation: each square is split along its (0,0)-(1,1) diagonal, each
 *   cube into six tetrahedra around its (0,0,0)-(1,1,1) diagonal.  The
 *   neighbours of a vertex are the 6 (2D) or 14 (3D) offsets +-b where b is a
 *   non-zero 0/1 vector; there is no periodic wrap.  nx*ny*nz must be below
 *   2^31 (vertex ids are int32); a 3D grid also needs (5*nx + 65) times the
 *   value size below 2^32 (nx < 214M for binary32, 107M for binary64).
 * Order.  Vertex a is above vertex b iff h_a > h_b, or h_a == h_b and a > b
 *   (ties broken by index).  n_max(i) / n_min(i) are the highest / lowest
 *   vertex of {i} plus its neighbours (Sec. IV-A); i is a maximum iff
 *   n_max(i) == i (Sec. III-A, extrema).
 * Direction byte.  One uint8 per vertex: bits 0-3 hold the code of n_max(i),
 *   bits 4-7 the code of n_min(i).  Code 0 = the vertex itself; codes 1..7 =
 *   offset +b, and 9..15 = offset -b, where b = (code&1, code>>1&1, code>>2&1)
 *   as (dx, dy, dz).  Code 8 is never produced.
 * Bounds.  xi_T is xi in the field type (for binary32 the nearest float,
 *   stepped toward zero if it rounded up).  lb_i is the smallest value of the
 *   field type >= f_i - xi_T and ub_i the largest <= f_i + xi_T, so a value in
 *   [lb_i, ub_i] satisfies |f_i - g_i| <= xi exactly.
 * Memory.  All array arguments are DEVICE pointers owned by the caller and
 *   must stay valid until the stream work finishes.  Scratch space is a caller
 *   supplied workspace whose size pmsz_workspace_size() reports; the library
 *   keeps no device memory between calls.  Structs marked "host" live in host
 *   memory.
 * Streams.  `stream` is a hipStream_t (NULL = the null stream).  Work is
 *   enqueued on it; the functions that must read results back (correct,
 *   verify, labels) synchronise with it before returning.
 * Errors.  Every function returns a pmsz_status code and never aborts.
 *   Argument errors are reported before any device work is enqueued and
 *   before any caller buffer is written.  pmsz_last_error() returns a
 *   thread-local message about the last failure.
 */
#ifndef PMSZ_H
#define PMSZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PMSZ_OK = 0,
  PMSZ_ERR_INVALID_ARG = 1,   /* bad grid, dtype, pointer, xi or size        */
  PMSZ_ERR_NONFINITE = 2,     /* f or fhat holds a NaN or an infinity        */
  PMSZ_ERR_INPUT_BOUND = 3,   /* fhat outside [lb, ub] somewhere             */
  PMSZ_ERR_NOT_CONVERGED = 4, /* max_iters edit rounds ran, flags remain     */
  PMSZ_ERR_STALLED = 5,       /* every flagged vertex already at its bound   */
  PMSZ_ERR_OOM = 6,           /* workspace too small                         */
  PMSZ_ERR_DEVICE = 7         /* a HIP runtime call failed                   */
} pmsz_status;

typedef enum { PMSZ_F32 = 0, PMSZ_F64 = 1 } pmsz_dtype;

typedef struct {
  int32_t ndim;  /* 2 or 3 */
  int32_t dtype; /* pmsz_dtype */
  int64_t nx, ny, nz;
} pmsz_grid;

/* Result of a correction (host struct). */
typedef struct {
  int64_t iterations;       /* edit rounds applied (0 if fhat already conforms) */
  int64_t steps_applied;    /* value changes summed over all rounds              */
  int64_t flagged_final;    /* size of the flag set at exit (0 when OK)          */
  int64_t stalled_flags;    /* flagged vertices at exit already at their bound   */
  int64_t mismatch_initial; /* (vertex, direction) mismatches of fhat vs f       */
  int32_t status;           /* pmsz_status of the run                            */
  int32_t reserved;
} pmsz_stats;

/* Evaluation counts (Sec. V-D: wrongly labelled points, false extrema). */
typedef struct {
  int64_t bound_violations; /* g outside [lb, ub] or non-finite              */
  int64_t asc_mismatch;     /* n_max under g differs from n_max under f      */
  int64_t desc_mismatch;    /* n_min under g differs from n_min under f      */
  int64_t false_max;        /* maximum in g, not in f                        */
  int64_t false_min;
  int64_t missed_max;       /* maximum in f, not in g                        */
  int64_t missed_min;
  int64_t wrong_max_label;  /* ascending-segmentation label differs          */
  int64_t wrong_min_label;  /* descending-segmentation label differs         */
  int64_t wrong_label;      /* either label differs (PLMSS region differs)   */
  int64_t vertices_edited;  /* g != fhat; -1 when fhat is not given          */
  double max_abs_err;       /* max |g - f| evaluated in binary64             */
} pmsz_report;

/* One member of a batch (host struct). */
typedef struct {
  pmsz_grid grid;
  const void* f; /* device, original field                        */
  void* g;       /* device, in: fhat, out: corrected field        */
  double xi;     /* absolute error bound of this field            */
} pmsz_field;

/* Workspace kinds for pmsz_workspace_size. */
enum { PMSZ_WS_CORRECT = 0, PMSZ_WS_VERIFY = 1, PMSZ_WS_LABELS = 2, PMSZ_WS_CORRECT_TARGETED = 3 };

/* Edit rules for pmsz_correct_mode. */
enum { PMSZ_EDIT_HALVING = 0, PMSZ_EDIT_TARGETED = 1 };

/* Bytes of device workspace that operation `op` needs for `grid`
 * (*bytes, host).  Returns PMSZ_ERR_INVALID_ARG for a bad grid or op. */
int pmsz_workspace_size(const pmsz_grid* grid, int op, size_t* bytes);

/* Steepest directions of a field (Sec. IV-A: n_min(i) and n_max(i) over the
 * neighbourhood; Sec. III-A: extrema are the vertices pointing at themselves).
 * field: device, nx*ny*nz values of grid->dtype.  dirs: device, nx*ny*nz
 * direction bytes (layout above), written.  Values must be finite; with a
 * non-finite value the bytes are unspecified.  Asynchronous on `stream`. */
int pmsz_directions(const pmsz_grid* grid, const void* field, uint8_t* dirs, void* stream);

/* The pMSz correction (Sec. III-B Eq. 1 with the FPmax rule; Sec. IV-A
 * ascending and descending rules), on one field:
 *   k = 0; repeat:
 *     F = { n_max^g(i) : n_max^g(i) != n_max^f(i) } u { n_min^f(i) : n_min^g(i) != n_min^f(i) }
 *         computed from g^k alone (Jacobi);
 *     F empty                        -> PMSZ_OK
 *     every t in F has g_t == lb_t   -> PMSZ_ERR_STALLED
 *     k == max_iters                 -> PMSZ_ERR_NOT_CONVERGED
 *     for t in F at once: g_t <- lb_t + (g_t - lb_t)/2 rounded, or lb_t when
 *     that would not decrease g_t (the edit size delta is left open by the
 *     paper; this halving is the reading used here); k += 1.
 * f: device, original field.  g: device, in: fhat, out: the last iterate
 * (always within [lb, fhat]).  dirs_f: device direction bytes of f, or NULL
 * to compute them into the workspace; given bytes are checked first (every
 * code must be 0 or name a neighbour of its vertex inside the grid: no code
 * 8, no z bit in 2D), and any invalid one returns PMSZ_ERR_INVALID_ARG with g
 * untouched.  ws: device workspace of at least
 * pmsz_workspace_size(grid, PMSZ_WS_CORRECT) bytes, 256-byte aligned.
 * max_iters >= 0.  stats: host, filled on every return after argument checks
 * (status mirrors the return code).  Validation failures (NONFINITE,
 * INPUT_BOUND) leave g unchanged.  Synchronises with `stream`. */
int pmsz_correct(const pmsz_grid* grid, const void* f, void* g, double xi,
                 const uint8_t* dirs_f, void* ws, size_t ws_bytes, int64_t max_iters,
                 pmsz_stats* stats, void* stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): pmsz_correct without a workspace argument.
 * Same arguments, results and errors as pmsz_correct (halving edit), except
 * that the workspace is the library's own static device array of 32 MiB
 * (PMSZ_NOALLOC_SCRATCH_BYTES; each device that runs it holds one copy until
 * the process ends).  A field whose pmsz_workspace_size(grid, PMSZ_WS_CORRECT)
 * exceeds it is refused with PMSZ_ERR_OOM before anything runs (binary32
 * 256^3 fits: 18.4 MiB; a 4096^2 2D field: 18.6 MiB).  The call allocates
 * nothing: no hipMalloc, no pinned host memory, no events; its host staging
 * lives on the caller's stack.  The stream must belong to the current device.
 * Every call on one device shares that device's array and clears what must
 * start at zero itself: calls that overlap on one device (two host threads,
 * or two streams) race and give undefined results; serialise them. */
#define PMSZ_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int pmsz_correct_noalloc(const pmsz_grid* grid, const void* f, void* g, double xi,
                         const uint8_t* dirs_f, int64_t max_iters, pmsz_stats* stats,
                         void* stream);

/* pmsz_correct with a choice of edit rule.  PMSZ_EDIT_HALVING is
 * pmsz_correct.  PMSZ_EDIT_TARGETED follows the worked examples of Sec. IV-A,
 * where a vertex is lowered to its rival's value "or slightly below": every
 * flag carries a proposal for its target, the highest value at which the
 * target no longer beats its rival in the (value, index) order (ascending
 * rule: the rival is n_max^f(i); descending rule: the current n_min^g(i)),
 * i.e. the rival's value when the target has the smaller index, else the next
 * value below it (+0 for zero); each flagged t then takes
 * max(lb_t, smallest proposal).  The stopping rules are those of
 * pmsz_correct.  ws: pmsz_workspace_size(grid, PMSZ_WS_CORRECT_TARGETED)
 * bytes for the targeted rule (one proposal word of the value size per
 * vertex more).  An unknown mode returns PMSZ_ERR_INVALID_ARG. */
int pmsz_correct_mode(const pmsz_grid* grid, const void* f, void* g, double xi,
                      const uint8_t* dirs_f, int edit_mode, void* ws, size_t ws_bytes,
                      int64_t max_iters, pmsz_stats* stats, void* stream);

/* Batched correction of n independent fields in one persistent launch.  Each
 * field follows exactly the iteration of pmsz_correct (bit-identical results
 * and statistics); fields retire independently.  fields, stats: host arrays
 * of n.  ws: device workspace of pmsz_batched_workspace_size() bytes.
 * Returns PMSZ_OK when every field converged, otherwise the first non-OK
 * field status (per-field codes are in stats).  Synchronises with `stream`. */
int pmsz_batched_workspace_size(int32_t n, const pmsz_field* fields, size_t* bytes);
int pmsz_correct_batched(int32_t n, const pmsz_field* fields, void* ws, size_t ws_bytes,
                         int64_t max_iters, pmsz_stats* stats, void* stream);

/* Tile shapes.  The correction sweeps each field in tiles of 64 x 4 columns
 * (3D) or 256-wide strips (2D) of `h` planes / rows, h between 2 and 32,
 * chosen to give about `tiles_target` tiles per field (without a set or
 * tuned target: 2048 / n for a batch of n fields, between 32 and 256; 256 for
 * a serving session's fields).  The
 * tile height changes neither results nor statistics, only speed (the
 * iteration of Sec. IV-A is the same; the tiles only decide which vertices a
 * detect pass reads).  The target is kept per (ndim, dtype) for the whole
 * process and read when a correction, batch or session field is planned.
 * pmsz_set_tiles_target: 0 restores the default rule, which
 * pmsz_get_tiles_target reports as 0.  Host-only, thread-safe.
 * Tune cache: when the environment variable PMSZ_TUNE_CACHE names a file,
 * the targets it records (a JSON object with the keys "2d_f32", "2d_f64",
 * "3d_f32", "3d_f64"; absent keys and unreadable or malformed files keep the
 * default) are installed before the first target is read or set in the
 * process, and pmsz_tune_tiles rewrites the file with every current target
 * (PMSZ_ERR_INVALID_ARG when it cannot be written; the tuned target is
 * installed either way).
 * pmsz_tune_tiles: the autotuner.  Corrects the batch `fields` (g holds fhat
 * and is NOT modified; copies are corrected in ws) once per candidate target,
 * `reps` times each, measures the device time of each run (directions pass +
 * engine, HIP events), writes the best time per candidate into ms (host,
 * n_candidates; may be NULL), sets the fastest target for the batch's (ndim,
 * dtype) and returns it in *best.  All fields must share ndim and dtype.
 * ws: device, 256-byte aligned, pmsz_tune_workspace_size() bytes.
 * Synchronises with `stream`. */
int pmsz_set_tiles_target(int32_t ndim, int32_t dtype, int32_t tiles_target);
int pmsz_get_tiles_target(int32_t ndim, int32_t dtype, int32_t* tiles_target);
int pmsz_tune_workspace_size(int32_t n, const pmsz_field* fields, size_t* bytes);
int pmsz_tune_tiles(int32_t n, const pmsz_field* fields, const int32_t* candidates,
                    int32_t n_candidates, int32_t reps, void* ws, size_t ws_bytes, double* ms,
                    int32_t* best, void* stream);

/* Decomposed domain (Sec. IV-B, domain decomposition, ghost layer
 * synchronisation and relaxed synchronisation), run on one GPU: the grid is
 * cut into blocks[0] x blocks[1] x blocks[2] blocks (blocks[2] == 1 in 2D);
 * along an axis of n vertices cut b ways, block k owns
 * [floor(k n / b), floor((k+1) n / b)), and its copy spans one more vertex on
 * each side that has a neighbour block (the ghost layer).  A phase corrects
 * every block's copy (only owned vertices are compared; a flag may lower a
 * ghost copy), then exchanges: every vertex takes the smallest of its copies
 * in all of them and in g.  per_round = 0: each block runs to local
 * convergence (at most max_iters rounds) before the exchange (pMSz);
 * per_round = 1: one edit round per block between exchanges (sync-pMSz).  The
 * loop ends with PMSZ_OK when every block's last check found no mismatch and
 * the exchange lowered no copy; PMSZ_ERR_STALLED (or NOT_CONVERGED) when a
 * phase changed no value; PMSZ_ERR_NOT_CONVERGED after max_phases phases.
 * Results are valid corrections but differ from pmsz_correct on the whole
 * grid (the blocks' iterate sequences differ).  f, g: device fields of `grid`
 * (g: fhat in, result out; left unchanged when the inputs are rejected).
 * blocks: host, three counts in [1, extent].  ws: device, 256-byte aligned,
 * pmsz_blocks_workspace_size() bytes (copies of f and g per block, their
 * direction bytes and an engine workspace for the blocks).  stats: host.
 * Synchronises with `stream`. */
typedef struct {
  int64_t phases;          /* exchanges performed                                */
  int64_t local_rounds;    /* edit rounds summed over blocks and phases          */
  int64_t critical_rounds; /* per phase the most rounds of any block, summed:
                              the schedule's length with one GPU per block      */
  int64_t lowered;         /* block copies lowered by the exchanges             */
  int64_t steps_applied;   /* value changes made by the local corrections      */
  double compute_ms;       /* device time of the local corrections, all phases */
  double exchange_ms;      /* device time of the exchanges, all phases         */
  int32_t status;          /* pmsz_status of the run                            */
  int32_t reserved;
} pmsz_blocks_stats;
int pmsz_blocks_workspace_size(const pmsz_grid* grid, const int32_t* blocks, size_t* bytes);
int pmsz_correct_blocks(const pmsz_grid* grid, const void* f, void* g, double xi,
                        const int32_t* blocks, int32_t per_round, int64_t max_phases,
                        int64_t max_iters, void* ws, size_t ws_bytes, pmsz_blocks_stats* stats,
                        void* stream);

/* Edit stream: the corrections as stored next to the compressed field
 * (Sec. V-D reports this storage as the method's overhead; the format is this
 * library's).  Layout, little-endian:
 *   header  "PMSE", u8 version 1, u8 dtype, u16 0, u64 vertices, u64 edits,
 *           u64 payload bytes, u32 chunk (4096), u32 chunks   (40 bytes)
 *   table   per chunk of 4096 entries: u64 payload offset of its first entry,
 *           u64 index of the edited vertex before it (all ones when none)
 *   payload per vertex i whose bits differ between fhat and g, ascending:
 *           gap = i - previous edited index - 1, then steps = the number of
 *           representable values in (g_i, fhat_i], each an unsigned LEB128
 *           varint.
 * pmsz_edits_workspace_size: device workspace for encoding up to max_edits
 * edits.  pmsz_edits_max_bytes: stream capacity that any n_edits edits fit.
 * pmsz_encode_edits: fhat, g: device fields of `grid`; out: device, 8-byte
 * aligned, out_cap bytes.  Sets *n_edits and *n_bytes (stream length); with
 * more than max_edits edits returns PMSZ_ERR_OOM with *n_edits set and writes
 * nothing; likewise when the stream exceeds out_cap (*n_bytes set).
 * Synchronises.  pmsz_decode_edits: g holds fhat on entry and the corrected
 * field on return; in: device stream of n_bytes bytes, 8-byte aligned; ws: 256
 * device bytes, 256-byte aligned.  A stream of another grid or type, or a
 * malformed payload, returns PMSZ_ERR_INVALID_ARG (with a malformed payload g
 * may be partly written).  Synchronises. */
int pmsz_edits_workspace_size(const pmsz_grid* grid, int64_t max_edits, size_t* bytes);
int pmsz_edits_max_bytes(int64_t n_edits, size_t* bytes);
int pmsz_encode_edits(const pmsz_grid* grid, const void* fhat, const void* g, int64_t max_edits,
                      void* ws, size_t ws_bytes, uint8_t* out, size_t out_cap, int64_t* n_edits,
                      int64_t* n_bytes, void* stream);
int pmsz_decode_edits(const pmsz_grid* grid, const uint8_t* in, size_t n_bytes, void* g,
                      void* ws, size_t ws_bytes, void* stream);

/* Segmentation labels (Sec. III-A: integral lines end at an extremum; the
 * ascending / descending segmentation groups vertices by that extremum).
 * dirs: device direction bytes.  max_label / min_label: device int32 arrays of
 * nx*ny*nz, written with the index of the maximum (resp. minimum) reached by
 * following n_max (resp. n_min); either may be NULL.  ws: device workspace of
 * pmsz_workspace_size(grid, PMSZ_WS_LABELS) bytes, 256-byte aligned.  The
 * labels are found by pointer jumping in place on the device, passes queued
 * in batches with one read-back per batch.  Bytes holding a code that does
 * not name a neighbour inside the grid, or pointers that do not form a
 * forest (never the case for bytes made by pmsz_directions), return
 * PMSZ_ERR_INVALID_ARG; the label arrays are then unspecified.
 * Synchronises. */
int pmsz_labels(const pmsz_grid* grid, const uint8_t* dirs, int32_t* max_label,
                int32_t* min_label, void* ws, size_t ws_bytes, void* stream);

/* Work and device time of the last pmsz_labels on this thread (pmsz_verify
 * runs it twice; the record is the second run's).  Host struct. */
typedef struct {
  int64_t vertices;    /* vertices labelled                                   */
  int64_t passes_max;  /* pointer-jumping passes of the max labels (the last
                          one found nothing to change; 0 when not requested)  */
  int64_t passes_min;  /* the same for the min labels                         */
  double ms;           /* device time from the first to the last kernel (HIP
                          events on the caller's stream)                      */
} pmsz_labels_info;
int pmsz_last_labels(pmsz_labels_info* out);

/* Evaluation counts of Sec. V-D, recomputed from (f, g) from scratch: bound
 * violations, direction mismatches, false / missed extrema, wrong labels,
 * edited vertices (needs fhat, else -1) and max |g - f|.  f, g, fhat: device
 * (fhat may be NULL).  ws: pmsz_workspace_size(grid, PMSZ_WS_VERIFY) bytes.
 * report: host.  Synchronises with `stream`. */
int pmsz_verify(const pmsz_grid* grid, const void* f, const void* g, const void* fhat,
                double xi, void* ws, size_t ws_bytes, pmsz_report* report, void* stream);

/* ---------------------------------------------------------------------------
 * Serving sessions (continuous batching).  Fields are admitted and retired
 * between steps; one step is one launch of the persistent correction kernel
 * over every admitted, unfinished field, running at most max_rounds rounds.
 * A field's iterate sequence, result and statistics are those of
 * pmsz_correct on the same field alone, whatever else shares its steps.
 * All calls except pmsz_session_sync are asynchronous on the session stream.
 * ------------------------------------------------------------------------- */
typedef struct pmsz_session pmsz_session;

/* Device bytes of a session's own workspace for up to max_fields fields. */
int pmsz_session_workspace_size(int32_t max_fields, size_t* bytes);
/* Device bytes of the per-field workspace of one admitted field (its flag
 * bitmap, direction bytes, tile activity and iteration state). */
int pmsz_field_workspace_size(const pmsz_grid* grid, size_t* bytes);
/* Create a session for fields of one dtype.  ws: device, 256-byte aligned,
 * pmsz_session_workspace_size(max_fields) bytes, owned by the caller until
 * pmsz_session_destroy.  stream: the hipStream_t every step runs on. */
int pmsz_session_create(int32_t dtype, int32_t max_fields, void* ws, size_t ws_bytes,
                        void* stream, pmsz_session** out);
/* Admit a field: f and g (fhat on entry) as in pmsz_correct, plus its own
 * field workspace (device, 256-byte aligned).  It joins the next step.  The
 * caller keeps f, g and field_ws alive until the field is removed.  *handle
 * receives the field's id.  Fails with PMSZ_ERR_OOM when the session is full. */
int pmsz_session_add(pmsz_session* s, const pmsz_field* field, int64_t max_iters, void* field_ws,
                     size_t field_ws_bytes, int32_t* handle);
/* Enqueue one step (max_rounds >= 1).  At most one step may be in flight. */
int pmsz_session_step(pmsz_session* s, int64_t max_rounds);
/* pmsz_session_step with max_rounds < 1 meaning "until every field is done",
 * and flags: PMSZ_STEP_STOP_ON_DONE ends the step after the round in which a
 * field is first seen finished (its result can then be collected while the
 * others continue in the next step).  A step also ends after the round in
 * progress when pmsz_session_request_stop is called (at most two rounds
 * later).  Results do not depend on where steps end. */
#define PMSZ_STEP_STOP_ON_DONE 1
int pmsz_session_step_ex(pmsz_session* s, int64_t max_rounds, int32_t flags);
/* Asks the step in flight to end after its current round (a new request is
 * waiting); thread-safe; spent by the next step's launch. */
int pmsz_session_request_stop(pmsz_session* s);
/* Asks the step in flight to end after the first round that begins with one
 * of its fields done (at most two rounds after that field finished), so that
 * finished fields can be collected without ending every step at the first
 * one; overrides nothing (a pending pmsz_session_request_stop stands).
 * Thread-safe; spent by the next step's launch. */
int pmsz_session_request_stop_when_done(pmsz_session* s);
/* *running = 1 while the step in flight has not ended (non-blocking). */
int pmsz_session_query(pmsz_session* s, int32_t* running);
/* After a sync: the handles (up to cap) and stats of the fields that
 * finished in that step; *n receives their number. */
int pmsz_session_finished(pmsz_session* s, int32_t cap, int32_t* handles, pmsz_stats* stats,
                          int32_t* n);
/* Wait for the step in flight and collect its results; *n_done (nullable)
 * receives how many fields finished in it. */
int pmsz_session_sync(pmsz_session* s, int32_t* n_done);
/* Statistics of a field after the last sync (host structs); *done is 1 once
 * the field has finished (stats->status is then final). */
int pmsz_session_result(pmsz_session* s, int32_t handle, pmsz_stats* stats, int32_t* done);
/* Retire a field (no step in flight); its buffers may be freed afterwards. */
int pmsz_session_remove(pmsz_session* s, int32_t handle);
int pmsz_session_destroy(pmsz_session* s);

/* Measurements of the last pmsz_correct / pmsz_correct_batched call made on
 * this thread (host struct): the durations of its kernels, timed with HIP
 * events recorded on the caller's stream around each launch, and the work it
 * did.  Used by the benchmark for roofline figures. */
typedef struct {
  double engine_ms;  /* the persistent correction kernel (all its launches),
                        with round 0's apply kernel of large batches and the
                        tail kernel                                           */
  int64_t rounds;    /* detect/apply rounds run                               */
  int64_t swept;     /* vertices examined by detect passes, all rounds        */
  int64_t edits;     /* value changes, all fields                             */
  int64_t voxels;    /* vertices of the batch                                 */
  int64_t tiles;     /* tiles of the batch                                    */
  int32_t grid;      /* blocks of the cooperative launch                      */
  int32_t sweeps;    /* tile sweeps run as kernels of their own (large
                        batches: 2 for rounds 0 and 1, one more per later
                        round with a large tile sweep; else 0)                 */
  double first_round_ms; /* first round: validation, detect, apply            */
  double detect_ms;  /* detect phases of the later rounds (block 0's clock)    */
  double apply_ms;   /* apply phases of the later rounds                       */
  double dirs_ms;    /* directions of f, computed before the correction kernel
                        (0 when the caller gave them)                           */
  double sweep_ms;   /* the sweep kernels; engine_ms covers the engine
                        launches only (with the tail kernel's)                  */
  int32_t tail_rounds; /* rounds run by the tail kernel: the sparse rounds
                        after a round with few edits, on the blocks of one
                        XCD (Sec. IV-A's loop, unchanged)                       */
  int32_t handbacks; /* times the tail kernel stopped before a round with
                        tile sweeps and the engine was launched again          */
} pmsz_timing;
int pmsz_last_timing(pmsz_timing* out);

/* Per-round record of the last pmsz_correct / pmsz_correct_batched on this
 * thread, for the first 64 rounds of the launch (diagnostics of the loop of
 * Sec. IV-A).  Times are block 0's view on the device clock; the counts are
 * totals over every field of the launch.  Round 0's detect_ms runs from the
 * launch start. */
typedef struct {
  double detect_ms;  /* start of the round to the end of its detect pass   */
  double apply_ms;   /* end of detect to the end of the apply pass          */
  int64_t swept;     /* vertices examined by the detect pass                */
  int64_t flagged;   /* |F|: distinct flagged vertices                      */
  int64_t edits;     /* values changed by the apply pass                    */
  int64_t sparse;    /* of `swept`, examinations of a sparse round (the
                        neighbours of the previous round's targets); the
                        rest were swept in tiles                               */
} pmsz_round;

/* Copies min(cap, rounds recorded) records into out[] (host) and stores the
 * number recorded (<= 64) in *n.  Returns PMSZ_ERR_INVALID_ARG if n is NULL,
 * or if out is NULL while cap > 0. */
int pmsz_last_rounds(pmsz_round* out, int64_t cap, int64_t* n);

/* Counter calibration (measurement aid, not part of the method): reads the
 * `bytes` bytes at device address p exactly once, as rows of dwords (pattern
 * 0: 256 contiguous bytes per 64-lane load, the shape of a plane row of
 * binary32 values in the tile marches; bytes a multiple of 4) or rows of
 * bytes (pattern 1: 64 contiguous bytes per load, the shape of a row of
 * direction bytes), and stores in *sum (host) the sum of the dwords / bytes.
 * A memory counter's reading for this launch, against `bytes`, calibrates
 * that counter for the pattern.  Allocates 8 bytes of device memory for the
 * call.  Synchronises with `stream`. */
int pmsz_probe_read(const void* p, int64_t bytes, int32_t pattern, uint64_t* sum, void* stream);

/* Frees the host resources the library keeps for reuse across calls (pinned
 * staging buffers and HIP events of every thread).  They are never freed by
 * destructors at thread or process exit, where the HIP runtime may already be
 * gone; call this before the process ends, while the runtime is up and no
 * other call of the library is running (the Python binding calls it from an
 * exit hook).  Later calls allocate them again.  Always PMSZ_OK. */
int pmsz_release(void);

/* Name of a status code (static string). */
const char* pmsz_status_string(int status);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* pmsz_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMSZ_H */
