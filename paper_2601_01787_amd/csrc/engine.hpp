// engine.hpp -- data of the persistent correction engine (internal).
//
// One cooperative launch runs the whole correction loop of Sec. IV-A for one
// or many fields: rounds of [detect over active tiles] -> grid barrier ->
// [apply edits] -> grid barrier, with per-field state so that fields of any
// size converge and retire independently.  The same structures serve a single
// field, a batch run to completion, and resumable serving steps.
#pragma once

#include <stddef.h>

#include "tiles.hpp"

namespace pmsz {

constexpr int64_t kSegWords = 4096;  // bitmap words per apply segment (128K vertices)

// Iteration state of one field at the start of a round.  Double-buffered by
// round parity: during round E block 0 persists the state of round E while
// every block derives it on the fly from the state and counters of round E-1.
struct FieldIter {
  unsigned long long k, steps, mism0, flagged_final, stalled_final, swept;
  int32_t status, done, started, pad;
};

// Counters of one round.  Triple-buffered by round index mod 3: round E adds
// to c[E%3], reads c[(E-1)%3], and clears c[(E+1)%3].  Each counter is spread
// over kCtrSlots slots on separate 128-byte lines (block b adds to slot
// b % kCtrSlots) and a count is the sum over the slots: atomics on one line
// serialise at about 11 ns each, so one line shared by 1024 blocks cost
// 10-40 us per round.
constexpr int kCtrSlots = 8;
struct alignas(128) CtrSlot {
  unsigned long long mism, nflag, at_lb, bad_nf, bad_b, swept;
  unsigned long long nlist;  // targets this slot's blocks appended to the target list
  unsigned long long pad;
};
struct FieldCtr {
  CtrSlot s[kCtrSlots];
};
// Sums over the slots.
struct CtrSum {
  unsigned long long mism, nflag, at_lb, bad_nf, bad_b, swept, nlist;
};

struct FieldState {
  FieldIter s[2];
  FieldCtr c[3];
};

// Read-only description of one field (uploaded by the host).
struct FieldDesc {
  const void* f;      // original field
  void* g;            // in: fhat, out: corrected
  uint8_t* dirs;      // direction bytes of f (workspace, or the caller's)
  uint32_t* bm;       // flag bitmap of this field
  FieldState* st;     // iteration state and counters of this field
  uint8_t* act;       // per tile and round parity: examine in that round
                      // (act[p * tiles + tile])
  uint32_t* list;     // targets of the last apply pass (list_cap entries, in
                      // kCtrSlots slices of list_cap / kCtrSlots, one per slot)
  uint8_t* marks;     // per apply segment: a tail round's examination flagged a
                      // vertex in it (set by detect, cleared by apply)
  void* prop;         // targeted edit: per-vertex proposal keys; nullptr for
                      // the halving edit
  TileGeo geo;
  double xi_t;        // xi in the field type, <= xi
  int64_t max_iters;
  int64_t tile_base;  // first global tile index
  int64_t seg_base;   // first global apply segment
  int64_t words;      // bitmap words
  int32_t dirs_given; // caller supplied the directions of f
  int32_t list_cap;   // capacity of the target list
};

// Grid barrier words, each on its own 256-byte line: arrivals are spread over
// counters whose last arrivals meet at a top counter, and the waiting blocks
// poll a generation word that no arrival touches.  The start-of-launch
// barrier groups blocks by block index (kBarGroups groups); every later one
// groups them by the XCD they run on (up to kXcdSlots), so that one block per
// XCD writes that XCD's L2 back, and elects one block per compute unit
// (kCuSlots: XCD x the 8-bit unit id of the hardware register HW_ID) to
// invalidate that unit's caches.
constexpr int kBarGroups = 32;
constexpr int kXcdSlots = 16;
constexpr int kCuSlots = kXcdSlots * 256;
struct alignas(256) BarWord {
  unsigned v;
  unsigned pad[63];
};

struct alignas(128) RoundTot {
  unsigned long long edits;    // value changes
  unsigned long long swept;    // vertices examined
  unsigned long long sparse;   // of which by sparse examination
  unsigned long long flagged;  // flagged vertices
  unsigned long long pad[4];
};

struct EngineCtl {
  BarWord bar_gen;
  BarWord bar[kBarGroups + 1];  // group counters, then the top counter
  // results of a launch (the host reads back the first kCtlHostBytes bytes)
  unsigned long long epoch;     // rounds run since the workspace was initialised
  unsigned long long rounds;    // rounds run by the last launch
  int error;                    // a grid barrier timed out
  int handoff;                  // how the last launch ended: kHandToTail, kHandToEngine,
                                // kTailDone, or 0 (an engine launch that kept its rounds)
  // per-launch barrier state, cleared before every launch (from xbar up to tot)
  BarWord xbar[kXcdSlots];      // arrivals per XCD
  BarWord xtop;                 // XCDs arrived
  BarWord stop;                 // nonzero: the launch ends after the current round
  BarWord lead;                 // k_tail: 1 + the XCD of block 0, where the tail runs
  BarWord arrived;              // k_tail: blocks that have read their XCD
  unsigned census[kXcdSlots];   // blocks of the launch on each XCD
  unsigned census_pad[64 - kXcdSlots];
  unsigned cu_claim[kCuSlots];  // last barrier generation claimed on each unit
  unsigned cu_done[kCuSlots];   // last generation whose invalidate completed
  // totals over all fields per round (mod 3), spread over slots like FieldCtr;
  // cleared a round ahead by block 0, like the field counters
  RoundTot tot[3][kCtrSlots];
};
constexpr size_t kCtlHostBytes = offsetof(EngineCtl, xbar);

// Batches (and fields) of at least this many vertices run their tile sweeps
// as kernels of their own (engine_sweep) where the host can place them.
constexpr int64_t kSplitVoxels = int64_t(1) << 23;

// Tail rounds: once a round edits few enough vertices that the next round's
// examinations (at most 15 per edit) come to at most kTailExams per thread of
// one XCD's share of the grid, the engine launch ends (handoff kHandToTail)
// and k_tail runs the following sparse rounds on the blocks of one XCD alone.
// They share one L2, so their barriers need no L2 write-back and their loads
// find each other's data in that L2 instead of in HBM.  A round in which a
// field sweeps tiles ends k_tail before it starts (handoff kHandToEngine) and
// the host launches the engine again.
constexpr int kTailExams = 4;
constexpr int kTailGrid = 256;  // blocks of a tail launch (32 per XCD)
// The tail's apply pass takes each segment marked by its detection whole: the
// engine hands over only once a round edits at most kTailSegs vertices (or
// the batch has at most kTailSegs segments), so that the marks stay few.
constexpr int64_t kTailSegs = 128;
constexpr int kHandToTail = 1, kHandToEngine = 2, kTailDone = 3;

// Values of the host's stop word: end the launch after the current round;
// end it after a round that begins with a field of the launch done.
constexpr unsigned kStopNow = 1u, kStopWhenDone = 2u;

struct EngineArgs {
  const FieldDesc* fd;
  FieldIter* out;        // state of every field at the end of the launch
  int32_t nf;
  int32_t has_fresh;     // some field has not started: all its tiles are active
  EngineCtl* ctl;
  int64_t total_tiles;
  int64_t total_segs;
  int64_t max_rounds;    // < 0: until every field is done
  unsigned long long* trace;  // nullable: per-round record (kTraceRounds x kTraceSlots)
  int32_t tiles_swept;   // the tile detection of the launch's first round has
                         // already run as its own kernel (engine_sweep)
  int32_t stop_on_done;  // end the launch after the round in which a field is
                         // first seen finished
  unsigned* stop_host;   // nullable, host memory: kStopNow / kStopWhenDone (below),
                         // read by block 0 at the start of every round
  int32_t split_tiles;   // end the launch before a round, other than its first, in
                         // which a field of kSplitVoxels vertices or more (among
                         // the first 256) sweeps tiles: a sweep kernel takes that
                         // round's tile detection and the next launch the rest
  int32_t tail_ok;       // the launch may hand its last rounds to k_tail (at most
                         // 256 fields; the host launches k_tail after it)
};

// Round trace, for the first kTraceRounds rounds since the workspace was
// initialised (indexed by the round number E): block 0 stamps
// the 100 MHz wall clock at the start of a round, after its detect barrier
// and after its apply barrier, then copies the round's totals (vertices
// examined, flagged vertices, edits, sparse examinations); slot
// kTraceRounds*kTraceSlots holds the launch start.
constexpr int kTraceRounds = 64;
constexpr int kTraceSlots = 7;
constexpr size_t kTraceBytes = (kTraceRounds * kTraceSlots + 1) * 8;

// Host side (engine.hip).
// clear: clear the launch's barrier state first (not needed on a workspace
// cleared since the last launch).
hipError_t engine_launch(int dtype, const EngineArgs& a, hipStream_t s, int* grid_out,
                         bool clear = true);
// The tail (k_tail) after an engine launch with tail_ok set: ends at once
// unless that launch handed its remaining rounds over.
hipError_t engine_tail(int dtype, const EngineArgs& a, hipStream_t s);
// Directions of f, before the engine, for every field of the device table fd
// whose dirs_given is 0 (into its dirs); the engine then starts every field
// from given directions.
hipError_t engine_dirs(int dtype, const FieldDesc* fd, int nf, int64_t total_tiles,
                       hipStream_t s);
// Tile detection of one round as a plain kernel (no grid barrier, so it runs
// at the march's own occupancy instead of the persistent engine's), for the
// round the workspace's epoch names: every tile of a field in its first
// round (kind KIND_FIRST_GIVEN) or every marked tile of a field in a tile
// round (KIND_NEXT); fields of the other kind, finished fields and fields in
// a sparse round are left to the engine.  The engine launch that follows
// sets tiles_swept and skips its first round's tile detection.
// prop: the batch uses the targeted edit (flags also propose values).  dims:
// bit 2 set when the batch holds 2D fields, bit 4 when it holds 3D fields
// (one kernel per dimension, each at its own occupancy).
hipError_t engine_sweep(int dtype, int kind, bool prop, int dims, const EngineArgs& a,
                        hipStream_t s);

// Round 0's apply pass as a plain kernel after a round-0 sweep, then the end
// of round 0 (every field's state at round 1, epoch 1, the round's record):
// the engine launch that follows starts at round 1.
hipError_t engine_apply_first(int dtype, const EngineArgs& a, hipStream_t s);

// Zero `bytes` bytes (multiple of 4, 4-byte aligned) with a kernel, so that
// the call can sit inside a captured graph.
hipError_t engine_zero(void* p, size_t bytes, hipStream_t s);
// Fill `bytes` bytes (multiple of 4, 4-byte aligned) with the 32-bit word v.
hipError_t engine_fill(void* p, size_t bytes, uint32_t v, hipStream_t s);

// Target list: the apply pass lists its targets, the pass over apply segment
// k in slice k mod S of the list (S = min(kCtrSlots, the field's segments),
// list_capacity / S entries each, counted in that counter slot); when no
// slice overflowed, the next round examines the Freudenthal neighbours of
// exactly those vertices instead of sweeping tiles.  A field of few segments
// thus keeps the whole capacity in few slices.  The capacity sits near the
// break-even point: examining one neighbour of a listed target costs about 15
// (3D) to 16 (2D) times one vertex of a tile sweep (measured), and a target
// has 15 (3D) or 7 (2D) of them, so sparse rounds pay below about N/222
// (3D) or N/112 (2D) targets.
inline int32_t list_capacity(const TileGeo& G) {
  return (G.ndim == 3 ? G.n / 256 : G.n / 128) + 1024;
}
__host__ __device__ inline int32_t list_slices(int64_t words) {
  const int64_t segs = (words + kSegWords - 1) / kSegWords;
  return segs < kCtrSlots ? (int32_t)(segs > 0 ? segs : 1) : kCtrSlots;
}

// Per-field workspace: [FieldState][activity bytes x 2][bitmap][target list]
// [segment marks][directions].
struct FieldLayout {
  size_t state, act, bm, list, marks, dirs, total;
};
inline size_t ws_align(size_t v) { return (v + 255) / 256 * 256; }
inline FieldLayout field_layout(const TileGeo& G, bool dirs_given) {
  FieldLayout L;
  L.state = 0;
  // activity bytes sized for the shortest tiles (2 planes / rows), so that a
  // field's workspace fits any tile height the tuner may pick
  const int64_t depth = G.ndim == 3 ? G.nz : G.ny;
  const size_t max_tiles = (size_t)G.tiles_x * (G.ndim == 3 ? G.tiles_y : 1) * ((depth + 1) / 2);
  L.act = ws_align(sizeof(FieldState));
  L.bm = L.act + ws_align(2 * max_tiles);
  L.list = L.bm + ws_align(((size_t)G.n + 31) / 32 * 4);
  L.marks = L.list + ws_align((size_t)list_capacity(G) * 4);
  L.dirs = L.marks + ws_align((size_t)((G.n + 32 * kSegWords - 1) / (32 * kSegWords)));
  L.total = L.dirs + (dirs_given ? 0 : ws_align((size_t)G.n));
  return L;
}

// Tile height (planes per 3D tile, rows per 2D strip) for the engine: about
// `tiles_target` tiles per field, between 2 and 32 planes / rows.  The target
// is the autotuned knob; results do not depend on it.  Without a set or
// tuned target a batch of nf fields takes 2048 / nf, between 32 and 256: a
// field of up to a few million vertices runs fastest in about 256 tiles
// (fewer, taller tiles than blocks: a march's first planes are halo), and a
// batch of many fields in about 32 each (measured on one MI355X, device time
// per correction against a target of 2048: 64^3 267 against 286 us, 96^3 338
// against 392 us, 1024^2 315 against 380 us; the 256-field batch 15.4 ms at
// 32 against 16.2 ms at 256).  Large fields reach the 32-plane limit at any
// of these targets.
inline int32_t default_tiles_target(int64_t nf) {
  const int64_t t = 2048 / (nf > 0 ? nf : 1);
  return (int32_t)(t < 32 ? 32 : t > 256 ? 256 : t);
}
inline int engine_chunk(int ndim, int64_t nx, int64_t ny, int64_t nz, int32_t tiles_target) {
  const int64_t cols = ndim == 3 ? ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY) : (nx + RX - 1) / RX;
  const int64_t depth = ndim == 3 ? nz : ny;
  int64_t c = depth * cols / (tiles_target > 0 ? tiles_target : default_tiles_target(1));
  if (c < 2) c = 2;
  if (c > kMaxChunk) c = kMaxChunk;
  return (int)c;
}

}  // namespace pmsz
