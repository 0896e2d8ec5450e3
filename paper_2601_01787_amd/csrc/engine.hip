// engine.hip -- the persistent correction kernel (gfx950).
//
// One cooperative launch runs the correction loop of Sec. IV-A for one or many
// fields, whose directions of f were computed beforehand (k_dirs_fields, or
// the caller).  Round E (p = E & 1, q = E % 3), for every field still running:
//   detect  directions of g^k, compared with the directions of f; targets are
//           set in the flag bitmap (Sec. IV-A ascending and descending rules,
//           Sec. III-B FPmax rule).  A field's first round sweeps all its
//           tiles and validates fhat; later rounds sweep only the tiles
//           within one vertex of last round's targets, or, when last round
//           flagged few vertices, examine exactly the Freudenthal neighbours
//           of those targets (sparse rounds).
//   barrier
//   apply   for fields with mismatches: count the flagged vertices (|F|) and
//           those already at their bound; unless the field is out of rounds,
//           give every flagged vertex above its bound one halving edit (Eq. 1),
//           list it for a sparse next round and mark the tiles within one
//           vertex of it active.  Either way only vertices whose mismatch can
//           be non-empty are examined, so the result is that of a full sweep.
//   barrier
// The decision of Sec. IV-A's loop (converged, stalled, out of rounds,
// continue) is a pure function of the state at the start of a round and that
// round's counters; every block evaluates it itself when it needs it, and
// block 0 persists it one round later, so no extra barrier is needed.  The
// loop ends when a round edits nothing (every field done) or after
// max_rounds rounds (resumable steps).
#include <map>
#include <mutex>

#include "engine.hpp"

namespace pmsz {

// ---------------------------------------------------------------------------
// Grid barrier for a cooperative launch.  Each block's thread 0 releases its
// writes (one L2 write-back at agent scope) and arrives on one of kBarGroups
// group counters; the last arrival of a group resets it and arrives on the
// top counter, and the last arrival there resets that and publishes the next
// generation with a release store.  The other blocks poll the generation
// word, which no arrival touches, with relaxed loads (they read the coherent
// copy without touching the caches) and acquire once at the end (one cache
// invalidate), so the next phase sees every block's writes.  Spreading the
// arrivals keeps them from serialising on one address.  The spin is bounded:
// after ~4 s the block records an error and the launch winds down instead of
// hanging.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned relaxed_load(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long relaxed_load(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long relaxed_load(gptr<const unsigned long long> p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void relaxed_add(gptr<unsigned long long> p, unsigned long long v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A load of data that another compute unit may have written since this unit
// last invalidated its cache.  CO (the tail rounds of k_tail, below): a
// device-scope load, which skips the unit's cache and reads the XCD's L2 where
// every unit's stores and atomics land; otherwise a plain load (a grid
// barrier's acquire has invalidated the unit's cache).
template <bool CO, class V>
__device__ __forceinline__ V ld(gptr<const V> p) {
  if constexpr (CO) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}

__device__ __forceinline__ void grid_sync(EngineCtl* ctl, unsigned nblocks, unsigned& gen) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned target = gen + 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned groups = nblocks < (unsigned)kBarGroups ? nblocks : (unsigned)kBarGroups;
    const unsigned grp = blockIdx.x % groups;
    const unsigned members = nblocks / groups + (grp < nblocks % groups ? 1u : 0u);
    bool last = false;
    const unsigned arrived =
        __hip_atomic_fetch_add(&ctl->bar[grp].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == members - 1) {
      __hip_atomic_store(&ctl->bar[grp].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // acq_rel: the reset is ordered before this group's arrival, and the
      // final arrival orders every group's reset before its release below
      const unsigned top = __hip_atomic_fetch_add(&ctl->bar[kBarGroups].v, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
      if (top == groups - 1) {
        __hip_atomic_store(&ctl->bar[kBarGroups].v, 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->bar_gen.v, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = true;
      }
    }
    if (!last) {
      const unsigned long long t0 = wall_clock64();
      while (relaxed_load(&ctl->bar_gen.v) != target) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > 400000000ull) {  // 100 MHz counter: 4 s
          __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    gen = target;
  }
  __syncthreads();
}

// Barrier after the start of a launch.  Release (making this block's writes
// visible to other XCDs) costs an L2 write-back of the whole XCD, so only the
// last block of each XCD to arrive performs it, after every block of that
// XCD has its writes completed in L2 (each wave waits for its stores before
// the block arrives).  Acquire (an invalidate of the compute unit's cache and
// of the XCD's L2) is needed once per compute unit: the blocks resident on
// one unit share its cache, so the first of them past the generation flip
// invalidates and the others wait until it has.  The L1-only invalidate
// does nothing outside thread-group-split mode, and an invalidate per block
// queues 128 of them per XCD (measured: 10.7 us per barrier at 1024 blocks
// against 6.2 us with one per unit).
struct XcdBar {
  unsigned xcc;      // XCD this block runs on
  unsigned members;  // blocks of the launch on it
  unsigned nx;       // XCDs with blocks of the launch
  unsigned cu;       // compute-unit slot: XCD x 256 + HW_ID bits 15:8
  unsigned rank;     // this block's index among the members (k_tail)
};

__device__ __forceinline__ unsigned xcd_of_block() {
  // hardware register XCC_ID, bits 3:0
  return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (unsigned)(kXcdSlots - 1);
}
__device__ __forceinline__ unsigned cu_of_block(unsigned xcc) {
  // hardware register HW_ID, bits 15:8 (CU_ID, SH_ID, SE_ID)
  return xcc * 256u + (__builtin_amdgcn_s_getreg((7 << 11) | (8 << 6) | 4) & 255u);
}

// Bounded spin until *p == target: after ~4 s the block records an error and
// the launch winds down instead of hanging.
__device__ __forceinline__ void spin_until(EngineCtl* ctl, const unsigned* p, unsigned target) {
  const unsigned long long t0 = wall_clock64();
  while (relaxed_load(p) != target) {
    __builtin_amdgcn_s_sleep(1);
    if (wall_clock64() - t0 > 400000000ull) {  // 100 MHz counter: 4 s
      __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
}

__device__ __forceinline__ void xcd_sync(EngineCtl* ctl, const XcdBar& xb, unsigned& gen) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores are complete in L2
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned target = gen + 1;
    bool last = false;
    const unsigned arrived = __hip_atomic_fetch_add(&ctl->xbar[xb.xcc].v, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == xb.members - 1) {
      __hip_atomic_store(&ctl->xbar[xb.xcc].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // every block of this XCD has arrived: write its L2 back once
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned top =
          __hip_atomic_fetch_add(&ctl->xtop.v, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (top == xb.nx - 1) {
        __hip_atomic_store(&ctl->xtop.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->bar_gen.v, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = true;
      }
    }
    if (!last) spin_until(ctl, &ctl->bar_gen.v, target);
    // one invalidate per compute unit; generations only grow within a launch
    // and the slots are cleared before it, so a claim never matches a stale one
    const unsigned old = __hip_atomic_exchange(&ctl->cu_claim[xb.cu], target, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
    if (old != target) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __builtin_amdgcn_s_waitcnt(0);  // the invalidate has completed
      __hip_atomic_store(&ctl->cu_done[xb.cu], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      spin_until(ctl, &ctl->cu_done[xb.cu], target);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    gen = target;
  }
  __syncthreads();
}

// Barrier of a sparse tail round (tail_round): only the blocks of one XCD
// are left, and every load of data that another unit may have written is a
// device-scope one (ld<true>), which skips the unit's cache and reads the
// XCD's L2.  The barrier then needs neither an L2 write-back nor an
// invalidate, only each wave's stores in L2 before its block arrives.  (An
// agent-scope acquire also drops the XCD's L2: every line read after it came
// from HBM at about 2 us, against about 0.12 us for a device-scope load that
// hits the L2, measured between two units of one XCD.)
__device__ __noinline__ void tail_sync(EngineCtl* ctl, const XcdBar& xb, unsigned& gen) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores are complete in L2
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned target = gen + 1;
    const unsigned arrived = __hip_atomic_fetch_add(&ctl->xbar[xb.xcc].v, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == xb.members - 1) {
      __hip_atomic_store(&ctl->xbar[xb.xcc].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);  // the reset lands before any block passes
      __hip_atomic_store(&ctl->bar_gen.v, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      spin_until(ctl, &ctl->bar_gen.v, target);
    }
    gen = target;
  }
  __syncthreads();
}

// Census of the launch's blocks per XCD (the XCD counters start cleared),
// ending with a full barrier.
__device__ __forceinline__ XcdBar xcd_census(EngineCtl* ctl, unsigned& gen) {
  XcdBar xb;
  xb.xcc = xcd_of_block();
  xb.cu = cu_of_block(xb.xcc);
  xb.rank = 0;
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(&ctl->census[xb.xcc], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  grid_sync(ctl, gridDim.x, gen);
  xb.members = __hip_atomic_load(&ctl->census[xb.xcc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  xb.nx = 0;
  for (int i = 0; i < kXcdSlots; ++i)
    xb.nx += __hip_atomic_load(&ctl->census[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u
                                                                                            : 0u;
  return xb;
}

__device__ __forceinline__ bool engine_failed(EngineCtl* ctl) {
  return __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Census of a tail launch (k_tail): block 0 publishes its XCD (the lead,
// where the tail runs), every block reads it and counts itself; the blocks of
// other XCDs then leave, and the lead's blocks wait until every block of the
// launch has counted itself, which fixes their number and their ranks (the
// counters start cleared).  Spins are bounded like the barriers'.  Returns
// false for a block that leaves.
__device__ __forceinline__ bool tail_census(EngineCtl* ctl, XcdBar& xb) {
  __shared__ unsigned s_info[3];  // XCD, rank among the lead XCD's blocks, their number
  if (threadIdx.x == 0) {
    const unsigned xcc = xcd_of_block();
    if (blockIdx.x == 0)
      __hip_atomic_store(&ctl->lead.v, xcc + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long t0 = wall_clock64();
    unsigned lead1;
    while ((lead1 = relaxed_load(&ctl->lead.v)) == 0u) {
      __builtin_amdgcn_s_sleep(1);
      if (wall_clock64() - t0 > 400000000ull) {  // 100 MHz counter: 4 s
        __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    const unsigned lead = lead1 - 1u;
    unsigned rank = ~0u, members = 0u;
    if (lead1 != 0u && xcc == lead)
      rank = __hip_atomic_fetch_add(&ctl->census[lead], 1u, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    // counted after the census word (whose add has returned)
    __hip_atomic_fetch_add(&ctl->arrived.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (rank != ~0u) {
      spin_until(ctl, &ctl->arrived.v, gridDim.x);
      members = relaxed_load(&ctl->census[lead]);
    }
    s_info[0] = xcc;
    s_info[1] = rank;
    s_info[2] = members;
  }
  __syncthreads();
  xb.xcc = s_info[0];
  xb.rank = s_info[1];
  xb.members = s_info[2];
  xb.nx = 1;
  xb.cu = 0;
  return xb.rank != ~0u && !engine_failed(ctl);
}


// Field owning global tile / segment v (fields sorted by base).
__device__ __forceinline__ int field_of_tile(const FieldDesc* fd, int nf, int64_t v) {
  int lo = 0, hi = nf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fd[mid].tile_base <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__device__ __forceinline__ int field_of_seg(const FieldDesc* fd, int nf, int64_t v) {
  int lo = 0, hi = nf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fd[mid].seg_base <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The loop decision of Sec. IV-A: state at the start of the next round from
// the state at the start of this round and this round's counters.
__device__ __forceinline__ FieldIter next_state(FieldIter s, const CtrSum& c,
                                                int64_t max_iters) {
  if (s.done) return s;
  const bool first = !s.started;
  s.started = 1;
  s.swept += c.swept;
  if (first) s.mism0 = c.mism;
  s.flagged_final = c.nflag;
  s.stalled_final = c.at_lb;
  if (first && (c.bad_nf || c.bad_b)) {
    s.done = 1;
    s.status = c.bad_nf ? PMSZ_ERR_NONFINITE : PMSZ_ERR_INPUT_BOUND;
    s.mism0 = s.flagged_final = s.stalled_final = 0;
  } else if (c.mism == 0) {
    s.done = 1;
    s.status = PMSZ_OK;
  } else if (c.at_lb == c.nflag) {
    s.done = 1;
    s.status = PMSZ_ERR_STALLED;
  } else if ((long long)s.k >= max_iters) {
    s.done = 1;
    s.status = PMSZ_ERR_NOT_CONVERGED;
  } else {
    s.k += 1;
    s.steps += c.nflag - c.at_lb;
    s.flagged_final = s.stalled_final = 0;
  }
  return s;
}

// Whole-struct copies through global-space pointers, member by member (the
// implicit copy operations take generic references).
template <bool CO = false>
__device__ __forceinline__ FieldIter load_iter(gptr<const FieldIter> p) {
  FieldIter r;
  r.k = ld<CO>(&p->k);
  r.steps = ld<CO>(&p->steps);
  r.mism0 = ld<CO>(&p->mism0);
  r.flagged_final = ld<CO>(&p->flagged_final);
  r.stalled_final = ld<CO>(&p->stalled_final);
  r.swept = ld<CO>(&p->swept);
  r.status = ld<CO>(&p->status);
  r.done = ld<CO>(&p->done);
  r.started = ld<CO>(&p->started);
  r.pad = ld<CO>(&p->pad);
  return r;
}
__device__ __forceinline__ void store_iter(gptr<FieldIter> p, const FieldIter& s) {
  p->k = s.k;
  p->steps = s.steps;
  p->mism0 = s.mism0;
  p->flagged_final = s.flagged_final;
  p->stalled_final = s.stalled_final;
  p->swept = s.swept;
  p->status = s.status;
  p->done = s.done;
  p->started = s.started;
  p->pad = s.pad;
}
__device__ __forceinline__ void clear_ctr(gptr<FieldCtr> c) {
  for (int k = 0; k < kCtrSlots; ++k) {
    const gptr<CtrSlot> x = &c->s[k];
    x->mism = x->nflag = x->at_lb = x->bad_nf = x->bad_b = x->swept = x->nlist = 0;
  }
}

// Counter slot of this block.
__device__ __forceinline__ int ctr_slot() { return (int)(blockIdx.x % (unsigned)kCtrSlots); }

// Counters of a finished round, summed over the slots.  They are read only
// after the grid barrier that completed them, whose acquire invalidated this
// unit's caches, so plain loads see the final values; plain loads also let
// the unit's cache serve the blocks that share it (every block of the grid
// reads the same few lines after each barrier, and one L2 channel serves
// each line).
template <bool CO = false>
__device__ __forceinline__ CtrSum load_ctr(gptr<const FieldCtr> c) {
  CtrSum r{0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < kCtrSlots; ++k) {
    const gptr<const CtrSlot> x = &c->s[k];
    r.mism += ld<CO>(&x->mism);
    r.nflag += ld<CO>(&x->nflag);
    r.at_lb += ld<CO>(&x->at_lb);
    r.bad_nf += ld<CO>(&x->bad_nf);
    r.bad_b += ld<CO>(&x->bad_b);
    r.swept += ld<CO>(&x->swept);
    r.nlist += ld<CO>(&x->nlist);
  }
  return r;
}
// Mismatches of a finished round (the apply pass's only test in later rounds).
template <bool CO = false>
__device__ __forceinline__ unsigned long long load_mism(gptr<const FieldCtr> c) {
  unsigned long long m = 0;
#pragma unroll
  for (int k = 0; k < kCtrSlots; ++k) m += ld<CO>(&c->s[k].mism);
  return m;
}

// Round totals over all fields, summed over the slots (read after the barrier
// that completed them, like the counters).
template <bool CO = false>
__device__ __forceinline__ RoundTot load_tot(const EngineCtl* ctl, int q) {
  RoundTot r{0, 0, 0, 0, {0, 0, 0, 0}};
  const gptr<const RoundTot> t = as_global(&ctl->tot[q][0]);
#pragma unroll
  for (int k = 0; k < kCtrSlots; ++k) {
    r.edits += ld<CO>(&t[k].edits);
    r.swept += ld<CO>(&t[k].swept);
    r.sparse += ld<CO>(&t[k].sparse);
    r.flagged += ld<CO>(&t[k].flagged);
  }
  return r;
}
template <bool CO = false>
__device__ __forceinline__ unsigned long long load_edits(const EngineCtl* ctl, int q) {
  const gptr<const RoundTot> t = as_global(&ctl->tot[q][0]);
  unsigned long long e = 0;
#pragma unroll
  for (int k = 0; k < kCtrSlots; ++k) e += ld<CO>(&t[k].edits);
  return e;
}

// State of a field at the start of round E.
template <bool CO = false>
__device__ __forceinline__ FieldIter state_at(const FieldDesc& d, unsigned long long E,
                                              unsigned long long E0) {
  const gptr<const FieldState> st = as_global((const FieldState*)d.st);
  if (E == E0) return load_iter<CO>(&st->s[E & 1]);
  return next_state(load_iter<CO>(&st->s[(E - 1) & 1]), load_ctr<CO>(&st->c[(E - 1) % 3]),
                    d.max_iters);
}

// Tiles containing a vertex within one step of target t (Freudenthal
// neighbours lie in the 3x3x3 box around t).
struct TileBox {
  int32_t x0, x1, y0, y1, z0, z1;
};

__device__ __forceinline__ TileBox box_of(const TileGeo& G, int32_t t) {
  TileBox b;
  const int32_t row = fdiv(t, G.div_nx);  // y + ny z
  const int32_t x = t - row * G.nx;
  const int32_t xl = x > 0 ? x - 1 : 0, xh = x + 1 < G.nx ? x + 1 : x;
  if (G.ndim == 3) {
    const int32_t z = fdiv(row, G.div_ny), y = row - z * G.ny;
    const int32_t yl = y > 0 ? y - 1 : 0, yh = y + 1 < G.ny ? y + 1 : y;
    const int32_t zl = z > 0 ? z - 1 : 0, zh = z + 1 < G.nz ? z + 1 : z;
    b = {xl / TX, xh / TX, yl / TY, yh / TY, fdiv(zl, G.div_chunk), fdiv(zh, G.div_chunk)};
  } else {
    const int32_t y = row;
    const int32_t yl = y > 0 ? y - 1 : 0, yh = y + 1 < G.ny ? y + 1 : y;
    b = {xl / RX, xh / RX, fdiv(yl, G.div_chunk), fdiv(yh, G.div_chunk), 0, 0};
  }
  return b;
}

// Plain byte stores into the field's activity bytes of the next round: every
// writer stores the same value.  The box spans at most two tiles per axis
// (tile boundaries lie at least two vertices apart), so its tiles are the
// eight corner combinations, duplicates included; all eight bytes are loaded
// before any store, so the loads overlap instead of forming a chain of
// dependent round trips (a store may alias a later load of the same array).
template <bool CO = false>
__device__ __forceinline__ void mark_box(const FieldDesc& d, const TileBox& b, gptr<uint8_t> nxt) {
  int32_t idx[8];
  uint8_t cur[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int32_t bx = (k & 1) ? b.x1 : b.x0, by = (k & 2) ? b.y1 : b.y0,
                  bz = (k & 4) ? b.z1 : b.z0;
    idx[k] = bx + d.geo.tiles_x * (by + d.geo.tiles_y * bz);
    // (the tail stores without reading: its few edits gain more from one
    // round trip less than from the stores a read saves)
    cur[k] = CO ? uint8_t(0) : ld<CO>(nxt + idx[k]);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (!cur[k]) nxt[idx[k]] = 1;
}

// Exclusive prefix sum over the block; *total receives the sum (all threads).
__device__ __forceinline__ int block_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  int before = 0, all = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) before += sh[w];
    all += sh[w];
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

// ---------------------------------------------------------------------------
// Sparse rounds.  A vertex whose mismatch set is non-empty in round E+1 is a
// Freudenthal neighbour of some vertex flagged in round E: either one of its
// neighbours was edited, or nothing around it changed and it flags the same
// target as before, which lies in its own neighbourhood.  So when round E
// flagged few vertices, examining the neighbours of exactly those (the apply
// pass lists them) gives the same flag set as any sweep that covers them.
// Duplicated examinations only repeat idempotent flag writes; the mismatch
// count is then an over-count, which is only ever tested against zero after
// a field's first round.
// ---------------------------------------------------------------------------

// Examinations needed by round E of a field in a sparse round, or -1 when the
// round sweeps its active tiles (first round, or a slot's slice of the target
// list overflowed).  cnt (nullable) receives the targets listed per slot.
template <bool CO = false>
__device__ __forceinline__ long long sparse_items(const FieldDesc& d, const FieldIter& s,
                                                  unsigned long long E, uint32_t* cnt = nullptr) {
  if (!s.started || s.done) return -1;
  const gptr<const FieldCtr> c = &as_global((const FieldState*)d.st)->c[(E + 2) % 3];
  const unsigned long long cap = (unsigned long long)(d.list_cap / list_slices(d.words));
  unsigned long long n = 0;
  bool over = false;
#pragma unroll
  for (int k = 0; k < kCtrSlots; ++k) {
    const unsigned long long nk = ld<CO>(&c->s[k].nlist);
    over |= nk > cap;
    n += nk;
    if (cnt) cnt[k] = (uint32_t)nk;
  }
  if (over) return -1;
  return (long long)n * (d.geo.ndim == 3 ? 15 : 7);
}

// The same count from list lengths loaded beforehand (nk, by load_nlist,
// whose loads then overlap those of the field's state: the tail).
__device__ __forceinline__ long long sparse_items_of(const FieldDesc& d, const FieldIter& s,
                                                     const unsigned long long* nk,
                                                     uint32_t* cnt) {
  if (!s.started || s.done) return -1;
  const unsigned long long cap = (unsigned long long)(d.list_cap / list_slices(d.words));
  unsigned long long n = 0;
  bool over = false;
#pragma unroll
  for (int k = 0; k < kCtrSlots; ++k) {
    over |= nk[k] > cap;
    n += nk[k];
    cnt[k] = (uint32_t)nk[k];
  }
  if (over) return -1;
  return (long long)n * (d.geo.ndim == 3 ? 15 : 7);
}

// List lengths of round E's sparse examination (the previous round's apply
// pass appended the targets), device-scope loads.
__device__ __forceinline__ void load_nlist(const FieldDesc& d, unsigned long long E,
                                           unsigned long long* nk) {
  const gptr<const FieldCtr> c = &as_global((const FieldState*)d.st)->c[(E + 2) % 3];
#pragma unroll
  for (int k = 0; k < kCtrSlots; ++k) nk[k] = ld<true>(&c->s[k].nlist);
}

// Signed vertex offset of a direction code.
__device__ __forceinline__ int32_t code_offset(const TileGeo& G, int code) {
  const int m = code & 7;
  const int32_t o = (m & 1) + ((m >> 1) & 1) * G.nx + ((m >> 2) & 1) * G.sxy;
  return (code & 8) ? -o : o;
}

// Directions of g at vertex v from gathered values: the same upper / lower
// box pair merges, in the same order, as the tile marches.
template <class T, bool CO = false>
__device__ __forceinline__ void gather_dirs(const TileGeo& G, gptr<const T> g, int32_t v,
                                            int32_t x, int32_t y, int32_t z, int& ca, int& cd) {
  const T nan = T(__builtin_nan(""));
  const bool xm = x > 0, xp = x + 1 < G.nx;
  if (G.ndim == 3) {
    const bool ym = y > 0, yp = y + 1 < G.ny, zm = z > 0, zp = z + 1 < G.nz;
    auto up = [&](int bx, int by, int bz) {
      const bool ok = (!bx || xp) && (!by || yp) && (!bz || zp);
      const T val = ok ? ld<CO>(g + (v + bx + by * G.nx + bz * G.sxy)) : nan;
      return ext_of(val, bx | (by << 1) | (bz << 2));
    };
    auto dn = [&](int bx, int by, int bz) {  // vertex v - (1-bx, 1-by, 1-bz)
      const int mx = 1 - bx, my = 1 - by, mz = 1 - bz, m = mx | (my << 1) | (mz << 2);
      const bool ok = (!mx || xm) && (!my || ym) && (!mz || zm);
      const T val = ok ? ld<CO>(g + (v - mx - my * G.nx - mz * G.sxy)) : nan;
      return ext_of(val, m ? (8 | m) : 0);
    };
    const Ext<T> U = merge_up(merge_up(merge_up(up(0, 0, 0), up(1, 0, 0)),
                                       merge_up(up(0, 1, 0), up(1, 1, 0))),
                              merge_up(merge_up(up(0, 0, 1), up(1, 0, 1)),
                                       merge_up(up(0, 1, 1), up(1, 1, 1))));
    const Ext<T> L = merge_dn(merge_dn(merge_dn(dn(0, 0, 0), dn(1, 0, 0)),
                                       merge_dn(dn(0, 1, 0), dn(1, 1, 0))),
                              merge_dn(merge_dn(dn(0, 0, 1), dn(1, 0, 1)),
                                       merge_dn(dn(0, 1, 1), dn(1, 1, 1))));
    const Ext<T> e = merge_up(L, U);
    ca = e.ca;
    cd = e.cd;
  } else {
    const bool ym = y > 0, yp = y + 1 < G.ny;
    auto up = [&](int bx, int by) {
      const bool ok = (!bx || xp) && (!by || yp);
      return ext_of(ok ? ld<CO>(g + (v + bx + by * G.nx)) : nan, bx | (by << 1));
    };
    auto dn = [&](int bx, int by) {
      const int mx = 1 - bx, my = 1 - by, m = mx | (my << 1);
      const bool ok = (!mx || xm) && (!my || ym);
      return ext_of(ok ? ld<CO>(g + (v - mx - my * G.nx)) : nan, m ? (8 | m) : 0);
    };
    const Ext<T> U = merge_up(merge_up(up(0, 0), up(1, 0)), merge_up(up(0, 1), up(1, 1)));
    const Ext<T> L = merge_dn(merge_dn(dn(0, 0), dn(1, 0)), merge_dn(dn(0, 1), dn(1, 1)));
    const Ext<T> e = merge_up(L, U);
    ca = e.ca;
    cd = e.cd;
  }
}

// Examination m of a sparse round: neighbour m % per of the target m / per
// listed by the previous round's apply pass (cnt: targets per list slice).
// Returns the targets the examined vertex flags (-1: none) and its number of
// mismatches.
struct Exam {
  int32_t ta, td;  // ascending-rule and descending-rule targets
  unsigned n;      // mismatches found (0, 1 or 2)
};

template <class T, bool CO = false>
__device__ __forceinline__ Exam sparse_examine(const FieldDesc& d, uint32_t m,
                                               const uint32_t* cnt) {
  const TileGeo& G = d.geo;
  const bool three = G.ndim == 3;
  const uint32_t k = three ? m / 15u : m / 7u;
  const uint32_t j = m - k * (three ? 15u : 7u);
  // the slice holding the k-th listed target
  uint32_t kk = k, at = 0;
  const uint32_t slice = (uint32_t)(d.list_cap / list_slices(d.words));
#pragma unroll
  for (int i = 0; i < kCtrSlots - 1; ++i) {
    const uint32_t ci = cnt[i];
    const bool past = at == (uint32_t)i * slice && kk >= ci;
    kk -= past ? ci : 0u;
    at += past ? slice : 0u;
  }
  const int32_t t = (int32_t)ld<CO>(as_global((const uint32_t*)d.list) + (at + kk));
  // the vertex itself, then its neighbours: 3D codes 1..7, 9..15; 2D 1..3, 9..11
  const int code = three ? (j < 8 ? (int)j : (int)j + 1) : (j < 4 ? (int)j : (int)j + 5);
  // the neighbour's offset
  const int mm = code & 7;
  const int sg = (code & 8) ? -1 : 1;
  const int32_t row = fdiv(t, G.div_nx);  // y + ny z
  const int32_t x = t - row * G.nx;
  const int32_t z = three ? fdiv(row, G.div_ny) : 0;
  const int32_t y = row - z * G.ny;
  const int32_t X = x + sg * (mm & 1), Y = y + sg * ((mm >> 1) & 1), Z = z + sg * ((mm >> 2) & 1);
  Exam ex{-1, -1, 0u};
  // only vertices of the detection box are examined (it lies inside the grid)
  if (X < G.cx0 || X >= G.cx1 || Y < G.cy0 || Y >= G.cy1 || Z < G.cz0 || Z >= G.cz1) return ex;
  const int32_t v = t + code_offset(G, code);
  int ca, cd;
  gather_dirs<T, CO>(G, as_global((const T*)d.g), v, X, Y, Z, ca, cd);
  const int d8 = as_global(d.dirs)[v];
  const int fa = d8 & 15, fd = d8 >> 4;
  // targets are neighbours of v, inside the box for directions made by the
  // direction pass; the range check only guards the bitmap
  const gptr<const T> g = as_global((const T*)d.g);
  if (ca != fa) {
    const int32_t tt = v + code_offset(G, ca);
    if ((uint32_t)tt < (uint32_t)G.n) {
      ex.ta = tt;
      if (d.prop) {
        const int32_t c = v + code_offset(G, fa);
        propose<T>(d.prop, tt, c, ld<CO>(g + c));
      }
    }
    ++ex.n;
  }
  if (cd != fd) {
    const int32_t tt = v + code_offset(G, fd);
    if ((uint32_t)tt < (uint32_t)G.n) {
      ex.td = tt;
      if (d.prop) {
        const int32_t r = v + code_offset(G, cd);
        propose<T>(d.prop, tt, r, ld<CO>(g + r));
      }
    }
    ++ex.n;
  }
  return ex;
}

// Per-thread running count for one field at a time, added to the field's
// counter when the thread moves to another field; `acc_flush` then adds the
// rest with one atomic per block when all threads agree on the field.
struct FieldAcc {
  int f = -1;
  unsigned long long n = 0;
};
template <class Ptr>
__device__ __forceinline__ void acc_add(FieldAcc& acc, int fi, unsigned long long v, Ptr ptr) {
  if (fi != acc.f) {
    if (acc.n) relaxed_add(ptr(acc.f), acc.n);
    acc.f = fi;
    acc.n = 0;
  }
  acc.n += v;
}
// Whole block.  sf (4 ints) and sn (4 counts) are LDS scratch; the caller
// synchronises the block before reusing them.
template <class Ptr>
__device__ __forceinline__ void acc_flush(FieldAcc& acc, Ptr ptr, int* sf,
                                          unsigned long long* sn) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int f0 = acc.n ? acc.f : -1;
  for (int off = 32; off > 0; off >>= 1) f0 = max(f0, __shfl_xor(f0, off, 64));
  const bool agree = __all(acc.f == f0 || acc.n == 0);
  if (!agree && acc.n) relaxed_add(ptr(acc.f), acc.n);
  const unsigned long long w = wave_sum(agree ? acc.n : 0ull);
  if (lane == 0) {
    sf[wave] = (agree && w) ? f0 : -1;
    sn[wave] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < 4; ++i) {
      if (sf[i] < 0) continue;
      unsigned long long t = sn[i];
      for (int j = i + 1; j < 4; ++j)
        if (sf[j] == sf[i]) {
          t += sn[j];
          sf[j] = -1;
        }
      relaxed_add(ptr(sf[i]), t);
    }
  }
  acc.f = -1;
  acc.n = 0;
}

// Inclusive prefix sums of one value per thread into s_pre; returns the
// total (all threads).  Scans within each wave with shuffles, then adds the
// totals of the waves before it.
__device__ __forceinline__ long long block_prefix(long long v, long long* s_pre) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  long long x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_pre[wave] = x;
  __syncthreads();
  long long before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const long long t = s_pre[w];
    before += w < wave ? t : 0;
    all += t;
  }
  __syncthreads();
  s_pre[tid] = before + x;
  __syncthreads();
  return all;
}
// First entry of s_pre[0..n) exceeding m.
__device__ __forceinline__ int prefix_find(const long long* s_pre, int n, long long m) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (s_pre[mid] > m) hi = mid; else lo = mid + 1;
  }
  return lo;
}

constexpr int kApplyCap = 2048;   // targets per compaction pass
constexpr int kEditUnroll = 2;    // targets per thread with loads in flight together

// Apply pass over bitmap words [w0, w1) of one field: the block reads the
// segment in one sweep (16 words per thread), compacts the set bits into an
// LDS list, and edits the listed targets with all threads at once.
template <class T, bool CO = false>
__device__ __forceinline__ void apply_segment(const FieldDesc& d, int32_t w0, int32_t w1,
                                              bool edit, gptr<uint8_t> nxt, uint32_t* list,
                                              int* scan, long long* lbase_sh, gptr<FieldCtr> cq,
                                              gptr<uint32_t> tlist, unsigned long long& nflag,
                                              unsigned long long& at_lb,
                                              unsigned long long& edits) {
  constexpr int kPer = 16;
  const int tid = threadIdx.x;
  // list slice of this segment (its counter slot for the list length)
  const int nls = list_slices(d.words);
  const int slot = (int)((w0 / kSegWords) % nls);
  const long long slice = d.list_cap / nls;
  // thread t owns words w0 + t + 256 k: each load instruction reads 256
  // consecutive words across the block
  const gptr<uint32_t> bm = as_global(d.bm);
  uint32_t wv[kPer];
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int32_t w = w0 + tid + 256 * k;
    wv[k] = ld<CO>(bm + (w < w1 ? w : w0));
    if (w >= w1) wv[k] = 0u;
    cnt += __popc(wv[k]);
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (wv[k]) bm[w0 + tid + 256 * k] = 0u;
  nflag += (unsigned)cnt;
  int total = 0;
  const int off = block_scan(cnt, scan, &total);
  const gptr<const T> f = as_global((const T*)d.f);
  const gptr<T> g = as_global((T*)d.g);
  const T xi = (T)d.xi_t;
  TileBox last{-1, -1, -1, -1, -1, -1};  // the tile box this thread marked last
  for (int base = 0; base < total; base += kApplyCap) {
    int o = off;
    if (o < base + kApplyCap && o + cnt > base) {
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        uint32_t bits = wv[k];
        while (bits) {
          const int b = __ffs(bits) - 1;
          bits &= bits - 1;
          if (o >= base && o < base + kApplyCap)
            list[o - base] = (uint32_t)((w0 + tid + 256 * k) * 32 + b);
          ++o;
        }
      }
    }
    const int n = total - base < kApplyCap ? total - base : kApplyCap;
    // In the tail, the first targets' gathers (below) go out before the
    // list-slot atomic, so that the two round trips overlap.
    int32_t t0[kEditUnroll];
    T gt0[kEditUnroll], ft0[kEditUnroll];
    if constexpr (CO) {
      lds_barrier();  // the list is complete
      if (tid < n) {
#pragma unroll
        for (int u = 0; u < kEditUnroll; ++u) {
          const int j = tid + 256 * u;
          t0[u] = (int32_t)list[j < n ? j : tid];
        }
#pragma unroll
        for (int u = 0; u < kEditUnroll; ++u) {
          gt0[u] = ld<CO>(g + t0[u]);
          ft0[u] = f[t0[u]];
        }
      }
    }
    // room in this block's slice of the field's target list for this pass
    // (next round's sparse examination); entries past the slice are
    // dropped, and the count then sends the next round to a tile sweep
    if (edit && tid == 0 && n > 0)
      *lbase_sh = (long long)__hip_atomic_fetch_add(&cq->s[slot].nlist, (unsigned long long)n,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    lds_barrier();
    const long long lbase = edit ? *lbase_sh : 0;
    // kEditUnroll targets per thread at a time: their loads are all issued
    // before any of their stores (the targets are distinct vertices), so a
    // thread keeps several gathers in flight instead of one dependent chain
    // per target
    for (int j0 = tid; j0 < n; j0 += 256 * kEditUnroll) {
      int32_t t[kEditUnroll];
      T gt[kEditUnroll], ft[kEditUnroll];
      if (CO && j0 == tid) {
#pragma unroll
        for (int u = 0; u < kEditUnroll; ++u) {
          t[u] = t0[u];
          gt[u] = gt0[u];
          ft[u] = ft0[u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < kEditUnroll; ++u) {
          const int j = j0 + 256 * u;
          t[u] = (int32_t)list[j < n ? j : j0];
        }
#pragma unroll
        for (int u = 0; u < kEditUnroll; ++u) {
          gt[u] = ld<CO>(g + t[u]);
          ft[u] = f[t[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < kEditUnroll; ++u) {
        const int j = j0 + 256 * u;
        if (j >= n) break;
        const T lb = lower_bound<T>(ft[u], xi);
        const bool above = gt[u] > lb;
        if (d.prop) {
          // targeted edit: the smallest proposal, never below the bound; the
          // proposal slot is reset for the next round
          using K = decltype(prop_key(gt[u]));
          const gptr<K> slot = (gptr<K>)d.prop + t[u];
          if (above && edit) {
            const T pv = prop_value(ld<CO>(slot));
            g[t[u]] = pv > lb ? pv : lb;
          }
          *slot = ~K(0);
        } else if (above && edit) {
          g[t[u]] = halving_edit<T>(gt[u], lb);
        }
        edits += (above && edit) ? 1u : 0u;
        at_lb += above ? 0u : 1u;
        if (edit && lbase + j < slice) tlist[(int64_t)slot * slice + lbase + j] = (uint32_t)t[u];
      }
      if (edit) {
#pragma unroll
        for (int u = 0; u < kEditUnroll; ++u) {
          if (j0 + 256 * u >= n) break;
          // a thread's successive targets lie a few rows apart in a dense
          // round and mostly share their tile box, whose marks are then set
          // already (marks of this round's parity are only ever set here)
          const TileBox b = box_of(d.geo, t[u]);
          if (b.x0 != last.x0 || b.x1 != last.x1 || b.y0 != last.y0 || b.y1 != last.y1 ||
              b.z0 != last.z0 || b.z1 != last.z1) {
            mark_box<CO>(d, b, nxt);
            last = b;
          }
        }
      }
    }
    lds_barrier();
  }
}

// Tile part of round E's detect: the block examines the active tiles among
// first, first + G, first + 2G, ... (activity bytes of round parity E & 1,
// read and cleared 256 at a time, one per thread, and the active ones
// listed); SETS planes are in flight per tile march.
// A block's detect counts for one field, added once per field change.
__device__ __forceinline__ void flush_counts(gptr<CtrSlot> c, unsigned long long m,
                                             unsigned long long nf, unsigned long long nb,
                                             unsigned long long sw, unsigned long long* all_sw) {
  if (m) relaxed_add(&c->mism, m);
  if (nf) relaxed_add(&c->bad_nf, nf);
  if (nb) relaxed_add(&c->bad_b, nb);
  if (sw) {
    relaxed_add(&c->swept, sw);
    atomicAdd(all_sw, sw);
  }
}

// Tile detection of round E over the grid's share of the tiles.  ONLY < 0:
// each field by its state (the engine); ONLY = KIND_FIRST_GIVEN: every tile
// of the fields in their first round, unmarked (engine_sweep); ONLY =
// KIND_NEXT: the marked tiles of fields in a tile round (engine_sweep).
template <class T, int SETS, int ONLY = -1, bool PROP = true, int DIM = 0>
__device__ void detect_tiles(const EngineArgs& a, TileLds<T>& sm, unsigned long long* red,
                             uint16_t* s_tiles, int* s_scan, unsigned long long* s_acc,
                             unsigned long long E, unsigned long long E0, int64_t first,
                             unsigned G) {
  const int tid = threadIdx.x;
  const int p = (int)(E & 1);
  const int q = (int)(E % 3);
  EngineCtl* ctl = a.ctl;
  // the current field's counts, kept by thread 0 in LDS (registers are the
  // tile march's)
  unsigned long long &acc_m = s_acc[0], &acc_nf = s_acc[1], &acc_nb = s_acc[2],
                     &acc_sw = s_acc[3];
  if (tid == 0) acc_m = acc_nf = acc_nb = acc_sw = 0;
  int cur = -1, cached = -1, cached_kind = -1;
  for (int64_t base = first; base < a.total_tiles; base += (int64_t)G * 256) {
    const int64_t mine = base + (int64_t)tid * G;
    int take = 0;
    if (mine < a.total_tiles) {
      const FieldDesc& d = a.fd[field_of_tile(a.fd, a.nf, mine)];
      if (DIM != 0 && d.geo.ndim != DIM) {
        // the other dimension's sweep kernel takes this tile (and its mark)
      } else if (ONLY == KIND_FIRST_GIVEN) {
        const FieldIter s = state_at(d, E, E0);
        take = !s.started && !s.done;
      } else {
        const gptr<uint8_t> flag = as_global(d.act) + p * tile_count(d.geo) + (mine - d.tile_base);
        if (*flag) {
          *flag = 0;
          take = 1;
        }
      }
    }
    int n_act = 0;
    const int pos = block_scan(take, s_scan, &n_act);
    if (take) s_tiles[pos] = (uint16_t)tid;
    __syncthreads();
    for (int j = 0; j < n_act; ++j) {
      // uniform over the block: read once and kept in scalar registers
      const int64_t tt = base + (int64_t)__builtin_amdgcn_readfirstlane(s_tiles[j]) * G;
      const int fi = field_of_tile(a.fd, a.nf, tt);
      if (fi != cached) {
        const FieldIter s = state_at(a.fd[fi], E, E0);
        cached = fi;
        cached_kind = (s.done || sparse_items(a.fd[fi], s, E) >= 0) ? -1
                    : s.started ? KIND_NEXT : KIND_FIRST_GIVEN;
      }
      const int kind = cached_kind;
      if (kind < 0 || (ONLY >= 0 && kind != ONLY)) continue;
      const FieldDesc& d = a.fd[fi];
      if (DIM != 0 && d.geo.ndim != DIM) continue;  // the other dimension's kernel
      if (tid == 0 && fi != cur) {
        if (cur >= 0) {
          flush_counts(&as_global(a.fd[cur].st)->c[q].s[ctr_slot()], acc_m, acc_nf, acc_nb,
                       acc_sw, &ctl->tot[q][ctr_slot()].swept);
        }
        acc_m = acc_nf = acc_nb = acc_sw = 0;
        cur = fi;
      }
      const int64_t tile = tt - d.tile_base;
      const T* g = (const T*)d.g;
      const T* f = (const T*)d.f;
      const T xi = (T)d.xi_t;
      void* const prop = PROP ? d.prop : nullptr;  // proposals of the targeted edit
      TileCounts tc;
      if (DIM == 3 || (DIM == 0 && d.geo.ndim == 3)) {
        if (ONLY != KIND_FIRST_GIVEN && kind == KIND_NEXT)
          tc = tile3<T, KIND_NEXT, SETS>(sm, red, g, f, d.dirs, d.bm, xi, d.geo, tile, prop);
        else if (ONLY != KIND_NEXT)
          tc = tile3<T, KIND_FIRST_GIVEN, SETS>(sm, red, g, f, d.dirs, d.bm, xi, d.geo, tile, prop);
      } else if (DIM != 3) {
        if (ONLY != KIND_FIRST_GIVEN && kind == KIND_NEXT)
          tc = tile2<T, KIND_NEXT, SETS>(sm, red, g, f, d.dirs, d.bm, xi, d.geo, tile, prop);
        else if (ONLY != KIND_NEXT)
          tc = tile2<T, KIND_FIRST_GIVEN, SETS>(sm, red, g, f, d.dirs, d.bm, xi, d.geo, tile, prop);
      }
      if (tid == 0) {
        acc_m += unpack3(tc, 0);
        acc_nf += unpack3(tc, 1);
        acc_nb += unpack3(tc, 2);
        acc_sw += (unsigned long long)tile_voxels(d.geo, tile);
      }
    }
    __syncthreads();  // s_tiles is rewritten by the next batch
  }
  if (tid == 0 && cur >= 0) {
    flush_counts(&as_global(a.fd[cur].st)->c[q].s[ctr_slot()], acc_m, acc_nf, acc_nb, acc_sw,
                 &ctl->tot[q][ctr_slot()].swept);
  }
}

// Apply pass of a round (parity p, counter set q) on one unit: segment
// u >> plog of the batch's flag bitmaps, part u & (2^plog - 1) of it.  Every
// thread of the block takes part (block reductions inside).
template <class T, bool CO = false>
__device__ __forceinline__ void apply_unit(const EngineArgs& a, int64_t u, int plog, int p, int q,
                                           uint32_t* s_list, int* s_scan, long long* s_lbase,
                                           unsigned long long* red) {
  const int tid = threadIdx.x;
  EngineCtl* ctl = a.ctl;
  const int64_t sg = u >> plog;
  const int32_t part = (int32_t)(u & ((int64_t(1) << plog) - 1));
  const int fi = field_of_seg(a.fd, a.nf, sg);
  const FieldDesc& d = a.fd[fi];
  // the state at the start of the round (persisted before this pass)
  const FieldIter s = load_iter<CO>(&as_global(d.st)->s[p]);
  const gptr<FieldCtr> cq = &as_global(d.st)->c[q];
  const gptr<uint8_t> nxt = as_global(d.act) + (p ^ 1) * tile_count(d.geo);
  const unsigned long long mism = load_mism<CO>(cq);
  bool bad = false;
  if (!s.started) {
    const CtrSum cs = load_ctr<CO>(cq);
    bad = cs.bad_nf || cs.bad_b;
  }
  if (s.done || bad || mism == 0) return;
  const bool edit = (long long)s.k < d.max_iters;
  const int32_t span = (int32_t)(kSegWords >> plog);
  const int32_t w0 = (int32_t)((sg - d.seg_base) * kSegWords) + part * span;
  const int32_t w1 = (w0 + span < d.words) ? w0 + span : (int32_t)d.words;
  if (w0 >= w1) return;  // a part past the end of the field's last segment
  unsigned long long nflag = 0, at_lb = 0, edits = 0;
  apply_segment<T, CO>(d, w0, w1, edit, nxt, s_list, s_scan, s_lbase, cq, as_global(d.list),
                       nflag, at_lb, edits);
  // a segment holds at most 128K vertices: the three counts pack into
  // 21-bit fields of one word for a single block reduction
  const unsigned long long tot =
      block_sum(pack3((unsigned)nflag, (unsigned)at_lb, (unsigned)edits), red);
  if (tid == 0) {
    const unsigned long long nf_ = unpack3(tot, 0), al_ = unpack3(tot, 1),
                             ed_ = unpack3(tot, 2);
    const int slot = ctr_slot();
    if (nf_) {
      relaxed_add(&cq->s[slot].nflag, nf_);
      atomicAdd(&ctl->tot[q][slot].flagged, nf_);
    }
    if (al_) relaxed_add(&cq->s[slot].at_lb, al_);
    if (ed_) atomicAdd(&ctl->tot[q][slot].edits, ed_);
  }
}

// Block 0 at the start of round E: persist the field states of round E, clear
// the next-but-one counters; a field finished at E (stop_on_done) or the
// host's request ends the launch after this round (every block reads the word
// after the detect barrier).  CO as for ld.
template <bool CO>
__device__ __forceinline__ void persist_round(const EngineArgs& a, unsigned long long E,
                                              unsigned long long E0, int p, int qn) {
  const int tid = threadIdx.x;
  EngineCtl* ctl = a.ctl;
  bool stop = false;
  for (int fi = tid; fi < a.nf; fi += 256) {
    const FieldDesc& d = a.fd[fi];
    const gptr<FieldState> st = as_global(d.st);
    bool done;
    if (E > E0) {
      const FieldIter s = state_at<CO>(d, E, E0);
      store_iter(&st->s[p], s);
      stop |= a.stop_on_done && s.done && !ld<CO>(&st->s[p ^ 1].done);
      done = s.done;
    } else {
      done = ld<CO>(&st->s[p].done);
      // a later launch of a step whose tile detection ran as sweeps: a
      // field done at its start finished in the step's earlier launch
      stop |= a.stop_on_done && a.tiles_swept && done;
    }
    // the host asked for the step to end once a field is done (every
    // field of a step was running when it began)
    if (done && a.stop_host &&
        __hip_atomic_load(a.stop_host, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) ==
            kStopWhenDone)
      stop = true;
    clear_ctr(&st->c[qn]);
  }
  if (tid == 0 && a.stop_host &&
      __hip_atomic_load(a.stop_host, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == kStopNow)
    stop = true;
  if (stop) __hip_atomic_store(&ctl->stop.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (tid < kCtrSlots) {
    ctl->tot[qn][tid].edits = 0;
    ctl->tot[qn][tid].swept = 0;
    ctl->tot[qn][tid].sparse = 0;
    ctl->tot[qn][tid].flagged = 0;
  }
}

// Round 0's apply pass of a batch whose round-0 tile detection ran as a sweep
// kernel, as a plain kernel at the apply pass's own occupancy instead of a
// one-round engine launch: the pass needs no grid barrier of its own, and
// its scattered gathers want more waves in flight than the engine's register
// budget allows.  k_first_round_end then does what the engine's block 0 and
// tracer do at the end of a round, and the engine starts at round 1.
template <class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_apply_first(
    EngineArgs a, int plog) {
  __shared__ uint32_t s_list[kApplyCap];
  __shared__ int s_scan[4];
  __shared__ long long s_lbase;
  __shared__ unsigned long long red[4];
  if (a.trace && blockIdx.x == 0 && threadIdx.x == 0) {
    // round 0 starts here (its detection was the sweep kernel's)
    const unsigned long long now = wall_clock64();
    a.trace[kTraceRounds * kTraceSlots] = now;
    a.trace[0] = now;
    a.trace[1] = now;
  }
  for (int64_t u = blockIdx.x; u < (a.total_segs << plog); u += gridDim.x)
    apply_unit<T>(a, u, plog, 0, 0, s_list, s_scan, &s_lbase, red);
}

__global__ __launch_bounds__(256) void k_first_round_end(EngineArgs a) {
  const int fi = blockIdx.x * 256 + threadIdx.x;
  if (fi < a.nf) {
    // the state at the start of round 1, as state_at(d, 1, 0) computes it
    const FieldDesc& d = a.fd[fi];
    const gptr<FieldState> st = as_global(d.st);
    store_iter(&st->s[1], state_at(d, 1, 0));
  }
  if (fi == 0) {
    a.ctl->epoch = 1;
    a.ctl->rounds = 1;
    if (a.trace) {
      unsigned long long* t = a.trace;
      const RoundTot rt = load_tot(a.ctl, 0);
      t[2] = wall_clock64();
      t[3] = rt.swept;
      t[4] = rt.flagged;
      t[5] = rt.edits;
      t[6] = rt.sparse;
    }
  }
}

// LDS of k_tail that a tail round uses.
struct RoundLds {
  long long* pre;           // [256] prefix sums of the fields' examinations
  uint32_t* slot;           // [256 * kCtrSlots] targets listed per slot, per field
  uint32_t* list;           // [kApplyCap] targets of an apply pass
  int* scan;                // [4]
  long long* lbase;         // [1]
  unsigned long long* red;  // [4]
  uint16_t* units;          // [256] marked segments of a batch
};

// One sparse round of the tail (k_tail), on the blocks of the lead XCD
// (rank, members): detection of the listed targets' neighbours, the apply
// pass over the segments that detection marked, and their barriers
// (tail_sync), with every load of data that another unit may have written a
// device-scope one.  Returns 0 when the round ran and the loop goes on, 1
// when the loop ends after it, and 2, before anything has run, when some
// field sweeps tiles in this round (the engine takes that round).  The tail
// holds at most 256 fields.
template <class T>
__device__ __forceinline__ int tail_round(const EngineArgs& a, const XcdBar& xb, unsigned& gen,
                                       unsigned long long& E, unsigned long long E0,
                                       const RoundLds L) {
  const int tid = threadIdx.x;
  EngineCtl* ctl = a.ctl;
  const int p = (int)(E & 1);
  const int q = (int)(E % 3), qn = (int)((E + 1) % 3);
  const bool tracer = a.trace && blockIdx.x == 0 && tid == 0;
  long long items = 0;
  int sweeps = 0;
  if (tid < a.nf) {
    const FieldDesc& d = a.fd[tid];
    unsigned long long nk[kCtrSlots];
    load_nlist(d, E, nk);
    const FieldIter s = state_at<true>(d, E, E0);
    items = sparse_items_of(d, s, nk, L.slot + tid * kCtrSlots);
    if (items < 0) {
      sweeps = !s.done;
      items = 0;
    }
  }
  if (__syncthreads_or(sweeps)) return 2;
  if (tracer && E < kTraceRounds) a.trace[kTraceSlots * E] = wall_clock64();
  if (blockIdx.x == 0) {
    // (the tail's first round is checked against the round before it, which
    // the engine launch ran: a field it finished ends the step after this
    // round, as the engine would have)
    persist_round<true>(a, E, E == E0 && E0 > 0 ? E0 - 1 : E0, p, qn);
    if (tid < a.nf && items > 0) {
      relaxed_add(&as_global(a.fd[tid].st)->c[q].s[0].swept, (unsigned long long)items);
      atomicAdd(&ctl->tot[q][0].swept, (unsigned long long)items);
      atomicAdd(&ctl->tot[q][0].sparse, (unsigned long long)items);
    }
  }
  // ---- detect: the examinations of all fields form one index space
  const long long total = block_prefix(items, L.pre);
  {
    FieldAcc mism;
    auto mism_ptr = [&](int f) { return &as_global(a.fd[f].st)->c[q].s[ctr_slot()].mism; };
    for (long long m = (long long)xb.rank * 256 + tid; m < total;
         m += (long long)xb.members * 256) {
      const int fx = prefix_find(L.pre, a.nf, m);
      const Exam ex = sparse_examine<T, true>(
          a.fd[fx], (uint32_t)(m - (fx ? L.pre[fx - 1] : 0)), L.slot + fx * kCtrSlots);
      acc_add(mism, fx, ex.n, mism_ptr);
      // the flags, and the marks of their segments for the apply pass below
      const gptr<uint32_t> bm = as_global(a.fd[fx].bm);
      const gptr<uint8_t> mk = as_global(a.fd[fx].marks);
      if (ex.ta >= 0) {
        __hip_atomic_fetch_or(bm + (ex.ta >> 5), 1u << (ex.ta & 31), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
        mk[ex.ta >> 17] = 1;
      }
      if (ex.td >= 0) {
        __hip_atomic_fetch_or(bm + (ex.td >> 5), 1u << (ex.td & 31), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
        mk[ex.td >> 17] = 1;
      }
    }
    acc_flush(mism, mism_ptr, L.scan, L.red);
  }
  tail_sync(ctl, xb, gen);
  if (engine_failed(ctl)) return 1;
  // written by block 0 before the barrier above
  const bool stop_here =
      __hip_atomic_load(&ctl->stop.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
  if (tracer && E < kTraceRounds) a.trace[kTraceSlots * E + 1] = wall_clock64();
  // ---- apply: the block reads the marks of its segments 256 at a time,
  // clears them, and takes the marked ones whole
  for (int64_t base = xb.rank; base < a.total_segs; base += (int64_t)xb.members * 256) {
    const int64_t mine = base + (int64_t)tid * xb.members;
    int take = 0;
    if (mine < a.total_segs) {
      const FieldDesc& d = a.fd[field_of_seg(a.fd, a.nf, mine)];
      const gptr<uint8_t> mk = as_global(d.marks) + (mine - d.seg_base);
      if (ld<true>(mk)) {
        *mk = 0;
        take = 1;
      }
    }
    int n_take = 0;
    const int pos = block_scan(take, L.scan, &n_take);
    if (take) L.units[pos] = (uint16_t)tid;
    __syncthreads();
    for (int j = 0; j < n_take; ++j) {
      const int64_t u = base + (int64_t)__builtin_amdgcn_readfirstlane(L.units[j]) * xb.members;
      apply_unit<T, true>(a, u, 0, p, q, L.list, L.scan, L.lbase, L.red);
    }
    __syncthreads();  // units is rewritten by the next batch
  }
  tail_sync(ctl, xb, gen);
  if (engine_failed(ctl)) return 1;
  if (tracer && E < kTraceRounds) {
    unsigned long long* t = a.trace + kTraceSlots * E;
    const RoundTot rt = load_tot<true>(ctl, q);
    t[2] = wall_clock64();
    t[3] = rt.swept;
    t[4] = rt.flagged;
    t[5] = rt.edits;
    t[6] = rt.sparse;
  }
  const unsigned long long edited = load_edits<true>(ctl, q);
  ++E;
  return (edited == 0 || stop_here) ? 1 : 0;
}

template <class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 3))) void k_engine(EngineArgs a) {
  __shared__ TileLds<T> sm;
  __shared__ unsigned long long red[4];
  __shared__ unsigned long long s_acc[4];
  __shared__ uint16_t s_tiles[256];
  __shared__ long long s_pre[256];
  __shared__ uint32_t s_slot[256 * kCtrSlots];
  __shared__ long long s_lbase;
  __shared__ uint32_t s_list[kApplyCap];
  __shared__ int s_scan[4];
  const unsigned G = gridDim.x;
  const int tid = threadIdx.x;
  for (int k = tid; k < kFlagWords; k += 256) sm.flags[k] = 0u;
  __syncthreads();
  EngineCtl* ctl = a.ctl;
  unsigned gen = relaxed_load(&ctl->bar_gen.v);
  const unsigned long long E0 = ctl->epoch;
  unsigned long long E = E0;
  const bool tracer = a.trace && blockIdx.x == 0 && tid == 0;
  if (tracer && E0 == 0) a.trace[kTraceRounds * kTraceSlots] = wall_clock64();

  // Fields that have not started: every tile is active in their first round.
  if (a.has_fresh && !a.tiles_swept) {
    for (int64_t tt = (int64_t)blockIdx.x * 256 + tid; tt < a.total_tiles; tt += (int64_t)G * 256) {
      const FieldDesc& d = a.fd[field_of_tile(a.fd, a.nf, tt)];
      const FieldIter s = load_iter(&as_global(d.st)->s[E0 & 1]);
      if (!s.started && !s.done)
        as_global(d.act)[(E0 & 1) * tile_count(d.geo) + (tt - d.tile_base)] = 1;
    }
  }
  // blocks per XCD (its closing barrier also orders the marks above)
  const XcdBar xb = xcd_census(ctl, gen);
  // apply parts per segment: a power of two up to 256 (16 words each), so
  // that the grid's blocks share the segments of small fields
  int parts_log2 = 0;
  while (parts_log2 < 8 && a.total_segs << (parts_log2 + 1) <= (int64_t)G) ++parts_log2;
  // the launch ends to hand its remaining rounds to k_tail
  bool handoff = false;

  for (long long r = 0; a.max_rounds < 0 || r < a.max_rounds; ++r) {
    if (engine_failed(ctl)) break;
    const int p = (int)(E & 1);
    const int q = (int)(E % 3), qn = (int)((E + 1) % 3);
    if (tracer && E < kTraceRounds) a.trace[kTraceSlots * E] = wall_clock64();

    if (blockIdx.x == 0) persist_round<false>(a, E, E0, p, qn);

    // ---- detect ------------------------------------------------------------
    // Sparse rounds first: the examinations of up to 256 fields at a time form
    // one index space (prefix sums in LDS) that the grid strides over.  The
    // mismatch counts are only tested against zero in these rounds.
    int any_tiles = 0;
    bool split_here = false;
    for (int f0 = 0; f0 < a.nf; f0 += 256) {
      const int fi = f0 + tid;
      long long items = 0;
      int sweeps = 0, big = 0;
      if (fi < a.nf) {
        const FieldDesc& d = a.fd[fi];
        const FieldIter s = state_at(d, E, E0);
        items = sparse_items(d, s, E, s_slot + tid * kCtrSlots);
        if (items < 0) {
          sweeps = !s.done;
          big = sweeps && s.started && d.geo.n >= kSplitVoxels;
          items = 0;
        }
      }
      any_tiles |= __syncthreads_or(sweeps);
      // A large tile round is left to a sweep kernel at the march's own
      // occupancy: every block sees the same states and leaves here, before
      // this round's detection has done anything (the marks of its active
      // tiles stay set for the sweep).
      if (a.split_tiles && r > 0 && f0 == 0 && __syncthreads_or(big)) {
        split_here = true;
        break;
      }
      if (fi < a.nf && items > 0 && blockIdx.x == 0) {
        const FieldDesc& d = a.fd[fi];
        relaxed_add(&as_global(d.st)->c[q].s[0].swept, (unsigned long long)items);
        atomicAdd(&ctl->tot[q][0].swept, (unsigned long long)items);
        atomicAdd(&ctl->tot[q][0].sparse, (unsigned long long)items);
      }
      const long long total = block_prefix(items, s_pre);
      const int nfc = a.nf - f0 < 256 ? a.nf - f0 : 256;
      FieldAcc mism;
      auto mism_ptr = [&](int f) { return &as_global(a.fd[f].st)->c[q].s[ctr_slot()].mism; };
      for (long long m = (long long)blockIdx.x * 256 + tid; m < total; m += (long long)G * 256) {
        const int lo = prefix_find(s_pre, nfc, m);
        const int fx = f0 + lo;
        const Exam ex = sparse_examine<T>(a.fd[fx], (uint32_t)(m - (lo ? s_pre[lo - 1] : 0)),
                                          s_slot + lo * kCtrSlots);
        acc_add(mism, fx, ex.n, mism_ptr);
        // fire-and-forget flags: the apply pass reads them after the barrier
        const gptr<uint32_t> bm = as_global(a.fd[fx].bm);
        if (ex.ta >= 0)
          __hip_atomic_fetch_or(bm + (ex.ta >> 5), 1u << (ex.ta & 31), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
        if (ex.td >= 0)
          __hip_atomic_fetch_or(bm + (ex.td >> 5), 1u << (ex.td & 31), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
      }
      acc_flush(mism, mism_ptr, s_scan, red);
      __syncthreads();  // s_pre is rewritten by the next group
    }
    if (split_here) break;
    // Tiles: skipped when every running field is in a sparse round (marks
    // left from earlier rounds then only widen a later tile round).
    if (any_tiles && !(r == 0 && a.tiles_swept))
      detect_tiles<T, sets_for<T, KIND_NEXT>()>(a, sm, red, s_tiles, s_scan, s_acc, E, E0,
                                                blockIdx.x, G);
    xcd_sync(ctl, xb, gen);
    if (engine_failed(ctl)) break;
    // written by block 0 before the barrier above
    const bool stop_here =
        __hip_atomic_load(&ctl->stop.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    if (tracer && E < kTraceRounds) a.trace[kTraceSlots * E + 1] = wall_clock64();

    // ---- apply -------------------------------------------------------------
    // One pass per 4096-word segment of each field's flag bitmap, or per part
    // of one when the grid has more blocks than there are segments (small
    // fields: a segment's edits would otherwise run through one block's
    // threads in a few long chains).
    // (Rounds after an all-sparse detect flag few vertices: whole segments.)
    const int plog = any_tiles ? parts_log2 : 0;
    for (int64_t u = blockIdx.x; u < (a.total_segs << plog); u += G)
      apply_unit<T>(a, u, plog, p, q, s_list, s_scan, &s_lbase, red);
    xcd_sync(ctl, xb, gen);
    if (engine_failed(ctl)) break;
    if (tracer && E < kTraceRounds) {
      unsigned long long* t = a.trace + kTraceSlots * E;
      const RoundTot rt = load_tot(ctl, q);
      t[2] = wall_clock64();
      t[3] = rt.swept;
      t[4] = rt.flagged;
      t[5] = rt.edits;
      t[6] = rt.sparse;
    }
    const unsigned long long edited = load_edits(ctl, q);
    ++E;
    if (edited == 0 || stop_here) break;
    // the next round examines at most 15 neighbours per edit: few enough for
    // the blocks of one XCD, and few enough segments to mark for its apply
    // pass, and k_tail takes the rest of the loop there
    if (a.tail_ok && a.nf <= 256 &&
        edited * 15ull <= (unsigned long long)(kTailGrid / 8) * 256ull * kTailExams &&
        (edited <= (unsigned long long)kTailSegs || a.total_segs <= kTailSegs)) {
      handoff = true;
      break;
    }
  }
  // persist the state at the start of the next round, and gather it
  if (blockIdx.x == 0 && !engine_failed(ctl)) {
    for (int fi = tid; fi < a.nf; fi += 256) {
      const FieldDesc& d = a.fd[fi];
      const FieldIter s = state_at(d, E, E0);
      if (E > E0) store_iter(&as_global(d.st)->s[E & 1], s);
      if (a.out) a.out[fi] = s;
    }
    if (tid == 0) {
      ctl->epoch = E;
      ctl->rounds = E - E0;
      ctl->handoff = handoff ? kHandToTail : 0;
    }
    // k_tail's census starts cleared (the XCD arrival counters are cleared
    // already: each barrier's last arrival resets its XCD's)
    if (handoff) {
      if (tid < kXcdSlots) ctl->census[tid] = 0u;
      if (tid == 0) {
        ctl->lead.v = 0u;
        ctl->arrived.v = 0u;
      }
    }
  }
}

// The tail of the correction loop (kHandToTail): the sparse rounds after the
// engine launch that handed them over, on the blocks of one XCD (tail_round),
// until every field is done, a round needs tile sweeps (kHandToEngine: the
// host launches the engine again), or a barrier times out.  Launched after
// every engine launch that may hand over; without a handover it ends at once.
template <class T>
__global__ __launch_bounds__(256) void k_tail(EngineArgs a) {
  __shared__ long long s_pre[256];
  __shared__ uint32_t s_slot[256 * kCtrSlots];
  __shared__ uint32_t s_list[kApplyCap];
  __shared__ int s_scan[4];
  __shared__ long long s_lbase;
  __shared__ unsigned long long red[4];
  __shared__ uint16_t s_units[256];
  EngineCtl* ctl = a.ctl;
  if (ctl->handoff != kHandToTail) return;
  XcdBar xb;
  if (!tail_census(ctl, xb)) return;
  unsigned gen = relaxed_load(&ctl->bar_gen.v);
  const unsigned long long E0 = ctl->epoch;
  unsigned long long E = E0;
  RoundLds L;
  L.pre = s_pre;
  L.slot = s_slot;
  L.list = s_list;
  L.scan = s_scan;
  L.lbase = &s_lbase;
  L.red = red;
  L.units = s_units;
  int rc = 0;
  while (!engine_failed(ctl) && (rc = tail_round<T>(a, xb, gen, E, E0, L)) == 0) {
  }
  // persist the state at the start of the next round, and gather it
  if (blockIdx.x == 0 && !engine_failed(ctl)) {
    const int tid = threadIdx.x;
    for (int fi = tid; fi < a.nf; fi += 256) {
      const FieldDesc& d = a.fd[fi];
      const FieldIter s = state_at<true>(d, E, E0);
      if (E > E0) store_iter(&as_global(d.st)->s[E & 1], s);
      if (a.out) a.out[fi] = s;
    }
    if (tid == 0) {
      ctl->epoch = E;
      ctl->rounds = E - E0;
      ctl->handoff = rc == 2 ? kHandToEngine : kTailDone;
    }
  }
}

// Directions of f for every field of a batch whose caller gave none, before
// the engine runs: a plain (non-cooperative) grid over the tiles of all
// fields, at the stencil's own occupancy.
template <class T>
__global__ __launch_bounds__(256) void k_dirs_fields(const FieldDesc* fd, int nf,
                                                     int64_t total_tiles) {
  __shared__ TileLds<T> sm;
  for (int64_t tt = blockIdx.x; tt < total_tiles; tt += gridDim.x) {
    const FieldDesc& d = fd[field_of_tile(fd, nf, tt)];
    if (d.dirs_given) continue;
    const T* f = (const T*)d.f;
    if (d.geo.ndim == 3)
      tile3<T, KIND_DIRS>(sm, nullptr, f, f, d.dirs, nullptr, T(0), d.geo, tt - d.tile_base);
    else
      tile2<T, KIND_DIRS>(sm, nullptr, f, f, d.dirs, nullptr, T(0), d.geo, tt - d.tile_base);
  }
}

// The sweep kernels' occupancy and prefetch depth (measured on the 512^3
// binary32 workload: seven waves per SIMD with two plane sets in flight beat
// five or six waves and four sets, spills included; binary64 keeps the
// engine's three waves).
constexpr int kSweepSets = 2;
constexpr int kSweepWaves32 = 7, kSweepWaves64 = 3;

// Tile detection of the round the workspace's epoch names, as a plain kernel
// (see engine_sweep in engine.hpp); it adds to the same counters, flag
// bitmaps and totals as the engine's own tile detection.
template <class T, int KIND, bool PROP, int DIM, int SETS>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? kSweepWaves32 : kSweepWaves64)))
void k_sweep(EngineArgs a) {
  __shared__ TileLds<T> sm;
  __shared__ unsigned long long red[4];
  __shared__ uint16_t s_tiles[256];
  __shared__ int s_scan[4];
  __shared__ unsigned long long s_acc[4];
  for (int k = threadIdx.x; k < kFlagWords; k += 256) sm.flags[k] = 0u;
  __syncthreads();
  const unsigned long long E = a.ctl->epoch;  // written by the previous launch
  detect_tiles<T, SETS, KIND, PROP, DIM>(a, sm, red, s_tiles, s_scan, s_acc, E, E, blockIdx.x,
                                         gridDim.x);
}

hipError_t engine_dirs(int dtype, const FieldDesc* fd, int nf, int64_t total_tiles,
                       hipStream_t s) {
  int64_t grid = total_tiles < 65536 ? total_tiles : 65536;
  if (grid < 1) grid = 1;
  if (dtype == PMSZ_F32)
    hipLaunchKernelGGL(k_dirs_fields<float>, dim3((unsigned)grid), dim3(256), 0, s, fd, nf,
                       total_tiles);
  else
    hipLaunchKernelGGL(k_dirs_fields<double>, dim3((unsigned)grid), dim3(256), 0, s, fd, nf,
                       total_tiles);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill(uint32_t* p, int64_t words, uint32_t v) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x; w < words; w += stride) p[w] = v;
}

hipError_t engine_fill(void* p, size_t bytes, uint32_t v, hipStream_t s) {
  const int64_t words = (int64_t)(bytes / 4);
  int64_t b = (words + 255) / 256;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)b), dim3(256), 0, s, (uint32_t*)p, words, v);
  return hipGetLastError();
}

hipError_t engine_zero(void* p, size_t bytes, hipStream_t s) { return engine_fill(p, bytes, 0u, s); }

// Cooperative grid: as many resident blocks as the chip holds, but no more
// than there is work for (fewer arrivals make the barrier cheaper).
// Resident blocks per compute unit and compute units of a device, looked up
// once per (device, kernel) under a lock (calls may come from several host
// threads).
struct Occupancy {
  int per_cu = -1, cus = -1;
};
// Resident blocks per compute unit of a 256-thread kernel on a device, and
// the device's compute units (cached per kernel and device).
static hipError_t occupancy_of(const void* kernel, int dev, Occupancy& out) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, Occupancy> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({kernel, dev});
  if (it == cache.end()) {
    Occupancy o;
    hipError_t e = hipDeviceGetAttribute(&o.cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o.per_cu, kernel, 256, 0);
    if (e != hipSuccess) return e;
    it = cache.emplace(std::make_pair(kernel, dev), o).first;
  }
  out = it->second;
  return hipSuccess;
}
template <class T>
static hipError_t occupancy(int dev, Occupancy& out) {
  return occupancy_of((const void*)k_engine<T>, dev, out);
}

// One block per resident slot of the chip (every block resident at once),
// at most one per tile.
template <class T, int KIND, bool PROP, int DIM>
static hipError_t sweep_t(const EngineArgs& a, hipStream_t s) {
  constexpr int SETS = kSweepSets;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  Occupancy occ;
  if ((e = occupancy_of((const void*)k_sweep<T, KIND, PROP, DIM, SETS>, dev, occ)) != hipSuccess)
    return e;
  int64_t grid = (int64_t)(occ.per_cu > 0 ? occ.per_cu : 1) * (occ.cus > 0 ? occ.cus : 1);
  if (grid > a.total_tiles) grid = a.total_tiles;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((k_sweep<T, KIND, PROP, DIM, SETS>), dim3((unsigned)grid), dim3(256), 0, s,
                     a);
  return hipGetLastError();
}

template <class T, int DIM>
static hipError_t sweep_kind(int kind, bool prop, const EngineArgs& a, hipStream_t s) {
  if (kind == KIND_FIRST_GIVEN)
    return prop ? sweep_t<T, KIND_FIRST_GIVEN, true, DIM>(a, s)
                : sweep_t<T, KIND_FIRST_GIVEN, false, DIM>(a, s);
  return prop ? sweep_t<T, KIND_NEXT, true, DIM>(a, s) : sweep_t<T, KIND_NEXT, false, DIM>(a, s);
}

template <class T>
static hipError_t sweep_dims(int kind, bool prop, int dims, const EngineArgs& a, hipStream_t s) {
  hipError_t e = hipSuccess;
  if ((dims & 2) && (e = sweep_kind<T, 2>(kind, prop, a, s)) != hipSuccess) return e;
  if (dims & 4) e = sweep_kind<T, 3>(kind, prop, a, s);
  return e;
}

hipError_t engine_sweep(int dtype, int kind, bool prop, int dims, const EngineArgs& a,
                        hipStream_t s) {
  if (dtype == PMSZ_F32) return sweep_dims<float>(kind, prop, dims, a, s);
  return sweep_dims<double>(kind, prop, dims, a, s);
}

template <class T>
static hipError_t apply_first_t(const EngineArgs& a, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  Occupancy occ;
  if ((e = occupancy_of((const void*)k_apply_first<T>, dev, occ)) != hipSuccess) return e;
  int64_t grid = (int64_t)(occ.per_cu > 0 ? occ.per_cu : 1) * (occ.cus > 0 ? occ.cus : 1);
  // parts per segment as in the engine: a power of two up to 256, so that
  // small fields' segments are shared by the grid's blocks
  int plog = 0;
  while (plog < 8 && (a.total_segs << (plog + 1)) <= grid) ++plog;
  const int64_t units = a.total_segs << plog;
  if (grid > units) grid = units;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_apply_first<T>, dim3((unsigned)grid), dim3(256), 0, s, a, plog);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned fb = (unsigned)((a.nf + 255) / 256);
  hipLaunchKernelGGL(k_first_round_end, dim3(fb > 0 ? fb : 1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t engine_apply_first(int dtype, const EngineArgs& a, hipStream_t s) {
  if (dtype == PMSZ_F32) return apply_first_t<float>(a, s);
  return apply_first_t<double>(a, s);
}

template <class T>
static hipError_t launch_t(const EngineArgs& a, hipStream_t s, int* grid_out, bool clear) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  Occupancy occ;
  if ((e = occupancy<T>(dev, occ)) != hipSuccess) return e;
  const int per_cu = occ.per_cu, cus = occ.cus;
  // the XCD and compute-unit barrier state starts cleared in every launch
  // (the round totals after it are kept: a sweep kernel may have added to
  // the current round's already)
  if (clear &&
      (e = engine_fill(&a.ctl->xbar[0], offsetof(EngineCtl, tot) - offsetof(EngineCtl, xbar), 0u,
                       s)) != hipSuccess)
    return e;
  int64_t want = a.total_tiles > a.total_segs ? a.total_tiles : a.total_segs;
  if (want < 1) want = 1;
  int64_t cap = (int64_t)per_cu * cus;
  if (cap < 1) cap = 1;
  const unsigned grid = (unsigned)(want < cap ? want : cap);
  if (grid_out) *grid_out = (int)grid;
  EngineArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel((const void*)k_engine<T>, dim3(grid), dim3(256), args, 0, s);
}

hipError_t engine_launch(int dtype, const EngineArgs& a, hipStream_t s, int* grid_out,
                         bool clear) {
  if (dtype == PMSZ_F32) return launch_t<float>(a, s, grid_out, clear);
  return launch_t<double>(a, s, grid_out, clear);
}

// kTailGrid blocks, all resident (cooperative); an engine launch that hands
// over leaves the census and barrier words of the tail cleared.
template <class T>
static hipError_t tail_t(const EngineArgs& a, hipStream_t s) {
  EngineArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel((const void*)k_tail<T>, dim3(kTailGrid), dim3(256), args, 0,
                                    s);
}

hipError_t engine_tail(int dtype, const EngineArgs& a, hipStream_t s) {
  if (dtype == PMSZ_F32) return tail_t<float>(a, s);
  return tail_t<double>(a, s);
}

}  // namespace pmsz
