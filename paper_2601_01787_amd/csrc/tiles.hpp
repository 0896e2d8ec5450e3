// tiles.hpp -- the steepest-direction stencil over one LDS tile (internal).
//
// Directions (Sec. IV-A, n_min / n_max): for every vertex, the highest and the
// lowest vertex of {i} plus its Freudenthal neighbours, ties broken by index
// (larger index wins the maximum, smaller the minimum).
//
// Separable evaluation.  The Freudenthal neighbourhood of i is the union of
// two lattice boxes that share i: the upper box i + {0,1}^d and the lower box
// i - {0,1}^d.  Each box is reduced in x, then y, then z pairs; in every pair
// all vertices of the second half have larger indices than all of the first
// (index = x + nx*y + nx*ny*z), so keeping the second half on a tie for the
// maximum and the first half for the minimum is exactly the index
// tie-break.  The two boxes are then merged the same way (every vertex of the
// lower box has an index <= i <= every vertex of the upper box).  A thread
// marching along z (rows along y in 2D) reduces the 2 x 2 squares of each
// plane once and uses them for the vertex below and the vertex above, so a
// vertex costs 9 pair merges per direction instead of 14 comparisons.
//
// Absent neighbours (outside the box) are NaN in the tile.  In the upper box
// the first half of a pair is present whenever the second is, in the lower box
// the second half is present whenever the first is, so one ordered comparison
// per pair both keeps present values over NaN and applies the tie-break.
//
// Tiles: a 3D tile is 64 x 4 columns marched along z; a 2D tile is a
// 256-wide strip marched along y.  Each step stages one haloed plane (66 x 6)
// or row (258) in LDS, double-buffered, with one barrier per step; loads are
// row-contiguous.  A block of 256 threads processes one tile at a time.
#pragma once

#include "common.hpp"

namespace pmsz {

constexpr int TX = 64, TY = 4;            // 3D tile columns (x, y)
constexpr int PX = TX + 2, PY = TY + 2;   // haloed plane 66 x 6
constexpr int PLANE = PX * PY;
constexpr int RX = 256, RW = RX + 2;      // 2D strip width, haloed row

// Extremes of a subset of the candidates: the highest and the lowest value
// and their direction codes (low three bits: +x, +y, +z of the offset mask;
// bit 3: negative offset; 0 = the vertex itself).
template <class T>
struct Ext {
  T hi, lo;
  int ca, cd;
};

template <class T>
__device__ __forceinline__ Ext<T> ext_of(T v, int code) {
  return Ext<T>{v, v, code, code};
}

template <class T>
__device__ __forceinline__ Ext<T> with_bits(Ext<T> e, int bits) {
  e.ca |= bits;
  e.cd |= bits;
  return e;
}

// Merge of disjoint halves A and B, every vertex of B having a larger index
// than every vertex of A; the maximum keeps B on a tie, the minimum keeps A.
// merge_up: valid when B is absent (NaN) whenever A is (upper box pairs);
// merge_dn: valid when A is absent whenever B is (lower box pairs).
template <class T>
__device__ __forceinline__ Ext<T> merge_up(const Ext<T>& A, const Ext<T>& B) {
  const bool bh = B.hi >= A.hi;  // false when B is NaN
  const bool bl = B.lo < A.lo;
  return Ext<T>{bh ? B.hi : A.hi, bl ? B.lo : A.lo, bh ? B.ca : A.ca, bl ? B.cd : A.cd};
}

template <class T>
__device__ __forceinline__ Ext<T> merge_dn(const Ext<T>& A, const Ext<T>& B) {
  const bool bh = !(A.hi > B.hi);  // true when A is NaN
  const bool bl = !(A.lo <= B.lo);
  return Ext<T>{bh ? B.hi : A.hi, bl ? B.lo : A.lo, bh ? B.ca : A.ca, bl ? B.cd : A.cd};
}

// Division of a vertex index n in [0, 2^31) by a divisor d >= 1 fixed per
// field, as a multiply and a shift: with l = ceil(log2 d) and
// m = ceil(2^(31+l) / d) < 2^32, floor(n m / 2^(31+l)) = floor(n / d),
// because n m / 2^(31+l) = n / d + n e / (d 2^(31+l)) with e = m d - 2^(31+l)
// in [0, d), and that excess is below 2^-l <= 1/d (zero when d = 2^l), less
// than the gap from n / d to the next integer.  The host computes m and the
// shift (make_div); the loops of the apply pass and the sparse examination
// then need no integer division per target.
struct FastDiv {
  uint32_t m;
  int32_t sh;  // 31 + l
};
__host__ __device__ inline int32_t fdiv(int32_t n, FastDiv d) {
  return (int32_t)(((uint64_t)(uint32_t)n * d.m) >> d.sh);
}
inline FastDiv make_div(int64_t d) {
  int l = 0;
  while ((int64_t(1) << l) < d) ++l;
  const unsigned __int128 p = (unsigned __int128)1 << (31 + l);
  FastDiv f;
  f.m = (uint32_t)((p + (unsigned __int128)d - 1) / (unsigned __int128)d);
  f.sh = 31 + l;
  return f;
}

// Shape of one field as the tile code sees it.
struct TileGeo {
  int32_t nx, ny, nz, sxy, n;  // vertex ids fit in int32 (n < 2^31)
  int32_t ndim;
  int32_t chunk;       // planes (3D) or rows (2D) per tile
  int32_t tiles_x, tiles_y, tiles_z;
  // Detection box [cx0, cx1) x [cy0, cy1) x [cz0, cz1): only the vertices in
  // it are compared and can flag (their targets may lie outside it).  The
  // whole grid, except for a block of a decomposed domain (Sec. IV-B), whose
  // outer layer is a ghost copy of its neighbours' vertices.
  int32_t cx0, cx1, cy0, cy1, cz0, cz1;
  FastDiv div_nx, div_ny, div_sxy, div_chunk;  // by nx, ny, nx * ny, chunk
};

// The geometry of the tile being marched, in scalar registers (see uniform).
__device__ __forceinline__ TileGeo uniform_geo(const TileGeo& g) {
  TileGeo u;
  u.nx = uniform(g.nx), u.ny = uniform(g.ny), u.nz = uniform(g.nz);
  u.sxy = uniform(g.sxy), u.n = uniform(g.n), u.ndim = uniform(g.ndim);
  u.chunk = uniform(g.chunk);
  u.tiles_x = uniform(g.tiles_x), u.tiles_y = uniform(g.tiles_y), u.tiles_z = uniform(g.tiles_z);
  u.cx0 = uniform(g.cx0), u.cx1 = uniform(g.cx1), u.cy0 = uniform(g.cy0);
  u.cy1 = uniform(g.cy1), u.cz0 = uniform(g.cz0), u.cz1 = uniform(g.cz1);
  u.div_nx = g.div_nx, u.div_ny = g.div_ny, u.div_sxy = g.div_sxy, u.div_chunk = g.div_chunk;
  return u;
}

__host__ __device__ inline int64_t tile_count(const TileGeo& G) {
  return (int64_t)G.tiles_x * G.tiles_y * G.tiles_z;
}

inline TileGeo make_tile_geo(int ndim, int64_t nx, int64_t ny, int64_t nz, int chunk) {
  TileGeo G;
  G.nx = (int32_t)nx;
  G.ny = (int32_t)ny;
  G.nz = (int32_t)nz;
  G.sxy = (int32_t)(nx * ny);
  G.n = (int32_t)(nx * ny * nz);
  G.ndim = ndim;
  G.chunk = chunk;
  G.cx0 = 0;
  G.cx1 = (int32_t)nx;
  G.cy0 = 0;
  G.cy1 = (int32_t)ny;
  G.cz0 = 0;
  G.cz1 = (int32_t)nz;
  G.div_nx = make_div(nx);
  G.div_ny = make_div(ny);
  G.div_sxy = make_div(nx * ny);
  G.div_chunk = make_div(chunk);
  if (ndim == 3) {
    G.tiles_x = (int32_t)((nx + TX - 1) / TX);
    G.tiles_y = (int32_t)((ny + TY - 1) / TY);
    G.tiles_z = (int32_t)((nz + chunk - 1) / chunk);
  } else {
    G.tiles_x = (int32_t)((nx + RX - 1) / RX);
    G.tiles_y = (int32_t)((ny + chunk - 1) / chunk);
    G.tiles_z = 1;
  }
  return G;
}

// What a tile pass does with the directions it computes.
enum TileKind {
  KIND_DIRS = 0,        // write the direction bytes of h
  KIND_FIRST_GIVEN = 2, // first round: validation of g against f, mismatch
                        // detection of g against the given directions of f
  KIND_NEXT = 3         // later rounds: mismatch detection of g
};

// Per-tile counts, packed three to a word (21 bits each) so that one block
// reduction carries them: {mismatches, non-finite, out of bound}.
__device__ __forceinline__ unsigned long long pack3(unsigned a, unsigned b, unsigned c) {
  return (unsigned long long)a | ((unsigned long long)b << 21) | ((unsigned long long)c << 42);
}
__device__ __forceinline__ unsigned unpack3(unsigned long long v, int k) {
  return (unsigned)((v >> (21 * k)) & 0x1FFFFFull);
}
using TileCounts = unsigned long long;  // packed, valid in thread 0

// Flag words of one tile in LDS, in tile-local rows: the targets of a tile's
// vertices lie in its one-vertex halo box, (chunk + 2) x (TY + 2) rows of
// TX + 2 vertices (3D) or chunk + 2 rows of RX + 2 vertices (2D).  Halo
// position lx of row r is bit r * kRowBits + lx, so a target's bit is the
// flagging vertex's own bit plus a constant per direction code (a 16-entry
// table); the flush shifts each row onto the global bitmap's word
// boundaries.
constexpr int kMaxChunk = 32;
// Planes in flight per tile march: four binary32 sets fit the register
// budget of four waves per SIMD; binary64 values take twice the registers.
template <class T, int KIND>
constexpr int sets_for() { return sizeof(T) == 4 ? 4 : 2; }
constexpr int kRowBits3 = 128, kRowBits2 = 320;  // >= TX + 2 and RX + 2
constexpr int kFlagW3 = kRowBits3 / 32, kFlagW2 = kRowBits2 / 32;
constexpr int kFlagWords = (kMaxChunk + 2) * (TY + 2) * kFlagW3 > (kMaxChunk + 2) * kFlagW2
                               ? (kMaxChunk + 2) * (TY + 2) * kFlagW3
                               : (kMaxChunk + 2) * kFlagW2;

template <class T>
struct TileLds {
  union {
    T p3[4][PLANE];  // [slot][haloed plane]: two pairs of planes
    T r2[2][RW];
  } ring;
  uint32_t flags[kFlagWords];
  int32_t fdelta[16];  // flag-bit offset of the neighbour with each direction code
};

// Fill the direction-code table of the flag layout (threads 0..15; read after
// the march's first barrier).  Code bits +x, +y, +z and "negative".
__device__ __forceinline__ void set_flag_deltas(int32_t* t, int32_t row_bits, int32_t plane_bits) {
  const int k = threadIdx.x;
  if (k < 16) {
    const int32_t d = (k & 1) + ((k >> 1) & 1) * row_bits + ((k >> 2) & 1) * plane_bits;
    t[k] = (k & 8) ? -d : d;
  }
}

__device__ __forceinline__ void flag_bit(uint32_t* flags, int32_t bi) {
  atomicOr(flags + (bi >> 5), 1u << (bi & 31));
}

// Targeted edit: a flag also proposes a value for its target, the highest
// value at which the target no longer beats its rival in the (value, index)
// order -- the rival's value when the target's index is the smaller (the tie
// then goes to the rival), else the next value below it; zero is +0.  The
// proposals for a target meet in prop[t] by atomic minimum over an
// order-preserving unsigned key (unset = all ones).
__device__ __forceinline__ uint32_t prop_key(float v) {
  const uint32_t b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ unsigned long long prop_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ float prop_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
__device__ __forceinline__ double prop_value(unsigned long long k) {
  return __longlong_as_double(
      (long long)((k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k));
}
template <class T>
__device__ __forceinline__ void propose(void* prop, int32_t t, int32_t rival, T rv) {
  T v = t < rival ? rv : next_down<T>(rv);
  if (v == T(0)) v = T(0);  // +0
  using K = decltype(prop_key(v));
  __hip_atomic_fetch_min((gptr<K>)prop + t, prop_key(v), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

// Flag the targets of one vertex's mismatches (Sec. IV-A):
//   ascending mismatch  -> the vertex that is now n_max (the spurious
//                          maximum; the vertex itself for a false maximum);
//   descending mismatch -> the original n_min, to be lowered below the rival.
// Targets go to the tile's LDS flag words (row r of the halo box, word
// offset from the row's first word); the tile flushes them to the global
// bitmap once at its end, so the march never waits on global atomics.
// bi: the vertex's own flag bit; v: its index in the field (proposals only).
// With prop set (targeted edit) each flag also proposes a value: the
// ascending rival is n_max under f (value read from g), the descending rival
// is the current n_min, whose value `lo` the stencil already holds.
template <class T>
__device__ __forceinline__ unsigned flag_targets(int32_t bi, int32_t v, int ca, int cd, int fa,
                                                 int fd, const TileGeo& G, uint32_t* flags,
                                                 const int32_t* fdelta, void* prop,
                                                 gptr<const T> g, T lo) {
  unsigned cnt = 0;
  if (ca != fa) {
    flag_bit(flags, bi + fdelta[ca]);
    if (prop) {
      const int32_t c = v + code_delta32(fa, G.nx, G.sxy);
      propose<T>(prop, v + code_delta32(ca, G.nx, G.sxy), c, g[c]);
    }
    ++cnt;
  }
  if (cd != fd) {
    flag_bit(flags, bi + fdelta[fd]);
    if (prop)
      propose<T>(prop, v + code_delta32(fd, G.nx, G.sxy), v + code_delta32(cd, G.nx, G.sxy), lo);
    ++cnt;
  }
  return cnt;
}

// Flush the tile's LDS flag rows into the field's bitmap and clear them; one
// row per thread.  Row r covers global bits row_start(r) .. + W * 32 - 1
// (row_start may be negative or run past the field for halo rows outside
// it, which hold no flags: targets are vertices of the field).  Must follow
// a barrier after the last flag of the tile.
template <int W, class RowStart>
__device__ __forceinline__ void flush_rows(uint32_t* flags, int32_t rows, RowStart row_start,
                                           gptr<uint32_t> bm) {
  for (int r = threadIdx.x; r < rows; r += 256) {
    uint32_t L[W];
    uint32_t any = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      L[j] = flags[r * W + j];
      any |= L[j];
    }
    if (!any) continue;
#pragma unroll
    for (int j = 0; j < W; ++j) flags[r * W + j] = 0u;
    const int32_t gb0 = row_start(r);
    const int32_t w0 = gb0 >> 5;  // arithmetic shift: floor
    const uint32_t sh = (uint32_t)gb0 & 31u;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      uint32_t w = L[j] << sh;
      if (j > 0 && sh) w |= L[j - 1] >> (32u - sh);
      if (w)
        __hip_atomic_fetch_or(bm + (w0 + j), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Validation of one vertex (problem statement of Sec. III-B): finite values
// and lb <= g <= ub.  Returns 0 (valid), 1 (non-finite) or 2 (out of bound).
// With a - xi = s1 + e1 and a + xi = s2 + e2 exactly (TwoSum), a value b lies
// at or above the smallest value >= a - xi iff b > s1, or b == s1 and
// e1 <= 0 (no value lies strictly between s1 and the next one up), and at or
// below the largest value <= a + xi iff b < s2, or b == s2 and e2 >= 0; an
// overflowed sum (infinite s) admits every finite b.
template <class T>
__device__ __forceinline__ int bound_class_exact(T a, T b, T xi) {
  if (!__builtin_isfinite(a) || !__builtin_isfinite(b)) return 1;
  T s1, e1, s2, e2;
  two_sum<T>(a, -xi, s1, e1);
  two_sum<T>(a, xi, s2, e2);
  const bool lo_ok = b > s1 || (b == s1 && e1 <= T(0));
  const bool hi_ok = b < s2 || (b == s2 && e2 >= T(0));
  return (lo_ok && hi_ok) ? 0 : 2;
}

// bound_class with a two-instruction test for the common case.  With
// d = fl(b - a), |d - (b - a)| <= 2^-p |b - a| (p = 24 / 53; a subnormal
// difference is exact), so |d| < xi (1 - 2^-(p-4)) proves |b - a| < xi: b is
// then finite and strictly inside (a - xi, a + xi), hence inside [lb, ub].
// A non-finite a or b makes d NaN or infinite and fails the test; so does a
// value near a bound, and both go to the exact classification.  xi_in: xi
// times (1 - 2^-(p-4)), rounded down (fast_margin).
template <class T>
__device__ __forceinline__ int bound_class(T a, T b, T xi, T xi_in) {
  const T d = b - a;
  if (__builtin_fabs(d) < xi_in) return 0;
  return bound_class_exact<T>(a, b, xi);
}
template <class T>
__device__ __forceinline__ T fast_margin(T xi) {
  const T m = xi * (T(1) - T(sizeof(T) == 4 ? 1.0 / (1 << 20) : 1.0 / (1ll << 49)));
  return m < xi ? m : next_down<T>(xi);  // strictly below xi (xi > 0)
}

// One 3D tile.  h: field whose directions are evaluated (g, or f for
// KIND_DIRS).  f: original field (its values for the first round's
// validation).  dirs: direction bytes of f, read (NEXT, FIRST_GIVEN) or
// written (DIRS).  bm: the field's flag bitmap.  Returns the packed counts in
// thread 0.
//
// The march visits planes p = z0-1 .. z1 (z1 = end of the tile), two per
// step.  For each plane p it reduces the thread's upper square (x..x+1,
// y..y+1) and lower square (x-1..x, y-1..y), completes the upper box of
// vertex p-1 and the lower box of vertex p, and finishes vertex p-1.  Two
// planes per barrier halve the barriers and give each wave two independent
// reduction chains to interleave.
//
// Software pipeline: the march is unrolled over kSets register sets (an
// even number); while a pair of planes is reduced, the next kSets-2 planes
// (and the direction bytes of the matching vertices) are in flight in the
// other sets.  Loads are unconditional (out-of-box lanes read a clamped
// in-box address and substitute NaN at commit), and the barriers order LDS
// only, so the wait before each commit covers just the sets being committed.
// Two pairs of LDS slots with one barrier per step suffice: a step reads
// only its own pair.
template <class T, int KIND, int SETS = sets_for<T, KIND>()>
__device__ TileCounts tile3(TileLds<T>& sm, unsigned long long* red, const T* h_in,
                            const T* f_in, uint8_t* dirs_in, uint32_t* bm_in, T xi,
                            const TileGeo G_in, int64_t tile_in, void* prop_in = nullptr) {
  // every argument is uniform over the block (one tile of one field)
  const TileGeo G = uniform_geo(G_in);
  const int64_t tile = (int64_t)uniform((int32_t)tile_in);
  void* const prop = uniform_ptr(prop_in);
  const gptr<const T> h = as_global(uniform_ptr(h_in));
  const gptr<const T> f = as_global(uniform_ptr(f_in));
  const gptr<uint8_t> dirs = as_global(uniform_ptr(dirs_in));
  const gptr<uint32_t> bm = as_global(uniform_ptr(bm_in));
  const T xi_in = fast_margin<T>(xi);  // validation's fast test (bound_class)
  constexpr int PER = (PLANE + 255) / 256;
  constexpr bool kReadDirs = (KIND == KIND_NEXT || KIND == KIND_FIRST_GIVEN);
  constexpr bool kGivenF = (KIND == KIND_FIRST_GIVEN);
  constexpr int kSets = SETS;
  const int tid = threadIdx.x, tx = tid & (TX - 1), ty = tid / TX;
  const int32_t t32 = (int32_t)tile;
  const int32_t bx = t32 % G.tiles_x, by = (t32 / G.tiles_x) % G.tiles_y,
                bz = t32 / (G.tiles_x * G.tiles_y);
  const int32_t x0 = bx * TX, y0 = by * TY, z0 = bz * G.chunk;
  const int32_t z1 = (z0 + G.chunk < G.nz) ? z0 + G.chunk : G.nz;

  // Addressing: a uniform base per plane, at the tile's halo corner
  // (x0-1, y0-1), plus a 32-bit per-lane byte offset fixed for the tile, so
  // every load is a scalar-base load with no per-step address arithmetic.
  // The corner itself may lie outside the array; lanes outside the box read
  // the tile's first vertex instead.  Offsets stay below 6 * nx * sizeof(T),
  // which the host keeps under 2^32.
  const int64_t corner = (int64_t)(x0 - 1) + (int64_t)G.nx * (y0 - 1);
  const uint32_t safe = (uint32_t)G.nx + 1u;  // (x0, y0) from the corner
  uint32_t offb[PER];
  uint32_t xymask[PER];  // NaN bits for halo positions outside the box
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * 256;
    const int r = e / PX, c = e - r * PX;
    const int32_t X = x0 + c - 1, Y = y0 + r - 1;
    const bool in = e < PLANE && X >= 0 && X < G.nx && Y >= 0 && Y < G.ny;
    xymask[k] = in ? 0u : nan_mask<T>();
    offb[k] = (in ? (uint32_t)r * (uint32_t)G.nx + (uint32_t)c : safe) * (uint32_t)sizeof(T);
  }
  struct Set {
    T h[PER];          // raw loaded values of one plane; masked to NaN at commit
    uint32_t zmask;    // NaN bits when the plane lies outside the box
    int d;             // direction byte of f at this column, one plane lower
    T fv;              // value of f there (given directions)
  };
  const int32_t X = x0 + tx, Y = y0 + ty;
  const bool mine = X < G.nx && Y < G.ny;
  const bool core_col = mine && X >= G.cx0 && X < G.cx1 && Y >= G.cy0 && Y < G.cy1;
  // this column from the corner (the tile's first vertex for idle lanes)
  uint32_t rel = mine ? (uint32_t)(ty + 1) * (uint32_t)G.nx + (uint32_t)(tx + 1) : safe;
  uint32_t relb = rel * (uint32_t)sizeof(T);
  auto fetch = [&](int32_t z, Set& S) {
    const bool zin = z >= 0 && z < G.nz;
    const int64_t zb = zin ? (int64_t)G.sxy * z : 0;
    S.zmask = zin ? 0u : nan_mask<T>();
    const gptr<const char> pb = (gptr<const char>)(h + (zb + corner));
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      opaque_off(offb[k]);
      S.h[k] = *(gptr<const T>)(pb + offb[k]);
    }
  };
  auto fetch_own = [&](int32_t v, Set& S) {
    const int64_t pl = (int64_t)G.sxy * (v >= 0 && v < G.nz ? v : 0) + corner;
    if (kReadDirs) {
      opaque_off(rel);
      S.d = (dirs + pl)[rel];
    }
    if (kGivenF) {
      opaque_off(relb);
      S.fv = *(gptr<const T>)((gptr<const char>)(f + pl) + relb);
    }
  };
  auto commit = [&](int buf, const Set& S) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * 256;
      if (e < PLANE) {
        sm.ring.p3[buf][e] = or_high(S.h[k], xymask[k] | S.zmask);
      }
    }
  };

  const int c = (ty + 1) * PX + (tx + 1);
  // upper and lower 2 x 2 squares of the plane in LDS around this column
  auto squares = [&](const T* P, Ext<T>& up, Ext<T>& dn) {
    const Ext<T> r0 = merge_up(ext_of(P[c], 0), ext_of(P[c + 1], 1));
    const Ext<T> r1 = merge_up(ext_of(P[c + PX], 2), ext_of(P[c + PX + 1], 3));
    up = merge_up(r0, r1);
    const Ext<T> q0 = merge_dn(ext_of(P[c - PX - 1], 11), ext_of(P[c - PX], 10));
    const Ext<T> q1 = merge_dn(ext_of(P[c - 1], 9), ext_of(P[c], 0));
    dn = merge_dn(q0, q1);
  };
  // flag bit of this column's vertex in the halo box's first plane
  constexpr int32_t kPlaneBits3 = kRowBits3 * (TY + 2);
  const int32_t bit0 = (ty + 1) * kRowBits3 + (tx + 1) - (z0 - 1) * kPlaneBits3;
  if (KIND != KIND_DIRS) set_flag_deltas(sm.fdelta, kRowBits3, kPlaneBits3);
  unsigned mism = 0, nf = 0, nb = 0;
  // carried from plane p-1: its squares, the lower box of vertex p-1 and the
  // centre value (for validation)
  Ext<T> gu{}, gl{}, gbox{};
  T gc = T(0);
  // Finish vertex v from the lower box `lob` of v, its upper square `up` in
  // its own plane and `upn` in the plane above.
  auto finish = [&](int32_t v, const Ext<T>& lob, const Ext<T>& up, const Ext<T>& upn, int d,
                    T fv, T centre) {
    const Ext<T> e = merge_up(lob, merge_up(up, with_bits(upn, 4)));
    const int ca = e.ca, cd = e.cd;
    if (KIND == KIND_DIRS) {
      (dirs + ((int64_t)G.sxy * v + corner))[rel] = (uint8_t)(ca | (cd << 4));
    } else {
      const int fa = d & 15, fd = d >> 4;
      if (kGivenF) {
        const int bc = bound_class<T>(fv, centre, xi, xi_in);
        nf += bc == 1;
        nb += bc == 2;
      }
      if (core_col && v >= G.cz0 && v < G.cz1)
        mism += flag_targets<T>(bit0 + v * kPlaneBits3, X + G.nx * Y + G.sxy * v, ca, cd, fa, fd,
                                G, sm.flags, sm.fdelta, prop, h, e.lo);
    }
  };
  // Two planes per barrier: step p stages planes p and p+1 in one pair of LDS
  // slots, reduces both planes' squares (two independent chains), and
  // finishes vertices p-1 and p.  Pairs alternate between the two slot
  // pairs, so one barrier per pair orders all reuse.
  auto step = [&](int32_t p, Set& S0, Set& S1, bool out0, bool out1) {
    const int a = ((p - z0 + 1) >> 1) & 1;
    T* P0 = sm.ring.p3[2 * a];
    T* P1 = sm.ring.p3[2 * a + 1];
    commit(2 * a, S0);
    commit(2 * a + 1, S1);
    const int d0 = S0.d, d1 = S1.d;
    const T f0 = S0.fv, f1 = S1.fv;
    fetch(p + kSets, S0);
    fetch(p + 1 + kSets, S1);
    lds_barrier();
    Ext<T> su0, sd0, su1, sd1;
    squares(P0, su0, sd0);
    squares(P1, su1, sd1);
    const Ext<T> glo0 = merge_dn(with_bits(gl, 12), sd0);   // lower box of vertex p
    const Ext<T> glo1 = merge_dn(with_bits(sd0, 12), sd1);  // lower box of vertex p+1
    const T c0 = P0[c];
    if (out0 && mine) finish(p - 1, gbox, gu, su0, d0, f0, gc);
    if (out1 && mine) finish(p, glo0, su0, su1, d1, f1, c0);
    gu = su1;
    gl = sd1;
    gbox = glo1;
    gc = P1[c];
    // issued after the evaluation so the old own values are dead (no
    // register copy of an in-flight load at the loop latch)
    fetch_own(p + kSets - 1, S0);
    fetch_own(p + kSets, S1);
  };

  Set Q[kSets];
#pragma unroll
  for (int k = 0; k < kSets; ++k) {
    Q[k].d = 0;
    Q[k].fv = T(0);
    fetch(z0 - 1 + k, Q[k]);
    fetch_own(z0 - 2 + k, Q[k]);
  }
  step(z0 - 1, Q[0], Q[1], false, false);
  for (int32_t p = z0 + 1; p <= z1; p += kSets) {
#pragma unroll
    for (int k = 0; k < kSets; k += 2)
      step(p + k, Q[(k + 2) % kSets], Q[(k + 3) % kSets], p + k <= z1, p + k + 1 <= z1);
  }
  lds_barrier();  // the next tile of this block reuses the LDS buffers
  if (KIND == KIND_DIRS) return 0;
  flush_rows<kFlagW3>(sm.flags, (z1 - z0 + 2) * (TY + 2), [&](int32_t r) {
    const int32_t lz = r / (TY + 2), ly = r - lz * (TY + 2);
    return G.nx * (y0 - 1 + ly) + G.sxy * (z0 - 1 + lz) + (x0 - 1);
  }, bm);
  return block_sum(pack3(mism, nf, nb), red);
}

// One 2D tile (256-wide strip, `chunk` rows), marched along y like tile3:
// step r stages row r, reduces the thread's upper pair (x..x+1) and lower
// pair (x-1..x) and finishes vertex r-1.
template <class T, int KIND, int SETS = sets_for<T, KIND>()>
__device__ TileCounts tile2(TileLds<T>& sm, unsigned long long* red, const T* h_in,
                            const T* f_in, uint8_t* dirs_in, uint32_t* bm_in, T xi,
                            const TileGeo G_in, int64_t tile_in, void* prop_in = nullptr) {
  // every argument is uniform over the block (one tile of one field)
  const TileGeo G = uniform_geo(G_in);
  const int64_t tile = (int64_t)uniform((int32_t)tile_in);
  void* const prop = uniform_ptr(prop_in);
  const gptr<const T> h = as_global(uniform_ptr(h_in));
  const gptr<const T> f = as_global(uniform_ptr(f_in));
  const gptr<uint8_t> dirs = as_global(uniform_ptr(dirs_in));
  const gptr<uint32_t> bm = as_global(uniform_ptr(bm_in));
  const T xi_in = fast_margin<T>(xi);  // validation's fast test (bound_class)
  constexpr int PER = (RW + 255) / 256;
  constexpr bool kReadDirs = (KIND == KIND_NEXT || KIND == KIND_FIRST_GIVEN);
  constexpr bool kGivenF = (KIND == KIND_FIRST_GIVEN);
  constexpr int kSets = SETS;
  const int tid = threadIdx.x;
  const int32_t t32 = (int32_t)tile;
  const int32_t bx = t32 % G.tiles_x, by = t32 / G.tiles_x;
  const int32_t x0 = bx * RX, y0 = by * G.chunk;
  const int32_t y1 = (y0 + G.chunk < G.ny) ? y0 + G.chunk : G.ny;

  // uniform base per row at the strip's halo corner x0-1, 32-bit lane offsets
  uint32_t offb[PER];
  uint32_t xmask[PER];  // NaN bits for halo positions outside the box
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * 256;
    const int32_t xx = x0 + e - 1;
    const bool in = e < RW && xx >= 0 && xx < G.nx;
    xmask[k] = in ? 0u : nan_mask<T>();
    offb[k] = (in ? (uint32_t)e : 1u) * (uint32_t)sizeof(T);
  }
  struct Set {
    T h[PER];
    uint32_t zmask;
    int d;
    T fv;
  };
  const int32_t X = x0 + tid;
  const bool mine = X < G.nx;
  const bool core_col = mine && X >= G.cx0 && X < G.cx1;
  uint32_t rel = mine ? (uint32_t)tid + 1u : 1u;  // from the corner x0-1
  uint32_t relb = rel * (uint32_t)sizeof(T);
  const int64_t corner = (int64_t)x0 - 1;
  auto fetch = [&](int32_t y, Set& S) {
    const bool yin = y >= 0 && y < G.ny;
    const int64_t yb = yin ? (int64_t)G.nx * y : 0;
    S.zmask = yin ? 0u : nan_mask<T>();
    const gptr<const char> pb = (gptr<const char>)(h + (yb + corner));
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      opaque_off(offb[k]);
      S.h[k] = *(gptr<const T>)(pb + offb[k]);
    }
  };
  auto fetch_own = [&](int32_t v, Set& S) {
    const int64_t pl = (int64_t)G.nx * (v >= 0 && v < G.ny ? v : 0) + corner;
    if (kReadDirs) {
      opaque_off(rel);
      S.d = (dirs + pl)[rel];
    }
    if (kGivenF) {
      opaque_off(relb);
      S.fv = *(gptr<const T>)((gptr<const char>)(f + pl) + relb);
    }
  };
  auto commit = [&](int buf, const Set& S) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * 256;
      if (e < RW) {
        sm.ring.r2[buf][e] = or_high(S.h[k], xmask[k] | S.zmask);
      }
    }
  };

  const int c = tid + 1;
  auto pairs = [&](const T* R, Ext<T>& up, Ext<T>& dn) {
    up = merge_up(ext_of(R[c], 0), ext_of(R[c + 1], 1));
    dn = merge_dn(ext_of(R[c - 1], 9), ext_of(R[c], 0));
  };
  // flag rows are the strip's rows y0-1 .. y1; this column's bit in the first
  const int32_t bit0 = tid + 1 - (y0 - 1) * kRowBits2;
  if (KIND != KIND_DIRS) set_flag_deltas(sm.fdelta, kRowBits2, 0);
  unsigned mism = 0, nf = 0, nb = 0;
  Ext<T> gu{}, gl{}, gbox{};
  T gc = T(0);
  auto step = [&](int32_t r, Set& S, bool out) {
    const int buf = (r - y0 + 1) & 1;
    commit(buf, S);
    const int d_cur = S.d;
    const T f_cur = S.fv;
    fetch(r + kSets, S);
    lds_barrier();
    Ext<T> su, sd;
    pairs(sm.ring.r2[buf], su, sd);
    const Ext<T> glo = merge_dn(with_bits(gl, 10), sd);  // lower box of vertex r
    if (out && mine) {
      const int32_t v = r - 1;
      const Ext<T> e = merge_up(gbox, merge_up(gu, with_bits(su, 2)));
      const int ca = e.ca, cd = e.cd;
      if (KIND == KIND_DIRS) {
        (dirs + ((int64_t)G.nx * v + corner))[rel] = (uint8_t)(ca | (cd << 4));
      } else {
        const int fa = d_cur & 15, fd = d_cur >> 4;
        if (kGivenF) {
          const int bc = bound_class<T>(f_cur, gc, xi, xi_in);
          nf += bc == 1;
          nb += bc == 2;
        }
        // 2D codes only use the x and y bits; rows are indexed by y
        const int32_t vi = X + G.nx * v;
        const bool core = core_col && v >= G.cy0 && v < G.cy1;
        const int32_t bi = bit0 + v * kRowBits2;
        if (core && ca != fa) {
          flag_bit(sm.flags, bi + sm.fdelta[ca]);
          if (prop) {
            const int32_t c = vi + code_delta32(fa, G.nx, G.sxy);
            propose<T>(prop, vi + code_delta32(ca, G.nx, G.sxy), c, h[c]);
          }
          ++mism;
        }
        if (core && cd != fd) {
          flag_bit(sm.flags, bi + sm.fdelta[fd]);
          if (prop)
            propose<T>(prop, vi + code_delta32(fd, G.nx, G.sxy),
                       vi + code_delta32(cd, G.nx, G.sxy), e.lo);
          ++mism;
        }
      }
    }
    gu = su;
    gl = sd;
    gbox = glo;
    gc = sm.ring.r2[buf][c];
    fetch_own(r + kSets - 1, S);
  };

  Set Q[kSets];
#pragma unroll
  for (int k = 0; k < kSets; ++k) {
    Q[k].d = 0;
    Q[k].fv = T(0);
    fetch(y0 - 1 + k, Q[k]);
    fetch_own(y0 - 2 + k, Q[k]);
  }
  step(y0 - 1, Q[0], false);
  step(y0, Q[1 % kSets], false);
  for (int32_t r = y0 + 1; r <= y1; r += kSets) {
#pragma unroll
    for (int k = 0; k < kSets; ++k) step(r + k, Q[(k + 2) % kSets], r + k <= y1);
  }
  lds_barrier();  // the next tile of this block reuses the LDS buffers
  if (KIND == KIND_DIRS) return 0;
  flush_rows<kFlagW2>(sm.flags, y1 - y0 + 2,
                      [&](int32_t r) { return G.nx * (y0 - 1 + r) + (x0 - 1); }, bm);
  return block_sum(pack3(mism, nf, nb), red);
}

// Voxels of a tile (for the swept-voxel statistics).
__device__ __forceinline__ int32_t tile_voxels(const TileGeo& G, int64_t tile) {
  const int32_t t32 = (int32_t)tile;
  if (G.ndim == 3) {
    const int32_t bx = t32 % G.tiles_x, by = (t32 / G.tiles_x) % G.tiles_y,
                  bz = t32 / (G.tiles_x * G.tiles_y);
    const int32_t w = (bx * TX + TX <= G.nx) ? TX : G.nx - bx * TX;
    const int32_t hgt = (by * TY + TY <= G.ny) ? TY : G.ny - by * TY;
    const int32_t d = (bz * G.chunk + G.chunk <= G.nz) ? G.chunk : G.nz - bz * G.chunk;
    return w * hgt * d;
  }
  const int32_t bx = t32 % G.tiles_x, by = t32 / G.tiles_x;
  const int32_t w = (bx * RX + RX <= G.nx) ? RX : G.nx - bx * RX;
  const int32_t hgt = (by * G.chunk + G.chunk <= G.ny) ? G.chunk : G.ny - by * G.chunk;
  return w * hgt;
}

}  // namespace pmsz
