// tiles.hpp -- the steepest-direction stencil over one LDS tile (internal).
//
// Directions (Sec. IV-A, n_min / n_max): for every vertex, the highest and the
// lowest vertex of {i} plus its Freudenthal neighbours, ties broken by index.
// The 15 (3D) or 7 (2D) candidates are visited in ascending vertex index,
// which is the order -7..-1, self, +1..+7 of the signed direction codes
// (index delta = bx + by*nx + bz*nx*ny is a mixed-radix number), so the
// tie-break costs nothing: ">=" keeps the last (largest-index) maximum and
// "<" keeps the first (smallest-index) minimum.  Neighbours outside the box
// are NaN in the tile, which fails both comparisons.
//
// Tiles: a 3D tile is 64 x 4 columns marched along z through a ring of three
// haloed planes (66 x 6) in LDS; a 2D tile is a 256-wide strip marched along
// y through a ring of three haloed rows (258).  Row loads are 64-wide and
// coalesced.  A block of 256 threads processes one tile at a time.
#pragma once

#include "common.hpp"

namespace pmsz {

constexpr int TX = 64, TY = 4;            // 3D tile columns (x, y)
constexpr int PX = TX + 2, PY = TY + 2;   // haloed plane 66 x 6
constexpr int PLANE = PX * PY;
constexpr int RX = 256, RW = RX + 2;      // 2D strip width, haloed row

// Codes of the candidates in ascending vertex index.
__device__ constexpr int kOrder3[15] = {15, 14, 13, 12, 11, 10, 9, 0, 1, 2, 3, 4, 5, 6, 7};
__device__ constexpr int kOrder2[7] = {11, 10, 9, 0, 1, 2, 3};

template <class T, int NC>
__device__ __forceinline__ void extremes(const T (&v)[NC], const int (&order)[NC], int& ca,
                                         int& cd) {
  T hi = -__builtin_inf(), lo = __builtin_inf();
  ca = 0;
  cd = 0;
#pragma unroll
  for (int p = 0; p < NC; ++p) {
    const T x = v[p];
    if (x >= hi) { hi = x; ca = order[p]; }
    if (x < lo) { lo = x; cd = order[p]; }
  }
}

// Shape of one field as the tile code sees it.
struct TileGeo {
  int32_t nx, ny, nz, sxy, n;  // vertex ids fit in int32 (n < 2^31)
  int32_t ndim;
  int32_t chunk;       // planes (3D) or rows (2D) per tile
  int32_t tiles_x, tiles_y, tiles_z;
};

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
  KIND_FIRST = 1,       // first round: directions of f (written), validation of g
                        // against f, mismatch detection of g
  KIND_FIRST_GIVEN = 2, // first round with the caller's directions of f
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

// Flag words of one tile in LDS: the targets of a tile's vertices lie in its
// one-vertex halo, i.e. in (chunk + 2) x (TY + 2) rows of 66 vertices (3D) or
// (chunk + 2) rows of 258 vertices (2D); a row of the flag bitmap then spans at
// most 4 (3D) or 10 (2D) 32-bit words, counted from the word holding the
// row's first halo vertex.
constexpr int kMaxChunk = 16;
// Planes in flight per tile march: four binary32 sets fit the register
// budget of four waves per SIMD; binary64 values take twice the registers.
template <class T>
constexpr int sets_for() { return sizeof(T) == 4 ? 4 : 2; }
constexpr int kFlagW3 = 4, kFlagW2 = 10;
constexpr int kFlagWords = (kMaxChunk + 2) * (TY + 2) * kFlagW3 > (kMaxChunk + 2) * kFlagW2
                               ? (kMaxChunk + 2) * (TY + 2) * kFlagW3
                               : (kMaxChunk + 2) * kFlagW2;

template <class T>
struct TileLds {
  union {
    T p3[2][3][PLANE];  // [field g or h, field f][ring slot][haloed plane]
    T r2[2][3][RW];
  } ring;
  uint32_t flags[kFlagWords];
};

// Flag the targets of one vertex's mismatches (Sec. IV-A):
//   ascending mismatch  -> the vertex that is now n_max (the spurious
//                          maximum; the vertex itself for a false maximum);
//   descending mismatch -> the original n_min, to be lowered below the rival.
// Targets go to the tile's LDS flag words (row r of the halo box, word
// offset from the row's first word); the tile flushes them to the global
// bitmap once at its end, so the march never waits on global atomics.
struct FlagBox {
  int32_t x0, y0, z0;   // tile origin
  int32_t nrow_y;       // rows per plane in the LDS flag layout (TY + 2 in 3D, 1 in 2D)
  int32_t words;        // words per row (kFlagW3 / kFlagW2)
  int32_t span;         // halo vertices per row minus one (TX + 1 or RX + 1)
};

__device__ __forceinline__ void flag_lds(uint32_t* flags, const FlagBox& fb, const TileGeo& G,
                                         int32_t tx, int32_t ty, int32_t tz) {
  const int32_t row = (tz - (fb.z0 - 1)) * fb.nrow_y + (fb.nrow_y > 1 ? ty - (fb.y0 - 1) : 0);
  const int32_t rbase = (G.ndim == 3 ? G.nx * ty + G.sxy * tz : G.nx * ty);
  const int32_t first = (rbase + fb.x0 - 1) >> 5;  // arithmetic shift: floor
  const int32_t gb = rbase + tx;
  atomicOr(flags + row * fb.words + ((gb >> 5) - first), 1u << (gb & 31));
}

__device__ __forceinline__ unsigned flag_targets3(int32_t X, int32_t Y, int32_t Z, int ca, int cd,
                                                  int fa, int fd, const FlagBox& fb,
                                                  const TileGeo& G, uint32_t* flags) {
  unsigned cnt = 0;
  if (ca != fa) {
    const int m = ca & 7, sg = (ca & 8) ? -1 : 1;
    flag_lds(flags, fb, G, X + sg * (m & 1), Y + sg * ((m >> 1) & 1), Z + sg * ((m >> 2) & 1));
    ++cnt;
  }
  if (cd != fd) {
    const int m = fd & 7, sg = (fd & 8) ? -1 : 1;
    flag_lds(flags, fb, G, X + sg * (m & 1), Y + sg * ((m >> 1) & 1), Z + sg * ((m >> 2) & 1));
    ++cnt;
  }
  return cnt;
}

// Flush the tile's LDS flag words into the field's bitmap and clear them.
// Must follow a barrier after the last flag_lds of the tile.
__device__ __forceinline__ void flush_flags(uint32_t* flags, const FlagBox& fb, const TileGeo& G,
                                            int32_t rows, gptr<uint32_t> bm) {
  const int32_t nw = rows * fb.words;
  for (int k = threadIdx.x; k < nw; k += 256) {
    const uint32_t v = flags[k];
    if (!v) continue;
    flags[k] = 0u;
    const int32_t row = k / fb.words, wo = k - row * fb.words;
    int32_t ty, tz;
    if (fb.nrow_y > 1) {
      tz = fb.z0 - 1 + row / fb.nrow_y;
      ty = fb.y0 - 1 + row % fb.nrow_y;
    } else {
      tz = 0;
      ty = fb.y0 - 1 + row;
    }
    const int32_t rbase = (G.ndim == 3 ? G.nx * ty + G.sxy * tz : G.nx * ty);
    const int32_t first = (rbase + fb.x0 - 1) >> 5;
    __hip_atomic_fetch_or(bm + first + wo, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Validation of one vertex (problem statement of Sec. III-B): finite values
// and lb <= g <= ub.  Returns 0 (valid), 1 (non-finite) or 2 (out of bound).
template <class T>
__device__ __forceinline__ int bound_class(T a, T b, T xi) {
  if (!__builtin_isfinite(a) || !__builtin_isfinite(b)) return 1;
  return (b < lower_bound<T>(a, xi) || b > upper_bound<T>(a, xi)) ? 2 : 0;
}

// One 3D tile.  h: field whose directions are evaluated (g, or f for
// KIND_DIRS).  f: original field (its stencil in the first round, its value
// for validation).  dirs: direction bytes of f, read (NEXT, FIRST_GIVEN) or
// written (FIRST, DIRS).  bm: the field's flag bitmap.  Returns the packed
// counts in thread 0.
//
// Software pipeline: the march is unrolled over kSets register sets.  While
// plane z is evaluated from the LDS ring, the next kSets planes (and the
// direction bytes of the next planes) are in flight in the other sets.
// Loads are unconditional (out-of-box lanes read a clamped in-box address
// and substitute NaN), and the barriers order LDS only, so the waits before
// each commit cover just the set being committed.
template <class T, int KIND>
__device__ TileCounts tile3(TileLds<T>& sm, unsigned long long* red, const T* h_in,
                            const T* f_in, uint8_t* dirs_in, uint32_t* bm_in, T xi,
                            const TileGeo G, int64_t tile) {
  const gptr<const T> h = as_global(h_in);
  const gptr<const T> f = as_global(f_in);
  const gptr<uint8_t> dirs = as_global(dirs_in);
  const gptr<uint32_t> bm = as_global(bm_in);
  constexpr int PER = (PLANE + 255) / 256;
  constexpr bool kTwo = (KIND == KIND_FIRST);          // f stencil needed
  constexpr bool kReadDirs = (KIND == KIND_NEXT || KIND == KIND_FIRST_GIVEN);
  constexpr bool kGivenF = (KIND == KIND_FIRST_GIVEN);
  constexpr bool kFlags = (KIND != KIND_DIRS);
  constexpr int kSets = sets_for<T>();
  const int tid = threadIdx.x, tx = tid & (TX - 1), ty = tid / TX;
  const int32_t t32 = (int32_t)tile;
  const int32_t bx = t32 % G.tiles_x, by = (t32 / G.tiles_x) % G.tiles_y,
                bz = t32 / (G.tiles_x * G.tiles_y);
  const int32_t x0 = bx * TX, y0 = by * TY, z0 = bz * G.chunk;
  const int32_t z1 = (z0 + G.chunk < G.nz) ? z0 + G.chunk : G.nz;

  int32_t off[PER];
  uint32_t xymask[PER];  // NaN bits for halo positions outside the box
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * 256;
    const int r = e / PX, c = e - r * PX;
    const int32_t X = x0 + c - 1, Y = y0 + r - 1;
    const bool in = e < PLANE && X >= 0 && X < G.nx && Y >= 0 && Y < G.ny;
    xymask[k] = in ? 0u : nan_mask<T>();
    off[k] = in ? X + G.nx * Y : 0;
  }
  struct Set {
    T h[PER], f[PER];  // raw loaded values; masked to NaN at commit
    uint32_t zmask;    // NaN bits when the plane lies outside the box
    int d;
    T fv;
  };
  const int32_t X = x0 + tx, Y = y0 + ty;
  const bool mine = X < G.nx && Y < G.ny;
  const int32_t col = mine ? X + G.nx * Y : 0;
  // plane z of the haloed values into a set (NaN outside the box)
  auto fetch = [&](int32_t z, Set& S) {
    const bool zin = z >= 0 && z < G.nz;
    const int32_t zb = zin ? G.sxy * z : 0;
    S.zmask = zin ? 0u : nan_mask<T>();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      S.h[k] = h[off[k] + zb];
      if (kTwo) S.f[k] = f[off[k] + zb];
    }
  };
  // this thread's direction byte (and f value) of plane z (z < nz)
  auto fetch_own = [&](int32_t z, Set& S) {
    const int32_t i = col + G.sxy * (z < G.nz ? z : 0);
    if (kReadDirs) S.d = dirs[i];
    if (kGivenF) S.fv = f[i];
  };
  auto commit = [&](int slot, const Set& S) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * 256;
      if (e < PLANE) {
        sm.ring.p3[0][slot][e] = or_high(S.h[k], xymask[k] | S.zmask);
        if (kTwo) sm.ring.p3[1][slot][e] = or_high(S.f[k], xymask[k] | S.zmask);
      }
    }
  };

  const int c = (ty + 1) * PX + (tx + 1);
  FlagBox fbx{x0, y0, z0, TY + 2, kFlagW3, TX + 1};
  unsigned mism = 0, nf = 0, nb = 0;
  auto compute = [&](int32_t z, int s, int d_cur, T f_cur) {
    if (!mine) return;
    const int32_t i = col + G.sxy * z;
    const T* L = sm.ring.p3[0][s % 3];
    const T* C = sm.ring.p3[0][(s + 1) % 3];
    const T* P = sm.ring.p3[0][(s + 2) % 3];
    const T v[15] = {L[c - PX - 1], L[c - PX], L[c - 1], L[c],     C[c - PX - 1],
                     C[c - PX],     C[c - 1],  C[c],     C[c + 1], C[c + PX],
                     C[c + PX + 1], P[c],      P[c + 1], P[c + PX], P[c + PX + 1]};
    int ca, cd;
    extremes<T, 15>(v, kOrder3, ca, cd);
    if (KIND == KIND_DIRS) {
      dirs[i] = (uint8_t)(ca | (cd << 4));
      return;
    }
    int fa, fd;
    if (KIND == KIND_FIRST) {
      const T* Lf = sm.ring.p3[1][s % 3];
      const T* Cf = sm.ring.p3[1][(s + 1) % 3];
      const T* Pf = sm.ring.p3[1][(s + 2) % 3];
      const T w[15] = {Lf[c - PX - 1], Lf[c - PX], Lf[c - 1], Lf[c],      Cf[c - PX - 1],
                       Cf[c - PX],     Cf[c - 1],  Cf[c],     Cf[c + 1],  Cf[c + PX],
                       Cf[c + PX + 1], Pf[c],      Pf[c + 1], Pf[c + PX], Pf[c + PX + 1]};
      extremes<T, 15>(w, kOrder3, fa, fd);
      dirs[i] = (uint8_t)(fa | (fd << 4));
      const int bc = bound_class<T>(Cf[c], C[c], xi);
      nf += bc == 1;
      nb += bc == 2;
    } else {
      fa = d_cur & 15;
      fd = d_cur >> 4;
      if (kGivenF) {
        const int bc = bound_class<T>(f_cur, C[c], xi);
        nf += bc == 1;
        nb += bc == 2;
      }
    }
    if (kFlags) mism += flag_targets3(X, Y, z, ca, cd, fa, fd, fbx, G, sm.flags);
  };
  // one step of the march using set S (holding plane z+1 and the own data of plane z)
  // Every global load of a step is unconditional (planes past the tile
  // read clamped addresses), so the number of loads in flight is the same
  // on every path and each commit waits only for its own set.
  auto step = [&](int32_t z, Set& S, bool valid) {
    const int s = z - z0;
    commit((s + 2) % 3, S);
    const int d_cur = S.d;
    const T f_cur = S.fv;
    fetch(z + 1 + kSets, S);
    lds_barrier();
    if (valid) compute(z, s, d_cur, f_cur);
    // issued after the compute so the old own values are dead (no register
    // copy of an in-flight load at the loop latch)
    fetch_own(z + kSets, S);
    lds_barrier();
  };

  Set Q[kSets];
#pragma unroll
  for (int k = 0; k < kSets; ++k) {
    Q[k].d = 0;
    Q[k].fv = T(0);
  }
  fetch(z0 - 1, Q[0]);
  commit(0, Q[0]);
  fetch(z0, Q[0]);
  commit(1, Q[0]);
#pragma unroll
  for (int k = 0; k < kSets; ++k) {
    fetch(z0 + 1 + k, Q[k]);
    fetch_own(z0 + k, Q[k]);
  }
  for (int32_t z = z0; z < z1; z += kSets) {
#pragma unroll
    for (int k = 0; k < kSets; ++k) step(z + k, Q[k], z + k < z1);
  }
  if (KIND == KIND_DIRS) return 0;
  flush_flags(sm.flags, fbx, G, (z1 - z0 + 2) * (TY + 2), bm);
  return block_sum(pack3(mism, nf, nb), red);
}

// One 2D tile (256-wide strip, `chunk` rows), pipelined like tile3.
template <class T, int KIND>
__device__ TileCounts tile2(TileLds<T>& sm, unsigned long long* red, const T* h_in,
                            const T* f_in, uint8_t* dirs_in, uint32_t* bm_in, T xi,
                            const TileGeo G, int64_t tile) {
  const gptr<const T> h = as_global(h_in);
  const gptr<const T> f = as_global(f_in);
  const gptr<uint8_t> dirs = as_global(dirs_in);
  const gptr<uint32_t> bm = as_global(bm_in);
  constexpr int PER = (RW + 255) / 256;
  constexpr bool kTwo = (KIND == KIND_FIRST);
  constexpr bool kReadDirs = (KIND == KIND_NEXT || KIND == KIND_FIRST_GIVEN);
  constexpr bool kGivenF = (KIND == KIND_FIRST_GIVEN);
  constexpr bool kFlags = (KIND != KIND_DIRS);
  constexpr int kSets = sets_for<T>();
  const int tid = threadIdx.x;
  const int32_t t32 = (int32_t)tile;
  const int32_t bx = t32 % G.tiles_x, by = t32 / G.tiles_x;
  const int32_t x0 = bx * RX, y0 = by * G.chunk;
  const int32_t y1 = (y0 + G.chunk < G.ny) ? y0 + G.chunk : G.ny;

  int32_t xs[PER];
  uint32_t xmask[PER];  // NaN bits for halo positions outside the box
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * 256;
    const int32_t xx = x0 + e - 1;
    const bool in = e < RW && xx >= 0 && xx < G.nx;
    xmask[k] = in ? 0u : nan_mask<T>();
    xs[k] = in ? xx : 0;
  }
  struct Set {
    T h[PER], f[PER];  // raw loaded values; masked to NaN at commit
    uint32_t zmask;    // NaN bits when the row lies outside the box
    int d;
    T fv;
  };
  const int32_t X = x0 + tid;
  const bool mine = X < G.nx;
  const int32_t xo = mine ? X : 0;
  auto fetch = [&](int32_t y, Set& S) {
    const bool yin = y >= 0 && y < G.ny;
    const int32_t yb = yin ? G.nx * y : 0;
    S.zmask = yin ? 0u : nan_mask<T>();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      S.h[k] = h[xs[k] + yb];
      if (kTwo) S.f[k] = f[xs[k] + yb];
    }
  };
  auto fetch_own = [&](int32_t y, Set& S) {
    const int32_t i = xo + G.nx * (y < G.ny ? y : 0);
    if (kReadDirs) S.d = dirs[i];
    if (kGivenF) S.fv = f[i];
  };
  auto commit = [&](int slot, const Set& S) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * 256;
      if (e < RW) {
        sm.ring.r2[0][slot][e] = or_high(S.h[k], xmask[k] | S.zmask);
        if (kTwo) sm.ring.r2[1][slot][e] = or_high(S.f[k], xmask[k] | S.zmask);
      }
    }
  };

  const int c = tid + 1;
  // 2D flag rows are indexed by y: the box's "z" origin is the first row
  FlagBox fbx{x0, y0, y0, 1, kFlagW2, RX + 1};
  unsigned mism = 0, nf = 0, nb = 0;
  auto compute = [&](int32_t y, int s, int d_cur, T f_cur) {
    if (!mine) return;
    const int32_t i = X + G.nx * y;
    const T* L = sm.ring.r2[0][s % 3];
    const T* C = sm.ring.r2[0][(s + 1) % 3];
    const T* P = sm.ring.r2[0][(s + 2) % 3];
    const T v[7] = {L[c - 1], L[c], C[c - 1], C[c], C[c + 1], P[c], P[c + 1]};
    int ca, cd;
    extremes<T, 7>(v, kOrder2, ca, cd);
    if (KIND == KIND_DIRS) {
      dirs[i] = (uint8_t)(ca | (cd << 4));
      return;
    }
    int fa, fd;
    if (KIND == KIND_FIRST) {
      const T* Lf = sm.ring.r2[1][s % 3];
      const T* Cf = sm.ring.r2[1][(s + 1) % 3];
      const T* Pf = sm.ring.r2[1][(s + 2) % 3];
      const T w[7] = {Lf[c - 1], Lf[c], Cf[c - 1], Cf[c], Cf[c + 1], Pf[c], Pf[c + 1]};
      extremes<T, 7>(w, kOrder2, fa, fd);
      dirs[i] = (uint8_t)(fa | (fd << 4));
      const int bc = bound_class<T>(Cf[c], C[c], xi);
      nf += bc == 1;
      nb += bc == 2;
    } else {
      fa = d_cur & 15;
      fd = d_cur >> 4;
      if (kGivenF) {
        const int bc = bound_class<T>(f_cur, C[c], xi);
        nf += bc == 1;
        nb += bc == 2;
      }
    }
    if (kFlags) {
      // 2D codes only use the x and y bits; rows are indexed by y
      if (ca != fa) {
        const int m = ca & 7, sg = (ca & 8) ? -1 : 1;
        const int32_t yy = y + sg * ((m >> 1) & 1);
        flag_lds(sm.flags, fbx, G, X + sg * (m & 1), yy, yy);
        ++mism;
      }
      if (cd != fd) {
        const int m = fd & 7, sg = (fd & 8) ? -1 : 1;
        const int32_t yy = y + sg * ((m >> 1) & 1);
        flag_lds(sm.flags, fbx, G, X + sg * (m & 1), yy, yy);
        ++mism;
      }
    }
  };
  // Every global load of a step is unconditional (planes past the tile
  // read clamped addresses), so the number of loads in flight is the same
  // on every path and each commit waits only for its own set.
  auto step = [&](int32_t y, Set& S, bool valid) {
    const int s = y - y0;
    commit((s + 2) % 3, S);
    const int d_cur = S.d;
    const T f_cur = S.fv;
    fetch(y + 1 + kSets, S);
    lds_barrier();
    if (valid) compute(y, s, d_cur, f_cur);
    // issued after the compute so the old own values are dead (no register
    // copy of an in-flight load at the loop latch)
    fetch_own(y + kSets, S);
    lds_barrier();
  };

  Set Q[kSets];
#pragma unroll
  for (int k = 0; k < kSets; ++k) {
    Q[k].d = 0;
    Q[k].fv = T(0);
  }
  fetch(y0 - 1, Q[0]);
  commit(0, Q[0]);
  fetch(y0, Q[0]);
  commit(1, Q[0]);
#pragma unroll
  for (int k = 0; k < kSets; ++k) {
    fetch(y0 + 1 + k, Q[k]);
    fetch_own(y0 + k, Q[k]);
  }
  for (int32_t y = y0; y < y1; y += kSets) {
#pragma unroll
    for (int k = 0; k < kSets; ++k) step(y + k, Q[k], y + k < y1);
  }
  if (KIND == KIND_DIRS) return 0;
  flush_flags(sm.flags, fbx, G, y1 - y0 + 2, bm);
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
