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

template <class T>
union TileLds {
  T p3[2][3][PLANE];  // [field g or h, field f][ring slot][haloed plane]
  T r2[2][3][RW];
};

// Flag the targets of one vertex's mismatches (Sec. IV-A):
//   ascending mismatch  -> the vertex that is now n_max (the spurious
//                          maximum; the vertex itself for a false maximum);
//   descending mismatch -> the original n_min, to be lowered below the rival.
// The atomicOr returns nothing, so the march never waits on it.
__device__ __forceinline__ unsigned flag_targets(int32_t i, int ca, int cd, int fa, int fd,
                                                 int32_t nx, int32_t sxy, uint32_t* bm) {
  unsigned cnt = 0;
  if (ca != fa) {
    const int32_t t = i + code_delta32(ca, nx, sxy);
    atomicOr(bm + (t >> 5), 1u << (t & 31));
    ++cnt;
  }
  if (cd != fd) {
    const int32_t t = i + code_delta32(fd, nx, sxy);
    atomicOr(bm + (t >> 5), 1u << (t & 31));
    ++cnt;
  }
  return cnt;
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
// written (FIRST, DIRS).  Returns the packed counts in thread 0.
//
// Software pipeline: while plane z is evaluated from the LDS ring, plane z+2
// and the direction bytes of plane z+1 are already on their way into
// registers, so the march does not wait on memory at every step.
template <class T, int KIND>
__device__ TileCounts tile3(TileLds<T>& sm, unsigned long long* red, const T* __restrict__ h,
                            const T* __restrict__ f, uint8_t* __restrict__ dirs,
                            uint32_t* __restrict__ bm, T xi, const TileGeo& G, int64_t tile) {
  constexpr int PER = (PLANE + 255) / 256;
  constexpr bool kTwo = (KIND == KIND_FIRST);          // f stencil needed
  constexpr bool kReadDirs = (KIND == KIND_NEXT || KIND == KIND_FIRST_GIVEN);
  const int tid = threadIdx.x, tx = tid & (TX - 1), ty = tid / TX;
  const int32_t t32 = (int32_t)tile;
  const int32_t bx = t32 % G.tiles_x, by = (t32 / G.tiles_x) % G.tiles_y,
                bz = t32 / (G.tiles_x * G.tiles_y);
  const int32_t x0 = bx * TX, y0 = by * TY, z0 = bz * G.chunk;
  const int32_t z1 = (z0 + G.chunk < G.nz) ? z0 + G.chunk : G.nz;

  // plane element e of this thread: (row, col) in the haloed plane
  int32_t off[PER];
  bool inxy[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * 256;
    const int r = e / PX, c = e - r * PX;
    const int32_t X = x0 + c - 1, Y = y0 + r - 1;
    inxy[k] = e < PLANE && X >= 0 && X < G.nx && Y >= 0 && Y < G.ny;
    off[k] = X + G.nx * Y;
  }
  T ph[PER], pf[PER];
  auto fetch = [&](int32_t z) {
    const bool zin = z >= 0 && z < G.nz;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const bool in = zin && inxy[k];
      ph[k] = in ? h[off[k] + G.sxy * z] : FP<T>::nan();
      if (kTwo) pf[k] = in ? f[off[k] + G.sxy * z] : FP<T>::nan();
    }
  };
  auto commit = [&](int slot) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * 256;
      if (e < PLANE) {
        sm.p3[0][slot][e] = ph[k];
        if (kTwo) sm.p3[1][slot][e] = pf[k];
      }
    }
  };

  const int32_t X = x0 + tx, Y = y0 + ty;
  const bool mine = X < G.nx && Y < G.ny;
  const int32_t col = X + G.nx * Y;
  const int c = (ty + 1) * PX + (tx + 1);
  fetch(z0 - 1);
  commit(0);
  fetch(z0);
  commit(1);
  fetch(z0 + 1);
  int d_next = 0;
  T f_next = T(0);
  if (kReadDirs && mine) d_next = dirs[col + G.sxy * z0];
  if (KIND == KIND_FIRST_GIVEN && mine) f_next = f[col + G.sxy * z0];

  unsigned mism = 0, nf = 0, nb = 0;
  for (int32_t z = z0; z < z1; ++z) {
    const int s = z - z0;
    commit((s + 2) % 3);
    if (z + 1 < z1) fetch(z + 2);
    const int d_cur = d_next;
    const T f_cur = f_next;
    if (z + 1 < z1 && mine) {
      if (kReadDirs) d_next = dirs[col + G.sxy * (z + 1)];
      if (KIND == KIND_FIRST_GIVEN) f_next = f[col + G.sxy * (z + 1)];
    }
    __syncthreads();
    if (mine) {
      const int32_t i = col + G.sxy * z;
      const T* L = sm.p3[0][s % 3];
      const T* C = sm.p3[0][(s + 1) % 3];
      const T* P = sm.p3[0][(s + 2) % 3];
      const T v[15] = {L[c - PX - 1], L[c - PX], L[c - 1], L[c],     C[c - PX - 1],
                       C[c - PX],     C[c - 1],  C[c],     C[c + 1], C[c + PX],
                       C[c + PX + 1], P[c],      P[c + 1], P[c + PX], P[c + PX + 1]};
      int ca, cd;
      extremes<T, 15>(v, kOrder3, ca, cd);
      if (KIND == KIND_DIRS) {
        dirs[i] = (uint8_t)(ca | (cd << 4));
      } else {
        int fa, fd;
        if (KIND == KIND_FIRST) {
          const T* Lf = sm.p3[1][s % 3];
          const T* Cf = sm.p3[1][(s + 1) % 3];
          const T* Pf = sm.p3[1][(s + 2) % 3];
          const T w[15] = {Lf[c - PX - 1], Lf[c - PX], Lf[c - 1], Lf[c],      Cf[c - PX - 1],
                           Cf[c - PX],     Cf[c - 1],  Cf[c],     Cf[c + 1],  Cf[c + PX],
                           Cf[c + PX + 1], Pf[c],      Pf[c + 1], Pf[c + PX], Pf[c + PX + 1]};
          extremes<T, 15>(w, kOrder3, fa, fd);
          dirs[i] = (uint8_t)(fa | (fd << 4));
          { const int bc = bound_class<T>(Cf[c], C[c], xi); nf += bc == 1; nb += bc == 2; }
        } else {
          fa = d_cur & 15;
          fd = d_cur >> 4;
          if (KIND == KIND_FIRST_GIVEN) { const int bc = bound_class<T>(f_cur, C[c], xi); nf += bc == 1; nb += bc == 2; }
        }
        mism += flag_targets(i, ca, cd, fa, fd, G.nx, G.sxy, bm);
      }
    }
    __syncthreads();
  }
  if (KIND == KIND_DIRS) return 0;
  return block_sum(pack3(mism, nf, nb), red);
}

// One 2D tile (256-wide strip, `chunk` rows), pipelined like tile3.
template <class T, int KIND>
__device__ TileCounts tile2(TileLds<T>& sm, unsigned long long* red, const T* __restrict__ h,
                            const T* __restrict__ f, uint8_t* __restrict__ dirs,
                            uint32_t* __restrict__ bm, T xi, const TileGeo& G, int64_t tile) {
  constexpr int PER = (RW + 255) / 256;
  constexpr bool kTwo = (KIND == KIND_FIRST);
  constexpr bool kReadDirs = (KIND == KIND_NEXT || KIND == KIND_FIRST_GIVEN);
  const int tid = threadIdx.x;
  const int32_t t32 = (int32_t)tile;
  const int32_t bx = t32 % G.tiles_x, by = t32 / G.tiles_x;
  const int32_t x0 = bx * RX, y0 = by * G.chunk;
  const int32_t y1 = (y0 + G.chunk < G.ny) ? y0 + G.chunk : G.ny;

  int32_t xs[PER];
  bool inx[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * 256;
    xs[k] = x0 + e - 1;
    inx[k] = e < RW && xs[k] >= 0 && xs[k] < G.nx;
  }
  T ph[PER], pf[PER];
  auto fetch = [&](int32_t y) {
    const bool yin = y >= 0 && y < G.ny;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const bool in = yin && inx[k];
      ph[k] = in ? h[xs[k] + G.nx * y] : FP<T>::nan();
      if (kTwo) pf[k] = in ? f[xs[k] + G.nx * y] : FP<T>::nan();
    }
  };
  auto commit = [&](int slot) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * 256;
      if (e < RW) {
        sm.r2[0][slot][e] = ph[k];
        if (kTwo) sm.r2[1][slot][e] = pf[k];
      }
    }
  };

  const int32_t X = x0 + tid;
  const bool mine = X < G.nx;
  const int c = tid + 1;
  fetch(y0 - 1);
  commit(0);
  fetch(y0);
  commit(1);
  fetch(y0 + 1);
  int d_next = 0;
  T f_next = T(0);
  if (kReadDirs && mine) d_next = dirs[X + G.nx * y0];
  if (KIND == KIND_FIRST_GIVEN && mine) f_next = f[X + G.nx * y0];

  unsigned mism = 0, nf = 0, nb = 0;
  for (int32_t y = y0; y < y1; ++y) {
    const int s = y - y0;
    commit((s + 2) % 3);
    if (y + 1 < y1) fetch(y + 2);
    const int d_cur = d_next;
    const T f_cur = f_next;
    if (y + 1 < y1 && mine) {
      if (kReadDirs) d_next = dirs[X + G.nx * (y + 1)];
      if (KIND == KIND_FIRST_GIVEN) f_next = f[X + G.nx * (y + 1)];
    }
    __syncthreads();
    if (mine) {
      const int32_t i = X + G.nx * y;
      const T* L = sm.r2[0][s % 3];
      const T* C = sm.r2[0][(s + 1) % 3];
      const T* P = sm.r2[0][(s + 2) % 3];
      const T v[7] = {L[c - 1], L[c], C[c - 1], C[c], C[c + 1], P[c], P[c + 1]};
      int ca, cd;
      extremes<T, 7>(v, kOrder2, ca, cd);
      if (KIND == KIND_DIRS) {
        dirs[i] = (uint8_t)(ca | (cd << 4));
      } else {
        int fa, fd;
        if (KIND == KIND_FIRST) {
          const T* Lf = sm.r2[1][s % 3];
          const T* Cf = sm.r2[1][(s + 1) % 3];
          const T* Pf = sm.r2[1][(s + 2) % 3];
          const T w[7] = {Lf[c - 1], Lf[c], Cf[c - 1], Cf[c], Cf[c + 1], Pf[c], Pf[c + 1]};
          extremes<T, 7>(w, kOrder2, fa, fd);
          dirs[i] = (uint8_t)(fa | (fd << 4));
          { const int bc = bound_class<T>(Cf[c], C[c], xi); nf += bc == 1; nb += bc == 2; }
        } else {
          fa = d_cur & 15;
          fd = d_cur >> 4;
          if (KIND == KIND_FIRST_GIVEN) { const int bc = bound_class<T>(f_cur, C[c], xi); nf += bc == 1; nb += bc == 2; }
        }
        mism += flag_targets(i, ca, cd, fa, fd, G.nx, G.sxy, bm);
      }
    }
    __syncthreads();
  }
  if (KIND == KIND_DIRS) return 0;
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
