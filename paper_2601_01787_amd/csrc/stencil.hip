// stencil.hip -- steepest-direction stencil, input validation, and the
// detect / apply passes of one correction round (gfx950).
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
// Tiles: a 3D block owns 64 x 4 columns and marches along z through a ring of
// three haloed planes in LDS (coalesced 64-wide row loads); a 2D block owns a
// 256-wide strip and marches along y through three haloed rows.
#include "launch.hpp"

namespace pmsz {

constexpr int TX = 64, TY = 4;               // 3D tile (x, y), 256 threads
constexpr int PX = TX + 2, PY = TY + 2;      // haloed plane 66 x 6
constexpr int PLANE = PX * PY;
constexpr int RX = 256, RW = RX + 2;         // 2D strip, haloed row 258

enum { MODE_DIRS = 0, MODE_DETECT = 1 };

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

// Per-vertex action shared by both kernels: write the direction byte, or
// compare with the original field's byte and flag the targets:
//   ascending mismatch  -> flag the vertex that is now n_max (the spurious
//                          maximum; the vertex itself for a false maximum),
//   descending mismatch -> flag the original n_min, to be lowered below the
//                          rival (Sec. IV-A).
template <int MODE>
__device__ __forceinline__ int act(int64_t i, int ca, int cd, const Geo& G, uint8_t* dirs_out,
                                   const uint8_t* dirs_f, uint32_t* bm) {
  if (MODE == MODE_DIRS) {
    dirs_out[i] = (uint8_t)(ca | (cd << 4));
    return 0;
  } else {
    const int d = dirs_f[i];
    const int fa = d & 15, fd = d >> 4;
    int cnt = 0;
    if (ca != fa) {
      const int64_t t = i + code_delta(ca, G.nx, G.sxy);
      atomicOr(bm + (t >> 5), 1u << (t & 31));
      ++cnt;
    }
    if (cd != fd) {
      const int64_t t = i + code_delta(fd, G.nx, G.sxy);
      atomicOr(bm + (t >> 5), 1u << (t & 31));
      ++cnt;
    }
    return cnt;
  }
}

// Common prologue of a detect launch: stop when the run is over, and turn a
// failed validation into the final status (only block 0 writes it).
__device__ __forceinline__ bool detect_should_stop(Ctl* ctl) {
  __shared__ int stop;
  if (threadIdx.x == 0) {
    const int done = ctl->done;
    const unsigned long long nf = ctl->bad_nonfinite, nb = ctl->bad_bound;
    stop = done || nf || nb;
    if (!done && (nf || nb) && blockIdx.x == 0) {
      ctl->status = nf ? PMSZ_ERR_NONFINITE : PMSZ_ERR_INPUT_BOUND;
      ctl->done = 1;
    }
  }
  __syncthreads();
  return stop != 0;
}

template <class T, int MODE>
__global__ __launch_bounds__(256) void k_stencil3(const T* __restrict__ h, Geo G, int zc,
                                                  int64_t nbx, int64_t nby,
                                                  uint8_t* __restrict__ dirs_out,
                                                  const uint8_t* __restrict__ dirs_f,
                                                  uint32_t* __restrict__ bm, Ctl* ctl) {
  __shared__ T sm[3][PLANE];
  __shared__ unsigned long long red[4];
  if (MODE == MODE_DETECT && detect_should_stop(ctl)) return;
  const int tid = threadIdx.x, tx = tid & (TX - 1), ty = tid / TX;
  const int64_t b = blockIdx.x;
  const int64_t bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
  const int64_t x0 = bx * TX, y0 = by * TY, z0 = bz * zc;
  const int64_t z1 = (z0 + zc < G.nz) ? z0 + zc : G.nz;

  auto load_plane = [&](int slot, int64_t z) {
    for (int e = tid; e < PLANE; e += 256) {
      const int r = e / PX, c = e - r * PX;
      const int64_t X = x0 + c - 1, Y = y0 + r - 1;
      T v = FP<T>::nan();
      if (z >= 0 && z < G.nz && X >= 0 && X < G.nx && Y >= 0 && Y < G.ny)
        v = h[X + G.nx * (Y + G.ny * z)];
      sm[slot][e] = v;
    }
  };

  load_plane(0, z0 - 1);
  load_plane(1, z0);
  int cnt = 0;
  const int64_t X = x0 + tx, Y = y0 + ty;
  const bool mine = X < G.nx && Y < G.ny;
  const int c = (ty + 1) * PX + (tx + 1);
  for (int64_t z = z0; z < z1; ++z) {
    const int s = (int)(z - z0);
    load_plane((s + 2) % 3, z + 1);
    __syncthreads();
    if (mine) {
      const T* L = sm[s % 3];
      const T* C = sm[(s + 1) % 3];
      const T* P = sm[(s + 2) % 3];
      const T v[15] = {L[c - PX - 1], L[c - PX], L[c - 1], L[c],     C[c - PX - 1],
                       C[c - PX],     C[c - 1],  C[c],     C[c + 1], C[c + PX],
                       C[c + PX + 1], P[c],      P[c + 1], P[c + PX], P[c + PX + 1]};
      int ca, cd;
      extremes<T, 15>(v, kOrder3, ca, cd);
      cnt += act<MODE>(X + G.nx * (Y + G.ny * z), ca, cd, G, dirs_out, dirs_f, bm);
    }
    __syncthreads();
  }
  if (MODE == MODE_DETECT) {
    const unsigned long long tot = block_sum((unsigned long long)cnt, red);
    if (tid == 0 && tot) atomicAdd(&ctl->mism, tot);
  }
}

template <class T, int MODE>
__global__ __launch_bounds__(256) void k_stencil2(const T* __restrict__ h, Geo G, int yc,
                                                  int64_t nbx, uint8_t* __restrict__ dirs_out,
                                                  const uint8_t* __restrict__ dirs_f,
                                                  uint32_t* __restrict__ bm, Ctl* ctl) {
  __shared__ T sm[3][RW];
  __shared__ unsigned long long red[4];
  if (MODE == MODE_DETECT && detect_should_stop(ctl)) return;
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t bx = b % nbx, by = b / nbx;
  const int64_t x0 = bx * RX, y0 = by * yc;
  const int64_t y1 = (y0 + yc < G.ny) ? y0 + yc : G.ny;

  auto load_row = [&](int slot, int64_t y) {
    for (int e = tid; e < RW; e += 256) {
      const int64_t X = x0 + e - 1;
      T v = FP<T>::nan();
      if (y >= 0 && y < G.ny && X >= 0 && X < G.nx) v = h[X + G.nx * y];
      sm[slot][e] = v;
    }
  };

  load_row(0, y0 - 1);
  load_row(1, y0);
  int cnt = 0;
  const int64_t X = x0 + tid;
  const bool mine = X < G.nx;
  const int c = tid + 1;
  for (int64_t y = y0; y < y1; ++y) {
    const int s = (int)(y - y0);
    load_row((s + 2) % 3, y + 1);
    __syncthreads();
    if (mine) {
      const T* L = sm[s % 3];
      const T* C = sm[(s + 1) % 3];
      const T* P = sm[(s + 2) % 3];
      const T v[7] = {L[c - 1], L[c], C[c - 1], C[c], C[c + 1], P[c], P[c + 1]};
      int ca, cd;
      extremes<T, 7>(v, kOrder2, ca, cd);
      cnt += act<MODE>(X + G.nx * y, ca, cd, G, dirs_out, dirs_f, bm);
    }
    __syncthreads();
  }
  if (MODE == MODE_DETECT) {
    const unsigned long long tot = block_sum((unsigned long long)cnt, red);
    if (tid == 0 && tot) atomicAdd(&ctl->mism, tot);
  }
}

// Validation of fhat against f (problem statement of Sec. III-B): finite
// values and lb <= fhat <= ub.
template <class T>
__global__ __launch_bounds__(256) void k_validate(const T* __restrict__ f,
                                                  const T* __restrict__ fh, int64_t n, T xi,
                                                  Ctl* ctl) {
  __shared__ unsigned long long red[4];
  unsigned long long nf = 0, nb = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const T a = f[i], b = fh[i];
    if (!__builtin_isfinite(a) || !__builtin_isfinite(b)) {
      ++nf;
    } else if (b < lower_bound<T>(a, xi) || b > upper_bound<T>(a, xi)) {
      ++nb;
    }
  }
  nf = block_sum(nf, red);
  nb = block_sum(nb, red);
  if (threadIdx.x == 0) {
    if (nf) atomicAdd(&ctl->bad_nonfinite, nf);
    if (nb) atomicAdd(&ctl->bad_bound, nb);
  }
}

__global__ __launch_bounds__(256) void k_init(Ctl* ctl, uint32_t* bm, int64_t nwords) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x; w < nwords; w += stride) bm[w] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < (int)(sizeof(Ctl) / 4)) ((uint32_t*)ctl)[threadIdx.x] = 0u;
}

// Apply pass: one edit (Eq. 1, halving) for every flagged vertex, the
// statistics of the round, and -- in the last block to finish -- the decision
// of Sec. IV-A's loop: converged, stalled, out of rounds, or next round.
template <class T>
__global__ __launch_bounds__(256) void k_apply(const T* __restrict__ f, T* __restrict__ g,
                                               uint32_t* __restrict__ bm, int64_t nwords,
                                               T xi, Ctl* ctl, int64_t max_iters) {
  __shared__ unsigned long long red[4];
  __shared__ int st[2];
  if (threadIdx.x == 0) {
    st[0] = ctl->done;
    st[1] = (long long)ctl->k < max_iters;
  }
  __syncthreads();
  if (st[0]) return;
  const bool edit = st[1] != 0;
  unsigned long long nflag = 0, at_lb = 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x; w < nwords; w += stride) {
    uint32_t bits = bm[w];
    if (!bits) continue;
    bm[w] = 0u;
    nflag += __popc(bits);
    while (bits) {
      const int bpos = __ffs(bits) - 1;
      bits &= bits - 1;
      const int64_t t = w * 32 + bpos;
      const T gt = g[t];
      const T lb = lower_bound<T>(f[t], xi);
      if (gt > lb) {
        if (edit) g[t] = halving_edit<T>(gt, lb);
      } else {
        ++at_lb;
      }
    }
  }
  nflag = block_sum(nflag, red);
  at_lb = block_sum(at_lb, red);
  if (threadIdx.x == 0) {
    if (nflag) atomicAdd(&ctl->nflag, nflag);
    if (at_lb) atomicAdd(&ctl->at_lb, at_lb);
    __threadfence();
    const unsigned int ticket = atomicAdd(&ctl->ticket, 1u);
    if (ticket == gridDim.x - 1) {
      __threadfence();
      const unsigned long long mism = load_acquire(&ctl->mism);
      const unsigned long long nf = load_acquire(&ctl->nflag);
      const unsigned long long al = load_acquire(&ctl->at_lb);
      const unsigned long long k = ctl->k;
      if (k == 0) ctl->mism0 = mism;
      ctl->flagged_final = nf;
      ctl->stalled_final = al;
      if (mism == 0) {
        ctl->status = PMSZ_OK;
        ctl->done = 1;
      } else if (al == nf) {
        ctl->status = PMSZ_ERR_STALLED;
        ctl->done = 1;
      } else if ((long long)k >= max_iters) {
        ctl->status = PMSZ_ERR_NOT_CONVERGED;
        ctl->done = 1;
      } else {
        ctl->k = k + 1;
        ctl->steps += nf - al;
      }
      ctl->mism = 0;
      ctl->nflag = 0;
      ctl->at_lb = 0;
      ctl->ticket = 0;
      __threadfence();
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------

static int pick_chunk(int64_t extent, int64_t cols) {
  // enough blocks to fill 256 CUs several times over, long marches otherwise
  int64_t want = 8192;
  int64_t c = (extent * cols) / want;
  if (c < 1) c = 1;
  if (c > 64) c = 64;
  return (int)c;
}

template <class T, int MODE>
static hipError_t launch_stencil(const T* h, const Geo& G, uint8_t* dirs_out,
                                 const uint8_t* dirs_f, uint32_t* bm, Ctl* ctl, hipStream_t s) {
  if (G.ndim == 3) {
    const int64_t nbx = (G.nx + TX - 1) / TX, nby = (G.ny + TY - 1) / TY;
    const int zc = pick_chunk(G.nz, nbx * nby);
    const int64_t nbz = (G.nz + zc - 1) / zc;
    hipLaunchKernelGGL((k_stencil3<T, MODE>), dim3((unsigned)(nbx * nby * nbz)), dim3(256), 0, s,
                       h, G, zc, nbx, nby, dirs_out, dirs_f, bm, ctl);
  } else {
    const int64_t nbx = (G.nx + RX - 1) / RX;
    const int yc = pick_chunk(G.ny, nbx);
    const int64_t nby = (G.ny + yc - 1) / yc;
    hipLaunchKernelGGL((k_stencil2<T, MODE>), dim3((unsigned)(nbx * nby)), dim3(256), 0, s, h, G,
                       yc, nbx, dirs_out, dirs_f, bm, ctl);
  }
  return hipGetLastError();
}

static unsigned grid_for(int64_t items, int64_t cap) {
  int64_t b = (items + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

hipError_t launch_init(Ctl* ctl, uint32_t* bm, int64_t nwords, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(grid_for(nwords, 4096)), dim3(256), 0, s, ctl, bm, nwords);
  return hipGetLastError();
}

hipError_t launch_dirs(int dtype, const void* h, const Geo& G, uint8_t* dirs, hipStream_t s) {
  if (dtype == PMSZ_F32)
    return launch_stencil<float, MODE_DIRS>((const float*)h, G, dirs, nullptr, nullptr, nullptr,
                                            s);
  return launch_stencil<double, MODE_DIRS>((const double*)h, G, dirs, nullptr, nullptr, nullptr,
                                           s);
}

hipError_t launch_detect(int dtype, const void* g, const Geo& G, const uint8_t* dirs_f,
                         uint32_t* bm, Ctl* ctl, hipStream_t s) {
  if (dtype == PMSZ_F32)
    return launch_stencil<float, MODE_DETECT>((const float*)g, G, nullptr, dirs_f, bm, ctl, s);
  return launch_stencil<double, MODE_DETECT>((const double*)g, G, nullptr, dirs_f, bm, ctl, s);
}

hipError_t launch_validate(int dtype, const void* f, const void* fhat, int64_t n, double xi_t,
                           Ctl* ctl, hipStream_t s) {
  const unsigned grid = grid_for(n, 8192);
  if (dtype == PMSZ_F32)
    hipLaunchKernelGGL(k_validate<float>, dim3(grid), dim3(256), 0, s, (const float*)f,
                       (const float*)fhat, n, (float)xi_t, ctl);
  else
    hipLaunchKernelGGL(k_validate<double>, dim3(grid), dim3(256), 0, s, (const double*)f,
                       (const double*)fhat, n, xi_t, ctl);
  return hipGetLastError();
}

hipError_t launch_apply(int dtype, const void* f, void* g, const Geo& G, uint32_t* bm,
                        double xi_t, Ctl* ctl, int64_t max_iters, hipStream_t s) {
  const int64_t nwords = bitmap_words(G.n);
  const unsigned grid = grid_for(nwords, 4096);
  if (dtype == PMSZ_F32)
    hipLaunchKernelGGL(k_apply<float>, dim3(grid), dim3(256), 0, s, (const float*)f, (float*)g,
                       bm, nwords, (float)xi_t, ctl, max_iters);
  else
    hipLaunchKernelGGL(k_apply<double>, dim3(grid), dim3(256), 0, s, (const double*)f,
                       (double*)g, bm, nwords, xi_t, ctl, max_iters);
  return hipGetLastError();
}

}  // namespace pmsz
