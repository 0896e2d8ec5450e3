// labels.hip -- ascending / descending segmentation labels (Sec. III-A:
// integral lines follow the steepest direction to an extremum; a segmentation
// groups the vertices that reach the same one), and the check of
// caller-supplied direction bytes.
//
// The steepest-direction pointers form a forest whose roots are the extrema
// (each pointer strictly climbs the index-tie-broken order, so there are no
// cycles).  Labels are found by pointer jumping in place: every pass replaces
// L[i] by an ancestor further up the chain, chasing a few hops per pass.  Any
// value a thread reads -- old or already updated -- is an ancestor of i, so
// the fixed point is the root whatever the interleaving.  In a forest a pass
// in which no label changed proves every label is a root: a chase from a
// non-root climbs at least one step.
#include "launch.hpp"

namespace pmsz {

// 1 when `code` names the vertex itself or a Freudenthal neighbour of (x, y, z)
// inside the grid: no code 8, no z bit in 2D, no step out of the box.
__device__ __forceinline__ bool code_valid(int code, int64_t x, int64_t y, int64_t z,
                                           const Geo& G) {
  if (code == 0) return true;
  if (code == 8) return false;
  const int m = code & 7;
  if (G.ndim == 2 && (m & 4)) return false;
  const int s = (code & 8) ? -1 : 1;
  const int64_t X = x + s * (m & 1), Y = y + s * ((m >> 1) & 1), Z = z + s * ((m >> 2) & 1);
  return X >= 0 && X < G.nx && Y >= 0 && Y < G.ny && Z >= 0 && Z < G.nz;
}

// Counts the direction bytes holding a code that is not valid for their vertex
// (either nibble).
__global__ __launch_bounds__(256) void k_check_dirs(const uint8_t* __restrict__ dirs, Geo G,
                                                    unsigned long long* bad) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  unsigned long long nb = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < G.n; i += stride) {
    const int d = dirs[i];
    const int64_t x = i % G.nx, y = (i / G.nx) % G.ny, z = i / G.sxy;
    nb += !(code_valid(d & 15, x, y, z, G) && code_valid(d >> 4, x, y, z, G));
  }
  nb = wave_sum(nb);
  if ((threadIdx.x & 63) == 0 && nb) atomicAdd(bad, nb);
}

// Initial labels: the neighbour each vertex points at.  An invalid code makes
// the vertex its own label (so every later read stays inside the arrays) and
// is counted in *bad.
__global__ __launch_bounds__(256) void k_labels_init(const uint8_t* __restrict__ dirs, Geo G,
                                                     int32_t* __restrict__ lmax,
                                                     int32_t* __restrict__ lmin,
                                                     unsigned long long* bad) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  unsigned long long nb = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < G.n; i += stride) {
    const int d = dirs[i];
    const int64_t x = i % G.nx, y = (i / G.nx) % G.ny, z = i / G.sxy;
    const bool va = code_valid(d & 15, x, y, z, G), vd = code_valid(d >> 4, x, y, z, G);
    nb += !(va && vd);
    if (lmax) lmax[i] = (int32_t)(va ? i + code_delta(d & 15, G.nx, G.sxy) : i);
    if (lmin) lmin[i] = (int32_t)(vd ? i + code_delta(d >> 4, G.nx, G.sxy) : i);
  }
  nb = wave_sum(nb);
  if ((threadIdx.x & 63) == 0 && nb) atomicAdd(bad, nb);
}

// Pass `pass` of pointer jumping over the labels of the nibble `shift` (0:
// n_max, 4: n_min) of `dirs`.  flags[pass] is set when some label moved; a
// pass whose predecessor moved nothing returns at once, so a batch of passes
// can be queued without reading anything back in between.
// Caller-supplied bytes need not form a forest; a cycle is caught two ways,
// counted in *bad: a chase that ends where it started without reaching a
// root has gone round it, and a vertex that reads as a root (its label is
// itself) while its code is not 0 was made one by in-place jumping round it.
// A vertex on a cycle only ever labels itself with vertices of that cycle,
// never with a true extremum, so the second test catches every cycle that
// settles; one that never settles fails on the pass limit.
__global__ __launch_bounds__(256) void k_labels_jump(int32_t* lab, int64_t n,
                                                     const uint8_t* __restrict__ dirs, int shift,
                                                     unsigned int* flags, unsigned long long* bad,
                                                     int pass) {
  if (pass > 0 && flags[pass - 1] == 0u) return;
  const int64_t stride = (int64_t)gridDim.x * 256;
  int any = 0;
  unsigned long long cyc = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const int32_t l0 = lab[i];
    int32_t l = l0;
    bool root = false;
#pragma unroll 1
    for (int hop = 0; hop < kLabelHops; ++hop) {
      const int32_t ll = lab[l];
      if (ll == l) {
        root = true;
        cyc += ((dirs[l] >> shift) & 15) != 0;  // a false root
        break;
      }
      l = ll;
    }
    if (l != l0) {
      lab[i] = l;
      any = 1;
    } else if (!root) {
      ++cyc;
    }
  }
  if (__ballot(any) != 0ull && (threadIdx.x & 63) == 0) atomicOr(flags + pass, 1u);
  cyc = wave_sum(cyc);
  if ((threadIdx.x & 63) == 0 && cyc) atomicAdd(bad, cyc);
}

static unsigned grid_for(int64_t items) {
  int64_t b = (items + 255) / 256;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

hipError_t launch_check_dirs(const uint8_t* dirs, const Geo& G, unsigned long long* bad,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_check_dirs, dim3(grid_for(G.n)), dim3(256), 0, s, dirs, G, bad);
  return hipGetLastError();
}

hipError_t launch_labels_init(const uint8_t* dirs, const Geo& G, int32_t* lmax, int32_t* lmin,
                              unsigned long long* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_labels_init, dim3(grid_for(G.n)), dim3(256), 0, s, dirs, G, lmax, lmin,
                     bad);
  return hipGetLastError();
}

hipError_t launch_labels_jump(int32_t* lab, int64_t n, const uint8_t* dirs, int shift,
                              unsigned int* flags, unsigned long long* bad, int pass,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_labels_jump, dim3(grid_for(n)), dim3(256), 0, s, lab, n, dirs, shift,
                     flags, bad, pass);
  return hipGetLastError();
}

}  // namespace pmsz
