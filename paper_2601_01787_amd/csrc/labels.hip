// labels.hip -- ascending / descending segmentation labels (Sec. III-A:
// integral lines follow the steepest direction to an extremum; a segmentation
// groups the vertices that reach the same one).
//
// The steepest-direction pointers form a forest whose roots are the extrema
// (each pointer strictly climbs the index-tie-broken order, so there are no
// cycles).  Labels are found by pointer jumping in place: every pass replaces
// L[i] by an ancestor further up the chain, chasing a few hops per pass.  Any
// value a thread reads -- old or already updated -- is an ancestor of i, so
// the fixed point is the root whatever the interleaving.
#include "launch.hpp"

namespace pmsz {

__global__ __launch_bounds__(256) void k_labels_init(const uint8_t* __restrict__ dirs, Geo G,
                                                     int32_t* __restrict__ lmax,
                                                     int32_t* __restrict__ lmin) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < G.n; i += stride) {
    const int d = dirs[i];
    if (lmax) lmax[i] = (int32_t)(i + code_delta(d & 15, G.nx, G.sxy));
    if (lmin) lmin[i] = (int32_t)(i + code_delta(d >> 4, G.nx, G.sxy));
  }
}

__global__ __launch_bounds__(256) void k_labels_jump(int32_t* lab, int64_t n,
                                                     unsigned int* changed) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  int any = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const int32_t l0 = lab[i];
    int32_t l = l0;
#pragma unroll 1
    for (int hop = 0; hop < 8; ++hop) {
      const int32_t ll = lab[l];
      if (ll == l) break;
      l = ll;
    }
    if (l != l0) {
      lab[i] = l;
      any = 1;
    }
  }
  if (__ballot(any) != 0ull && (threadIdx.x & 63) == 0) atomicOr(changed, 1u);
}

static unsigned grid_for(int64_t items) {
  int64_t b = (items + 255) / 256;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

hipError_t launch_labels_init(const uint8_t* dirs, const Geo& G, int32_t* lmax, int32_t* lmin,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_labels_init, dim3(grid_for(G.n)), dim3(256), 0, s, dirs, G, lmax, lmin);
  return hipGetLastError();
}

hipError_t launch_labels_jump(int32_t* lab, int64_t n, unsigned int* changed, hipStream_t s) {
  hipLaunchKernelGGL(k_labels_jump, dim3(grid_for(n)), dim3(256), 0, s, lab, n, changed);
  return hipGetLastError();
}

}  // namespace pmsz
