// probe.hip -- read-only kernels of known traffic for calibrating the memory
// counters (FETCH_SIZE) against the access patterns of the tile marches:
// every byte of the buffer is read exactly once, in the shape the marches
// use, and the values are summed so that no load is elided.
#include "launch.hpp"

namespace pmsz {

// pattern 0: dword rows (64 lanes read 256 contiguous bytes per instruction,
// like a plane row of binary32 values); pattern 1: byte rows (64 contiguous
// bytes per instruction, like the direction bytes of a row of vertices).
template <int PATTERN>
__global__ __launch_bounds__(256) void k_probe_read(const uint8_t* __restrict__ p, int64_t bytes,
                                                    unsigned long long* out) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  unsigned long long acc = 0;
  if (PATTERN == 0) {
    const gptr<const uint32_t> w = as_global((const uint32_t*)p);
    const int64_t n = bytes / 4;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) acc += w[i];
  } else {
    const gptr<const uint8_t> b = as_global(p);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < bytes; i += stride) acc += b[i];
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, acc);
}

hipError_t launch_probe_read(const void* p, int64_t bytes, int pattern, unsigned long long* out,
                             hipStream_t s) {
  int64_t items = pattern == 0 ? bytes / 4 : bytes;
  int64_t grid = (items + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  if (pattern == 0)
    hipLaunchKernelGGL(k_probe_read<0>, dim3((unsigned)grid), dim3(256), 0, s,
                       (const uint8_t*)p, bytes, out);
  else
    hipLaunchKernelGGL(k_probe_read<1>, dim3((unsigned)grid), dim3(256), 0, s,
                       (const uint8_t*)p, bytes, out);
  return hipGetLastError();
}

}  // namespace pmsz
