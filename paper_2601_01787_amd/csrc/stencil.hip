// stencil.hip -- standalone steepest-direction pass (pmsz_directions and the
// directions used by verification): one block per tile of the shared tile
// code, writing one direction byte per vertex.
#include "launch.hpp"
#include "tiles.hpp"

namespace pmsz {

template <class T>
__global__ __launch_bounds__(256) void k_dirs(const T* __restrict__ h, TileGeo G,
                                              uint8_t* __restrict__ dirs) {
  __shared__ TileLds<T> sm;
  __shared__ unsigned long long red[4];
  if (G.ndim == 3)
    tile3<T, KIND_DIRS>(sm, red, h, nullptr, dirs, nullptr, T(0), G, blockIdx.x);
  else
    tile2<T, KIND_DIRS>(sm, red, h, nullptr, dirs, nullptr, T(0), G, blockIdx.x);
}

// Longer marches than the correction engine uses (no frontier to keep fine),
// while still giving the chip several blocks per compute unit.
static int dirs_chunk(int ndim, int64_t nx, int64_t ny, int64_t nz) {
  const int64_t cols = ndim == 3 ? ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY) : (nx + RX - 1) / RX;
  const int64_t depth = ndim == 3 ? nz : ny;
  int64_t c = depth * cols / 4096;
  if (c < 2) c = 2;
  if (c > 64) c = 64;
  return (int)c;
}

hipError_t launch_dirs(int dtype, const void* h, const Geo& g, uint8_t* dirs, hipStream_t s) {
  const TileGeo G = make_tile_geo(g.ndim, g.nx, g.ny, g.nz, dirs_chunk(g.ndim, g.nx, g.ny, g.nz));
  const unsigned grid = (unsigned)tile_count(G);
  if (dtype == PMSZ_F32)
    hipLaunchKernelGGL(k_dirs<float>, dim3(grid), dim3(256), 0, s, (const float*)h, G, dirs);
  else
    hipLaunchKernelGGL(k_dirs<double>, dim3(grid), dim3(256), 0, s, (const double*)h, G, dirs);
  return hipGetLastError();
}

}  // namespace pmsz
