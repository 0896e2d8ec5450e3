// blocks.hip -- copies and ghost-layer exchange of a decomposed domain.
//
// Sec. IV-B cuts the domain into non-overlapping blocks, each extended by a
// one-vertex ghost layer, corrects every block on its own and then
// reconciles the copies of shared vertices by taking their minimum.  On one
// GPU the blocks are fields of one batched engine launch (each compares only
// its core); these kernels move values between the global field and the
// block copies.
//
// Cuts: along an axis of n vertices split into b blocks, block k owns
// [floor(k n / b), floor((k+1) n / b)); its copy spans one more vertex on
// each side that has a neighbour block, so a coordinate is held by its owner,
// by the block before when it is the owner's first vertex and by the block
// after when it is the owner's last (the host tabulates this per axis).
#include "launch.hpp"

namespace pmsz {

// Copy the box [o, o + l) of a global field into a dense block array.
template <class T>
__global__ __launch_bounds__(256) void k_box_gather(const T* __restrict__ src, int64_t nx,
                                                    int64_t sxy, int64_t ox, int64_t oy,
                                                    int64_t oz, int64_t lnx, int64_t lny,
                                                    int64_t ln, T* __restrict__ dst) {
  const gptr<const T> s = as_global(src);
  const gptr<T> d = as_global(dst);
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < ln;
       j += (int64_t)gridDim.x * 256) {
    const int64_t lx = j % lnx, ly = (j / lnx) % lny, lz = j / (lnx * lny);
    d[j] = s[(ox + lx) + nx * (oy + ly) + sxy * (oz + lz)];
  }
}

hipError_t blocks_gather(int dtype, const void* src, const Geo& G, const int64_t o[3],
                         const int64_t l[3], void* dst, hipStream_t s) {
  const int64_t ln = l[0] * l[1] * l[2];
  if (ln == 0) return hipSuccess;
  int64_t grid = (ln + 255) / 256;
  if (grid > 16384) grid = 16384;
  if (dtype == PMSZ_F32)
    hipLaunchKernelGGL(k_box_gather<float>, dim3((unsigned)grid), dim3(256), 0, s,
                       (const float*)src, G.nx, G.sxy, o[0], o[1], o[2], l[0], l[1], ln,
                       (float*)dst);
  else
    hipLaunchKernelGGL(k_box_gather<double>, dim3((unsigned)grid), dim3(256), 0, s,
                       (const double*)src, G.nx, G.sxy, o[0], o[1], o[2], l[0], l[1], ln,
                       (double*)dst);
  return hipGetLastError();
}

// Owner copy-back: the core of block copy `src` (core box [c0, c1) in the
// copy's coordinates, copy origin o in the grid) into the global field.  One
// row (y, z) of the core per workgroup iteration, x across threads.
template <class T>
__global__ __launch_bounds__(256) void k_core_scatter(const T* __restrict__ src, int64_t lnx,
                                                      int64_t lny, int32_t cx0, int32_t cx1,
                                                      int32_t cy0, int32_t cy1, int32_t cz0,
                                                      int32_t cz1, int64_t ox, int64_t oy,
                                                      int64_t oz, T* __restrict__ dst, int64_t nx,
                                                      int64_t sxy) {
  const gptr<const T> sp = as_global(src);
  const gptr<T> dp = as_global(dst);
  const int32_t ry = cy1 - cy0;
  const int64_t rows = (int64_t)ry * (cz1 - cz0);
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const int32_t ly = cy0 + (int32_t)(r % ry), lz = cz0 + (int32_t)(r / ry);
    const int64_t lrow = lnx * (ly + lny * lz);
    const int64_t grow = (ox) + nx * (oy + ly) + sxy * (oz + lz);
    for (int32_t lx = cx0 + threadIdx.x; lx < cx1; lx += 256) dp[grow + lx] = sp[lrow + lx];
  }
}

hipError_t blocks_scatter_core(int dtype, const void* src, const int64_t l[3], const int64_t c[6],
                               const int64_t o[3], void* dst, const Geo& G, hipStream_t s) {
  const int64_t rows = (c[3] - c[2]) * (c[5] - c[4]);
  if (rows <= 0 || c[1] <= c[0]) return hipSuccess;
  int64_t grid = rows < 16384 ? rows : 16384;
  if (dtype == PMSZ_F32)
    hipLaunchKernelGGL(k_core_scatter<float>, dim3((unsigned)grid), dim3(256), 0, s,
                       (const float*)src, l[0], l[1], (int32_t)c[0], (int32_t)c[1], (int32_t)c[2],
                       (int32_t)c[3], (int32_t)c[4], (int32_t)c[5], o[0], o[1], o[2], (float*)dst,
                       G.nx, G.sxy);
  else
    hipLaunchKernelGGL(k_core_scatter<double>, dim3((unsigned)grid), dim3(256), 0, s,
                       (const double*)src, l[0], l[1], (int32_t)c[0], (int32_t)c[1],
                       (int32_t)c[2], (int32_t)c[3], (int32_t)c[4], (int32_t)c[5], o[0], o[1],
                       o[2], (double*)dst, G.nx, G.sxy);
  return hipGetLastError();
}

// Ghost-layer exchange of the shared vertices: every vertex held by more
// than one block copy lies on a boundary layer (the two vertices either side
// of a cut) of some axis.  planes lists those layers as (axis, coordinate);
// a vertex is handled in the plane of the first axis on which it is shared.
// It takes the smallest of its copies (the later block in block order among
// equal values), the global field receives it, and every copy whose bits
// differ is overwritten; *lowered counts the copies that were larger.
// hold: per axis and coordinate, the (up to three, ascending, -1 padded)
// blocks along that axis whose copies hold it, for x, then y, then z.
template <class T>
__global__ __launch_bounds__(256) void k_exchange(T* __restrict__ g_out, int32_t nx, int32_t ny,
                                                  int32_t nz, int32_t bx, int32_t by,
                                                  const BlockCopy* __restrict__ tab,
                                                  const int32_t* __restrict__ hold,
                                                  const int32_t* __restrict__ planes,
                                                  int32_t n_planes, unsigned long long* lowered) {
  const gptr<T> gg = as_global(g_out);
  const gptr<const BlockCopy> tb = as_global(tab);
  const gptr<const int32_t> hx = as_global(hold);
  const gptr<const int32_t> hy = hx + 3 * (int64_t)nx;
  const gptr<const int32_t> hz = hy + 3 * (int64_t)ny;
  const gptr<const int32_t> pl = as_global(planes);
  unsigned long long low = 0;
  const int32_t dims[3] = {nx, ny, nz};
  for (int32_t q = 0; q < n_planes; ++q) {
    const int32_t axis = pl[2 * q], coord = pl[2 * q + 1];
    // the plane's two other axes: u varies fastest
    const int32_t ua = axis == 0 ? 1 : 0, va = axis == 2 ? 1 : 2;
    const int64_t nu = dims[ua], nv = dims[va];
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nu * nv;
         e += (int64_t)gridDim.x * 256) {
      int32_t xyz[3];
      xyz[axis] = coord;
      xyz[ua] = (int32_t)(e % nu);
      xyz[va] = (int32_t)(e / nu);
      const int32_t x = xyz[0], y = xyz[1], z = xyz[2];
      int32_t kx[3], ky[3], kz[3];
      for (int j = 0; j < 3; ++j) {
        kx[j] = hx[3 * (int64_t)x + j];
        ky[j] = hy[3 * (int64_t)y + j];
        kz[j] = hz[3 * (int64_t)z + j];
      }
      // shared on an earlier axis: that axis' plane handles it
      if (axis >= 1 && kx[1] >= 0) continue;
      if (axis == 2 && ky[1] >= 0) continue;
      T m = T(0);
      bool first = true;
      for (int c = 0; c < 3 && kz[c] >= 0; ++c)
        for (int b = 0; b < 3 && ky[b] >= 0; ++b)
          for (int a = 0; a < 3 && kx[a] >= 0; ++a) {
            const int32_t id = kx[a] + bx * (ky[b] + by * kz[c]);
            const int64_t li = (x - tb[id].ox) + tb[id].lnx * ((y - tb[id].oy) + tb[id].lny * (z - tb[id].oz));
            const T cv = as_global((const T*)tb[id].g)[li];
            m = (first || !(m < cv)) ? cv : m;
            first = false;
          }
      gg[(int64_t)x + (int64_t)nx * (y + (int64_t)ny * z)] = m;
      for (int c = 0; c < 3 && kz[c] >= 0; ++c)
        for (int b = 0; b < 3 && ky[b] >= 0; ++b)
          for (int a = 0; a < 3 && kx[a] >= 0; ++a) {
            const int32_t id = kx[a] + bx * (ky[b] + by * kz[c]);
            const int64_t li = (x - tb[id].ox) + tb[id].lnx * ((y - tb[id].oy) + tb[id].lny * (z - tb[id].oz));
            const gptr<T> p = as_global((T*)tb[id].g) + li;
            const T cv = *p;
            low += cv > m ? 1u : 0u;
            if (FP<T>::bits(cv) != FP<T>::bits(m)) *p = m;
          }
    }
  }
  const unsigned long long w = wave_sum(low);
  if ((threadIdx.x & 63) == 0 && w)
    __hip_atomic_fetch_add(as_global(lowered), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t blocks_exchange(int dtype, void* g, const Geo& G, const int32_t nb[3],
                           const BlockCopy* tab, const int32_t* hold, const int32_t* planes,
                           int32_t n_planes, int64_t max_plane, unsigned long long* lowered,
                           hipStream_t s) {
  if (n_planes == 0) return hipSuccess;
  int64_t grid = (max_plane + 255) / 256;
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  if (dtype == PMSZ_F32)
    hipLaunchKernelGGL(k_exchange<float>, dim3((unsigned)grid), dim3(256), 0, s, (float*)g,
                       (int32_t)G.nx, (int32_t)G.ny, (int32_t)G.nz, nb[0], nb[1], tab, hold,
                       planes, n_planes, lowered);
  else
    hipLaunchKernelGGL(k_exchange<double>, dim3((unsigned)grid), dim3(256), 0, s, (double*)g,
                       (int32_t)G.nx, (int32_t)G.ny, (int32_t)G.nz, nb[0], nb[1], tab, hold,
                       planes, n_planes, lowered);
  return hipGetLastError();
}

}  // namespace pmsz
