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
// each side that has a neighbour block.  The owner of coordinate x is
// floor(((x+1) b - 1) / n); x is also held by block k-1 when it is block k's
// first vertex, and by block k+1 when it is block k's last.
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

// Blocks holding coordinate x of an axis of n vertices cut b ways, in
// increasing order (one to three).
__device__ __forceinline__ int holders(int64_t x, int64_t n, int64_t b, int32_t* k) {
  const int64_t o = ((x + 1) * b - 1) / n;
  int c = 0;
  if (o > 0 && x == o * n / b) k[c++] = (int32_t)(o - 1);
  k[c++] = (int32_t)o;
  if (o < b - 1 && x == (o + 1) * n / b - 1) k[c++] = (int32_t)(o + 1);
  return c;
}

// Ghost-layer exchange: every vertex takes the smallest of its copies (the
// later block in block order among equal values), the global field receives
// it, and every copy whose bits differ is overwritten.  *lowered counts the
// copies that were larger.
template <class T>
__global__ __launch_bounds__(256) void k_exchange(T* __restrict__ g_out, int64_t nx, int64_t ny,
                                                  int64_t nz, int32_t bx, int32_t by, int32_t bz,
                                                  const BlockCopy* __restrict__ tab,
                                                  unsigned long long* lowered) {
  const gptr<T> gg = as_global(g_out);
  const gptr<const BlockCopy> tb = as_global(tab);
  const int64_t sxy = nx * ny, n = sxy * nz;
  unsigned long long low = 0;
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * 256) {
    const int64_t x = v % nx, y = (v / nx) % ny, z = v / sxy;
    int32_t kx[3], ky[3], kz[3];
    const int cx = holders(x, nx, bx, kx), cy = holders(y, ny, by, ky),
              cz = holders(z, nz, bz, kz);
    T m = T(0);
    bool first = true;
    for (int c = 0; c < cz; ++c)
      for (int b = 0; b < cy; ++b)
        for (int a = 0; a < cx; ++a) {
          const int32_t id = kx[a] + bx * (ky[b] + by * kz[c]);
          const int64_t li = (x - tb[id].ox) + tb[id].lnx * ((y - tb[id].oy) + tb[id].lny * (z - tb[id].oz));
          const T cv = as_global((const T*)tb[id].g)[li];
          m = (first || !(m < cv)) ? cv : m;
          first = false;
        }
    gg[v] = m;
    if (cx * cy * cz > 1) {
      for (int c = 0; c < cz; ++c)
        for (int b = 0; b < cy; ++b)
          for (int a = 0; a < cx; ++a) {
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
                           const BlockCopy* tab, unsigned long long* lowered, hipStream_t s) {
  int64_t grid = (G.n + 255) / 256;
  if (grid > 65536) grid = 65536;
  if (dtype == PMSZ_F32)
    hipLaunchKernelGGL(k_exchange<float>, dim3((unsigned)grid), dim3(256), 0, s, (float*)g, G.nx,
                       G.ny, G.nz, nb[0], nb[1], nb[2], tab, lowered);
  else
    hipLaunchKernelGGL(k_exchange<double>, dim3((unsigned)grid), dim3(256), 0, s, (double*)g,
                       G.nx, G.ny, G.nz, nb[0], nb[1], nb[2], tab, lowered);
  return hipGetLastError();
}

}  // namespace pmsz
