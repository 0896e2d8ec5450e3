// verify.hip -- evaluation counts (Sec. V-D: wrongly labelled points, false
// maxima and minima), recomputed from the direction bytes and labels of f and
// g, plus bound checks and the largest |g - f|.
#include "launch.hpp"

namespace pmsz {

template <class T>
__global__ __launch_bounds__(256) void k_verify(
    const T* __restrict__ f, const T* __restrict__ g, const T* __restrict__ fh, int64_t n, T xi,
    const uint8_t* __restrict__ df, const uint8_t* __restrict__ dg,
    const int32_t* __restrict__ lfx, const int32_t* __restrict__ lfn,
    const int32_t* __restrict__ lgx, const int32_t* __restrict__ lgn, VerifyCounts* out) {
  __shared__ unsigned long long red[4];
  __shared__ unsigned long long emax[4];
  unsigned long long c[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  double err = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const T a = f[i], b = g[i];
    const bool inside = __builtin_isfinite(b) && b >= lower_bound<T>(a, xi) &&
                        b <= upper_bound<T>(a, xi);
    c[0] += !inside;
    const double e = __builtin_fabs((double)b - (double)a);
    if (!(e <= err)) err = (e != e) ? __builtin_inf() : e;
    const int af = df[i] & 15, ag = dg[i] & 15, nf = df[i] >> 4, ng = dg[i] >> 4;
    c[1] += af != ag;
    c[2] += nf != ng;
    c[3] += (ag == 0 && af != 0);
    c[4] += (ng == 0 && nf != 0);
    c[5] += (af == 0 && ag != 0);
    c[6] += (nf == 0 && ng != 0);
    const bool w1 = lfx[i] != lgx[i], w2 = lfn[i] != lgn[i];
    c[7] += w1;
    c[8] += w2;
    c[9] += (w1 || w2);
    if (fh) c[10] += (fh[i] != b);
  }
#pragma unroll
  for (int k = 0; k < 11; ++k) {
    const unsigned long long t = block_sum(c[k], red);
    if (threadIdx.x == 0 && t) atomicAdd(&out->c[k], t);
  }
  // non-negative doubles order like their bit patterns
  unsigned long long eb = (unsigned long long)__double_as_longlong(err);
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(eb, off, 64);
    eb = o > eb ? o : eb;
  }
  if ((threadIdx.x & 63) == 0) emax[threadIdx.x >> 6] = eb;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int w = 0; w < 4; ++w) m = emax[w] > m ? emax[w] : m;
    atomicMax(&out->max_err_bits, m);
  }
}

hipError_t launch_verify(int dtype, const void* f, const void* g, const void* fhat, int64_t n,
                         double xi_t, const uint8_t* df, const uint8_t* dg, const int32_t* lf_max,
                         const int32_t* lf_min, const int32_t* lg_max, const int32_t* lg_min,
                         VerifyCounts* out, hipStream_t s) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  if (dtype == PMSZ_F32)
    hipLaunchKernelGGL(k_verify<float>, dim3((unsigned)b), dim3(256), 0, s, (const float*)f,
                       (const float*)g, (const float*)fhat, n, (float)xi_t, df, dg, lf_max,
                       lf_min, lg_max, lg_min, out);
  else
    hipLaunchKernelGGL(k_verify<double>, dim3((unsigned)b), dim3(256), 0, s, (const double*)f,
                       (const double*)g, (const double*)fhat, n, xi_t, df, dg, lf_max, lf_min,
                       lg_max, lg_min, out);
  return hipGetLastError();
}

}  // namespace pmsz
