// common.hpp -- device-side building blocks of libpmsz (gfx950).
//
// Everything here is the GPU library's own: it shares nothing with the CPU
// oracle that checks it.  Arithmetic follows IEEE-754 round-to-nearest in the
// field type; every source is compiled with -ffp-contract=off so that no
// product is fused into an add, and without fast-math.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pmsz.h"

namespace pmsz {

// ---------------------------------------------------------------------------
// Direction codes: 0 = self, m in 1..7 = offset +(m&1, m>>1&1, m>>2&1),
// 8+m = the negated offset.  Linear index delta of a code.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t code_delta(int code, int64_t nx, int64_t sxy) {
  int m = code & 7;
  int64_t d = (int64_t)(m & 1) + (int64_t)((m >> 1) & 1) * nx + (int64_t)((m >> 2) & 1) * sxy;
  return (code & 8) ? -d : d;
}

__device__ __forceinline__ int32_t code_delta32(int code, int32_t nx, int32_t sxy) {
  const int m = code & 7;
  const int32_t d = (m & 1) + ((m >> 1) & 1) * nx + ((m >> 2) & 1) * sxy;
  return (code & 8) ? -d : d;
}

// ---------------------------------------------------------------------------
// Floating-point helpers, per type.
// ---------------------------------------------------------------------------
template <class T> struct FP;

template <> struct FP<float> {
  using U = uint32_t;
  __device__ static __forceinline__ float nan() { return __builtin_nanf(""); }
  __device__ static __forceinline__ float maxv() { return 3.40282347e+38f; }
  __device__ static __forceinline__ float min_sub() { return __uint_as_float(1u); }
  __device__ static __forceinline__ U bits(float x) { return __float_as_uint(x); }
  __device__ static __forceinline__ float from(U b) { return __uint_as_float(b); }
};

template <> struct FP<double> {
  using U = uint64_t;
  __device__ static __forceinline__ double nan() { return __builtin_nan(""); }
  __device__ static __forceinline__ double maxv() { return 1.7976931348623157e+308; }
  __device__ static __forceinline__ double min_sub() { return __longlong_as_double(1ll); }
  __device__ static __forceinline__ U bits(double x) { return (U)__double_as_longlong(x); }
  __device__ static __forceinline__ double from(U b) { return __longlong_as_double((long long)b); }
};

// x with the bits of `m` OR-ed into its top 32 bits: m = 0 keeps x, m =
// 0x7fc00000 (binary32) / 0x7ff80000 (binary64 high word) makes it a quiet
// NaN.  A bitwise blend instead of a select keeps the load of x unconditional.
__device__ __forceinline__ float or_high(float x, uint32_t m) {
  return __uint_as_float(__float_as_uint(x) | m);
}
__device__ __forceinline__ double or_high(double x, uint32_t m) {
  return __longlong_as_double(__double_as_longlong(x) | ((long long)m << 32));
}
template <class T>
__device__ __forceinline__ uint32_t nan_mask();
template <>
__device__ __forceinline__ uint32_t nan_mask<float>() { return 0x7fc00000u; }
template <>
__device__ __forceinline__ uint32_t nan_mask<double>() { return 0x7ff80000u; }

// Next representable value toward +inf (x finite).
template <class T>
__device__ __forceinline__ T next_up(T x) {
  if (x == T(0)) return FP<T>::min_sub();
  typename FP<T>::U b = FP<T>::bits(x);
  return FP<T>::from(x > T(0) ? b + 1 : b - 1);
}
template <class T>
__device__ __forceinline__ T next_down(T x) {
  return -next_up<T>(-x);
}

// Knuth's TwoSum: a + b == s + e exactly (round-to-nearest, no fusion).
template <class T>
__device__ __forceinline__ void two_sum(T a, T b, T& s, T& e) {
  s = a + b;
  T bp = s - a;
  T ap = s - bp;
  e = (a - ap) + (b - bp);
}

// Smallest value >= f - xi and largest value <= f + xi (exact bounds).
template <class T>
__device__ __forceinline__ T lower_bound(T f, T xi) {
  T s, e;
  two_sum<T>(f, -xi, s, e);
  if (__builtin_isinf(s)) return -FP<T>::maxv();
  return e > T(0) ? next_up<T>(s) : s;
}
template <class T>
__device__ __forceinline__ T upper_bound(T f, T xi) {
  T s, e;
  two_sum<T>(f, xi, s, e);
  if (__builtin_isinf(s)) return FP<T>::maxv();
  return e < T(0) ? next_down<T>(s) : s;
}

// Eq. 1 with the halving edit: lb + (g - lb)/2, or lb when that would not
// decrease g.
template <class T>
__device__ __forceinline__ T halving_edit(T g, T lb) {
  T h = g - lb;
  T m = lb + T(0.5) * h;
  return (m < g) ? m : lb;
}

// ---------------------------------------------------------------------------
// Global-address-space views of pointers that arrive as generic pointers (for
// instance through a descriptor table).  Loads through them are global loads,
// which count only in the vector-memory counter; generic (flat) loads also
// count in the LDS counter, so every LDS barrier would wait for them.
// ---------------------------------------------------------------------------
template <class T>
using gptr = T __attribute__((address_space(1)))*;

template <class T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}

// A pointer or integer that is the same in every active lane, moved into
// scalar registers.  Values read from a descriptor table through a vector
// load stay in vector registers, and every address formed from them then
// costs 64-bit vector arithmetic per load; from scalar registers the loads
// take a scalar base and a 32-bit lane offset.
__device__ __forceinline__ int32_t uniform(int32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}
// Makes a loop-invariant 32-bit lane offset opaque to loop-invariant code
// motion, in place (an empty asm statement that claims to rewrite the
// register; no instruction is emitted).  Otherwise the compiler widens the
// offset to 64 bits outside the loop, and every load inside it then pays a
// 64-bit vector add instead of taking the scalar-base + 32-bit-offset form.
__device__ __forceinline__ void opaque_off(uint32_t& o) { asm volatile("" : "+v"(o)); }

template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return (T*)(((unsigned long long)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Block barrier that orders LDS only.  A plain __syncthreads() also waits for
// every outstanding global load of the wave (gfx9 counts loads and stores in
// one counter), which would cancel the register prefetch of the tile marches;
// this barrier leaves global loads in flight.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Reductions.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block; the result is valid in thread 0.  `sh` needs one slot
// per wave.
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v,
                                                        unsigned long long* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  unsigned long long r = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;
}

// Device-scope load that bypasses stale caches.
__device__ __forceinline__ unsigned long long load_acquire(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace pmsz
