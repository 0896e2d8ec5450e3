// edits.hip -- the edit stream: encoding of the corrections for storage.
//
// The correction changes a few values of the decompressed field; storing it
// means storing those changes (Sec. V-D reports this as the method's storage
// overhead; the paper fixes no format).  Stream layout (little-endian):
//   header   'PMSE', u8 version 1, u8 dtype, u16 0, u64 vertices, u64 edits,
//            u64 payload bytes, u32 chunk (entries per chunk), u32 chunks
//   table    per chunk: u64 payload offset of its first entry, u64 index of
//            the edited vertex before it (all ones when none)
//   payload  per vertex i whose bits changed, ascending: gap = i - previous
//            edited index - 1 and steps = key(fhat_i) - key(g_i), each as an
//            unsigned LEB128 varint; key() maps values to integers in value
//            order, so steps counts the representable values in (g_i, fhat_i].
// Encoding is a chain of data-parallel passes (count, scan, compact, sizes,
// scan, write); decoding runs one thread per chunk of the table.
#include <string.h>

#include "launch.hpp"

namespace pmsz {

constexpr int kEditChunk = 4096;    // entries per chunk of the table
constexpr int kScanItems = 4096;    // items per block of the scans
constexpr int kCountItems = 4096;   // vertices per block of the count / compact

__device__ __forceinline__ unsigned long long order_key(float v) {
  const uint32_t b = __float_as_uint(v);
  return (b & 0x80000000u) ? (unsigned long long)(~b) : (unsigned long long)(b | 0x80000000u);
}
__device__ __forceinline__ unsigned long long order_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ void from_order_key(unsigned long long k, float* out) {
  const uint32_t kk = (uint32_t)k;
  *out = __uint_as_float((kk & 0x80000000u) ? (kk & 0x7fffffffu) : ~kk);
}
__device__ __forceinline__ void from_order_key(unsigned long long k, double* out) {
  *out = __longlong_as_double(
      (long long)((k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k));
}

template <class T>
__device__ __forceinline__ bool bits_differ(T a, T b);
template <>
__device__ __forceinline__ bool bits_differ<float>(float a, float b) {
  return __float_as_uint(a) != __float_as_uint(b);
}
template <>
__device__ __forceinline__ bool bits_differ<double>(double a, double b) {
  return __double_as_longlong(a) != __double_as_longlong(b);
}

__device__ __forceinline__ uint32_t leb_len(unsigned long long v) {
  uint32_t n = 1;
  while (v >= 0x80ull) {
    v >>= 7;
    ++n;
  }
  return n;
}

// Exclusive sum over the 256 threads of a block; *total (all threads).
__device__ __forceinline__ unsigned long long block_excl(unsigned long long v,
                                                         unsigned long long* sh,
                                                         unsigned long long* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  unsigned long long before = 0, all = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) before += sh[w];
    all += sh[w];
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

// ---- exclusive scan of n uint32 values into uint64 offsets -----------------
// Pass 1: sum of each block of kScanItems items.
__global__ __launch_bounds__(256) void k_scan_sums(const uint32_t* in, int64_t n,
                                                   unsigned long long* sums) {
  __shared__ unsigned long long sh[4];
  const int64_t b0 = (int64_t)blockIdx.x * kScanItems;
  unsigned long long v = 0;
  for (int k = 0; k < kScanItems / 256; ++k) {
    const int64_t i = b0 + threadIdx.x + 256 * k;
    if (i < n) v += in[i];
  }
  unsigned long long total;
  block_excl(v, sh, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}
// Pass 2: one block scans the block sums in place (exclusive); the grand
// total goes to *total.
__global__ __launch_bounds__(256) void k_scan_top(unsigned long long* sums, int64_t nb,
                                                  unsigned long long* total) {
  __shared__ unsigned long long sh[4];
  const int64_t per = (nb + 255) / 256;
  const int64_t b0 = threadIdx.x * per;
  unsigned long long v = 0;
  for (int64_t i = b0; i < b0 + per && i < nb; ++i) v += sums[i];
  unsigned long long all;
  unsigned long long run = block_excl(v, sh, &all);
  for (int64_t i = b0; i < b0 + per && i < nb; ++i) {
    const unsigned long long s = sums[i];
    sums[i] = run;
    run += s;
  }
  if (threadIdx.x == 0) *total = all;
}
// Pass 3: each block rescans its items from its offset.  A thread takes a
// contiguous run of kScanItems/256 items so the order is preserved.
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* in, int64_t n,
                                                    const unsigned long long* sums,
                                                    unsigned long long* out) {
  __shared__ unsigned long long sh[4];
  constexpr int kPer = kScanItems / 256;
  const int64_t i0 = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kPer;
  unsigned long long v = 0;
  for (int k = 0; k < kPer; ++k)
    if (i0 + k < n) v += in[i0 + k];
  unsigned long long total;
  unsigned long long run = sums[blockIdx.x] + block_excl(v, sh, &total);
  for (int k = 0; k < kPer; ++k)
    if (i0 + k < n) {
      out[i0 + k] = run;
      run += in[i0 + k];
    }
}

// ---- encoder passes ----------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_edit_count(const T* fhat, const T* g, int64_t n,
                                                    uint32_t* counts) {
  __shared__ unsigned long long sh[4];
  constexpr int kPer = kCountItems / 256;
  const int64_t i0 = (int64_t)blockIdx.x * kCountItems + (int64_t)threadIdx.x * kPer;
  unsigned long long c = 0;
  for (int k = 0; k < kPer; ++k)
    if (i0 + k < n && bits_differ<T>(fhat[i0 + k], g[i0 + k])) ++c;
  unsigned long long total;
  block_excl(c, sh, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = (uint32_t)total;
}

// Index of every changed vertex, in ascending order, at its rank (block base
// from the scanned counts plus the rank inside the block); ranks at or past
// cap are not written.
template <class T>
__global__ __launch_bounds__(256) void k_edit_compact(const T* fhat, const T* g, int64_t n,
                                                      const unsigned long long* base,
                                                      uint32_t* idx, int64_t cap) {
  __shared__ unsigned long long sh[4];
  constexpr int kPer = kCountItems / 256;
  const int64_t i0 = (int64_t)blockIdx.x * kCountItems + (int64_t)threadIdx.x * kPer;
  unsigned long long c = 0;
  for (int k = 0; k < kPer; ++k)
    if (i0 + k < n && bits_differ<T>(fhat[i0 + k], g[i0 + k])) ++c;
  unsigned long long total;
  unsigned long long r = base[blockIdx.x] + block_excl(c, sh, &total);
  for (int k = 0; k < kPer; ++k)
    if (i0 + k < n && bits_differ<T>(fhat[i0 + k], g[i0 + k])) {
      if ((int64_t)r < cap) idx[r] = (uint32_t)(i0 + k);
      ++r;
    }
}

template <class T>
__device__ __forceinline__ void edit_entry(const T* fhat, const T* g, const uint32_t* idx,
                                           int64_t r, unsigned long long& gap,
                                           unsigned long long& steps) {
  const int64_t i = idx[r];
  const int64_t prev = r ? (int64_t)idx[r - 1] : -1;
  gap = (unsigned long long)(i - prev - 1);
  steps = order_key(fhat[i]) - order_key(g[i]);
}

template <class T>
__global__ __launch_bounds__(256) void k_edit_sizes(const T* fhat, const T* g,
                                                    const uint32_t* idx, int64_t ne,
                                                    uint32_t* len) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= ne) return;
  unsigned long long gap, steps;
  edit_entry<T>(fhat, g, idx, r, gap, steps);
  len[r] = leb_len(gap) + leb_len(steps);
}

__device__ __forceinline__ uint8_t* put_leb(uint8_t* p, unsigned long long v) {
  while (v >= 0x80ull) {
    *p++ = (uint8_t)(v | 0x80ull);
    v >>= 7;
  }
  *p++ = (uint8_t)v;
  return p;
}

template <class T>
__global__ __launch_bounds__(256) void k_edit_write(const T* fhat, const T* g,
                                                    const uint32_t* idx, int64_t ne,
                                                    const unsigned long long* off,
                                                    uint8_t* table, uint8_t* payload) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= ne) return;
  unsigned long long gap, steps;
  edit_entry<T>(fhat, g, idx, r, gap, steps);
  uint8_t* p = put_leb(payload + off[r], gap);
  put_leb(p, steps);
  if (r % kEditChunk == 0) {
    unsigned long long* t = (unsigned long long*)(table + 16 * (r / kEditChunk));
    t[0] = off[r];
    t[1] = r ? (unsigned long long)idx[r - 1] : ~0ull;
  }
}

// ---- decoder -------------------------------------------------------------------
// One thread per chunk: walks its entries and lowers g (holding fhat) at each
// edited vertex by `steps` representable values.  Reads past the payload or
// indices past the field set *err and stop the chunk.
template <class T>
__global__ __launch_bounds__(256) void k_edit_decode(const uint8_t* table, const uint8_t* payload,
                                                     int64_t payload_bytes, int64_t ne,
                                                     int64_t n, T* g, int* err) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nch = (ne + kEditChunk - 1) / kEditChunk;
  if (c >= nch) return;
  const unsigned long long* t = (const unsigned long long*)(table + 16 * c);
  int64_t pos = (int64_t)t[0];
  int64_t prev = t[1] == ~0ull ? -1 : (int64_t)t[1];
  const int64_t cnt = (ne - c * kEditChunk) < kEditChunk ? ne - c * kEditChunk : kEditChunk;
  for (int64_t e = 0; e < cnt; ++e) {
    unsigned long long v[2];
    for (int w = 0; w < 2; ++w) {
      unsigned long long x = 0;
      int shift = 0;
      for (;;) {
        if (pos >= payload_bytes || shift > 63) {
          *err = 1;
          return;
        }
        const uint8_t b = payload[pos++];
        x |= (unsigned long long)(b & 0x7f) << shift;
        shift += 7;
        if (!(b & 0x80)) break;
      }
      v[w] = x;
    }
    const int64_t i = prev + 1 + (int64_t)v[0];
    if (v[0] >= (unsigned long long)n || i >= n || v[1] == 0) {
      *err = 1;
      return;
    }
    T out;
    from_order_key(order_key(g[i]) - v[1], &out);
    g[i] = out;
    prev = i;
  }
}

// ---- host side -------------------------------------------------------------------
struct EditLayout {
  size_t counts, base, sums, total, idx, len, off, bytes;
  int64_t nblocks, nscan;
};

static size_t al256(size_t v) { return (v + 255) / 256 * 256; }

static EditLayout edit_layout(int64_t n, int64_t cap) {
  EditLayout L;
  L.nblocks = (n + kCountItems - 1) / kCountItems;
  const int64_t items = cap > L.nblocks ? cap : L.nblocks;
  L.nscan = (items + kScanItems - 1) / kScanItems;
  L.counts = 0;
  L.base = L.counts + al256(4 * (size_t)L.nblocks);
  L.sums = L.base + al256(8 * (size_t)L.nblocks);
  L.total = L.sums + al256(8 * (size_t)L.nscan);
  L.idx = L.total + 256;
  L.len = L.idx + al256(4 * (size_t)(cap > 0 ? cap : 1));
  L.off = L.len + al256(4 * (size_t)(cap > 0 ? cap : 1));
  L.bytes = L.off + al256(8 * (size_t)(cap > 0 ? cap : 1));
  return L;
}

size_t edits_workspace_bytes(int64_t n, int64_t cap) { return edit_layout(n, cap).bytes; }

size_t edits_stream_bytes(int64_t ne) {
  const int64_t nch = (ne + kEditChunk - 1) / kEditChunk;
  return 40 + 16 * (size_t)nch + 15 * (size_t)ne;
}

static hipError_t scan_u32(const uint32_t* in, int64_t n, unsigned long long* sums,
                           unsigned long long* total, unsigned long long* out, hipStream_t s) {
  const int64_t nb = (n + kScanItems - 1) / kScanItems;
  if (nb < 1) return hipSuccess;
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, s, in, n, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, sums, nb, total);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, in, n,
                     (const unsigned long long*)sums, out);
  return hipGetLastError();
}

// Returns 0, or 1 when the edits exceed cap (*ne set), or 2 when the stream
// does not fit out_cap (*nbytes set); hip errors through *herr.
template <class T>
static int encode_t(const T* fhat, const T* g, int64_t n, int64_t cap, char* ws, uint8_t* out,
                    size_t out_cap, int64_t* ne_out, int64_t* nbytes_out, hipError_t* herr,
                    hipStream_t s) {
  const EditLayout L = edit_layout(n, cap);
  uint32_t* counts = (uint32_t*)(ws + L.counts);
  unsigned long long* base = (unsigned long long*)(ws + L.base);
  unsigned long long* sums = (unsigned long long*)(ws + L.sums);
  unsigned long long* total = (unsigned long long*)(ws + L.total);
  uint32_t* idx = (uint32_t*)(ws + L.idx);
  uint32_t* len = (uint32_t*)(ws + L.len);
  unsigned long long* off = (unsigned long long*)(ws + L.off);
  *herr = hipSuccess;
#define EDIT_TRY(x)                        \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) {                \
      *herr = e_;                          \
      return -1;                           \
    }                                      \
  } while (0)
  if (L.nblocks > 0) {
    hipLaunchKernelGGL(k_edit_count<T>, dim3((unsigned)L.nblocks), dim3(256), 0, s, fhat, g, n,
                       counts);
    EDIT_TRY(hipGetLastError());
    EDIT_TRY(scan_u32(counts, L.nblocks, sums, total, base, s));
  }
  unsigned long long ne = 0;
  EDIT_TRY(hipMemcpyAsync(&ne, total, 8, hipMemcpyDeviceToHost, s));
  EDIT_TRY(hipStreamSynchronize(s));
  if (L.nblocks == 0) ne = 0;
  *ne_out = (int64_t)ne;
  if ((int64_t)ne > cap) return 1;
  unsigned long long nb = 0;
  if (ne > 0) {
    hipLaunchKernelGGL(k_edit_compact<T>, dim3((unsigned)L.nblocks), dim3(256), 0, s, fhat, g,
                       n, (const unsigned long long*)base, idx, cap);
    EDIT_TRY(hipGetLastError());
    const unsigned grid = (unsigned)((ne + 255) / 256);
    hipLaunchKernelGGL(k_edit_sizes<T>, dim3(grid), dim3(256), 0, s, fhat, g,
                       (const uint32_t*)idx, (int64_t)ne, len);
    EDIT_TRY(hipGetLastError());
    EDIT_TRY(scan_u32(len, (int64_t)ne, sums, total, off, s));
    EDIT_TRY(hipMemcpyAsync(&nb, total, 8, hipMemcpyDeviceToHost, s));
    EDIT_TRY(hipStreamSynchronize(s));
  }
  const int64_t nch = ((int64_t)ne + kEditChunk - 1) / kEditChunk;
  const size_t head = 40 + 16 * (size_t)nch;
  *nbytes_out = (int64_t)(head + nb);
  if (head + nb > out_cap) return 2;
  unsigned char h[40];
  memcpy(h, "PMSE", 4);
  h[4] = 1;
  h[5] = sizeof(T) == 8 ? 1 : 0;
  h[6] = h[7] = 0;
  const unsigned long long nv = (unsigned long long)n;
  const uint32_t chunk = kEditChunk, chunks = (uint32_t)nch;
  memcpy(h + 8, &nv, 8);
  memcpy(h + 16, &ne, 8);
  memcpy(h + 24, &nb, 8);
  memcpy(h + 32, &chunk, 4);
  memcpy(h + 36, &chunks, 4);
  EDIT_TRY(hipMemcpyAsync(out, h, 40, hipMemcpyHostToDevice, s));
  if (ne > 0) {
    const unsigned grid = (unsigned)((ne + 255) / 256);
    hipLaunchKernelGGL(k_edit_write<T>, dim3(grid), dim3(256), 0, s, fhat, g,
                       (const uint32_t*)idx, (int64_t)ne, (const unsigned long long*)off,
                       out + 40, out + head);
    EDIT_TRY(hipGetLastError());
  }
  EDIT_TRY(hipStreamSynchronize(s));  // the header copy reads host memory
#undef EDIT_TRY
  return 0;
}

int edits_encode(int dtype, const void* fhat, const void* g, int64_t n, int64_t cap, void* ws,
                 uint8_t* out, size_t out_cap, int64_t* ne, int64_t* nbytes, hipError_t* herr,
                 hipStream_t s) {
  if (dtype == PMSZ_F32)
    return encode_t<float>((const float*)fhat, (const float*)g, n, cap, (char*)ws, out, out_cap,
                           ne, nbytes, herr, s);
  return encode_t<double>((const double*)fhat, (const double*)g, n, cap, (char*)ws, out, out_cap,
                          ne, nbytes, herr, s);
}

hipError_t edits_decode(int dtype, const uint8_t* table, const uint8_t* payload,
                        int64_t payload_bytes, int64_t ne, int64_t n, void* g, int* err,
                        hipStream_t s) {
  const int64_t nch = (ne + kEditChunk - 1) / kEditChunk;
  if (nch == 0) return hipSuccess;
  const unsigned grid = (unsigned)((nch + 255) / 256);
  if (dtype == PMSZ_F32)
    hipLaunchKernelGGL(k_edit_decode<float>, dim3(grid), dim3(256), 0, s, table, payload,
                       payload_bytes, ne, n, (float*)g, err);
  else
    hipLaunchKernelGGL(k_edit_decode<double>, dim3(grid), dim3(256), 0, s, table, payload,
                       payload_bytes, ne, n, (double*)g, err);
  return hipGetLastError();
}

}  // namespace pmsz
