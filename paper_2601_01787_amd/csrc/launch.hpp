// launch.hpp -- host-side launchers of the libpmsz kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace pmsz {

struct Geo {
  int ndim;
  int64_t nx, ny, nz, sxy, n;
};

inline Geo make_geo(const pmsz_grid& g) {
  Geo G;
  G.ndim = g.ndim;
  G.nx = g.nx;
  G.ny = g.ny;
  G.nz = g.nz;
  G.sxy = g.nx * g.ny;
  G.n = G.sxy * g.nz;
  return G;
}

inline int64_t bitmap_words(int64_t n) { return (n + 31) / 32; }

// stencil.hip
hipError_t launch_dirs(int dtype, const void* h, const Geo& G, uint8_t* dirs, hipStream_t s);

// labels.hip
// Pointer jumping: each pass follows up to kLabelHops links per vertex;
// passes are queued kLabelBatch at a time between read-backs of their
// changed flags, at most kLabelMaxPasses per label array.
constexpr int kLabelHops = 8;
constexpr int kLabelBatch = 8;
constexpr int kLabelMaxPasses = 64;
// Labels workspace: [bad-code counter (8 bytes), padded to 256][changed flag
// per pass (kLabelMaxPasses words)].
constexpr size_t kLabelsWsBytes = 256 + 4 * kLabelMaxPasses;
hipError_t launch_check_dirs(const uint8_t* dirs, const Geo& G, unsigned long long* bad,
                             hipStream_t s);
hipError_t launch_labels_init(const uint8_t* dirs, const Geo& G, int32_t* lmax, int32_t* lmin,
                              unsigned long long* bad, hipStream_t s);
hipError_t launch_labels_jump(int32_t* lab, int64_t n, const uint8_t* dirs, int shift,
                              unsigned int* flags, unsigned long long* bad, int pass,
                              hipStream_t s);

// verify.hip
struct VerifyCounts {
  unsigned long long c[11];  // bound, asc, desc, fmax, fmin, mmax, mmin, wmax, wmin, wany, edited
  unsigned long long max_err_bits;
};
hipError_t launch_verify(int dtype, const void* f, const void* g, const void* fhat, int64_t n,
                         double xi_t, const uint8_t* df, const uint8_t* dg, const int32_t* lf_max,
                         const int32_t* lf_min, const int32_t* lg_max, const int32_t* lg_min,
                         VerifyCounts* out, hipStream_t s);

// blocks.hip: one block of a decomposed domain as the exchange sees it --
// the origin of its copy in the global grid, the copy's x and y extents and
// the copy's values (dense, x fastest).
struct BlockCopy {
  int64_t ox, oy, oz;
  int64_t lnx, lny;
  void* g;
};
hipError_t blocks_gather(int dtype, const void* src, const Geo& G, const int64_t o[3],
                         const int64_t l[3], void* dst, hipStream_t s);
hipError_t blocks_scatter_core(int dtype, const void* src, const int64_t l[3], const int64_t c[6],
                               const int64_t o[3], void* dst, const Geo& G, hipStream_t s);
hipError_t blocks_exchange(int dtype, void* g, const Geo& G, const int32_t nb[3],
                           const BlockCopy* tab, const int32_t* hold, const int32_t* planes,
                           int32_t n_planes, int64_t max_plane, unsigned long long* lowered,
                           hipStream_t s);

// edits.hip
size_t edits_workspace_bytes(int64_t n, int64_t cap);
size_t edits_stream_bytes(int64_t ne);
int edits_encode(int dtype, const void* fhat, const void* g, int64_t n, int64_t cap, void* ws,
                 uint8_t* out, size_t out_cap, int64_t* ne, int64_t* nbytes, hipError_t* herr,
                 hipStream_t s);
hipError_t edits_decode(int dtype, const uint8_t* table, const uint8_t* payload,
                        int64_t payload_bytes, int64_t ne, int64_t n, void* g, int* err,
                        hipStream_t s);

// Counter-calibration probe (probe.hip): reads `bytes` bytes of p once, as
// dword rows (pattern 0) or byte rows (pattern 1), adding their sum to *out.
hipError_t launch_probe_read(const void* p, int64_t bytes, int pattern, unsigned long long* out,
                             hipStream_t s);

}  // namespace pmsz
