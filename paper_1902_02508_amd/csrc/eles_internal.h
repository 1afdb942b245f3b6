// Internal declarations of the filter library: launch parameters shared by
// the host orchestration (eles_host.hip) and the kernel sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace eles {

constexpr int kXzThreads = 256;   // x/z pass block size (one column per thread)
constexpr int kXzTileX = 8;       // x outputs per x/z tile
constexpr int kXzRunZ = 8;        // z outputs per thread in the z stage
constexpr int kXzRowPad = 16;     // LDS row padding of the x-filtered tile
constexpr int kMaxHalfX = 128;    // largest x stencil half-width
constexpr int kMaxHalfZ = 120;    // largest z stencil half-width: 2m + 8 <= 256
constexpr int kYBlockM = 16;      // rows of one y-pass output tile
constexpr int kYTileN = 16;       // columns (z) of one wave's y-pass tile
constexpr int kYWaves = 4;        // waves per y-pass block
constexpr int kKAlign = 32;       // column padding of the y operators
constexpr int kMeanSlabs = 8;     // x-slabs sampled for the shift profile

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical tiles so neighbouring tiles share its L2.
__device__ inline int xcd_remap(int b, int nb) {
  const int per = nb / 8, rem = nb % 8;
  const int xcd = b % 8, local = b / 8;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Length of a zero-padded FP32 tap array of half-width m.
__host__ __device__ inline int tap_pad_len(int m) { return 2 * m + 2 * kXzTileX + 8; }

// Operators resident in the caller's state buffer.
struct OpsView {
  int nx, ny, nz, mx, mz, mpad, kpad;
  double lx, lz, dx, dy, dz, tau;
  double *y64, *wp64, *wm64, *wx64, *wz64, *shift64;
  float *wx32, *wz32;     // padded taps, tap_pad_len(m) entries
  float *a32[4];          // W^+, W^-, C^+, C^-  [mpad][kpad]
  uint16_t *ahi[4], *alo[4];
  int *rowband;           // [mpad][2]: first and one-past-last nonzero column
  float *prof32;          // [3][mpad]: m, M = W^+ m, s = W^+ m^2 - M^2
};

// Operator build (FP64), k_ops.hip.
hipError_t launch_build_ops(const OpsView &v, hipStream_t s);
hipError_t launch_shift_ops(const OpsView &v, const float *u1, hipStream_t s);

// x/z pass, k_xz.hip. sgs: 3 velocity components -> 9 fields (u1 shifted by
// prof32[0]); otherwise ncomp (<= 3) independent fields.
struct XzArgs {
  const float *in;
  size_t in_stride;    // elements between input components
  float *out;          // fields interleaved by row: [nx][ny][out_nf][nz]
  int out_nf;
  const float *wx, *wz, *mshift;
  int nx, ny, nz, mx, mz, zt, nzt, nxt, ncomp;
};
hipError_t launch_xz(const XzArgs &a, bool sgs, hipStream_t s);
int xz_tile_z(int nz, int mz);

// y pass, k_y.hip.
struct YArgs {
  const float *in;        // x/z-filtered fields, [nx][ny][in_nf][nz]
  int in_nf;
  float *ubar, *tau;      // sgs outputs
  float *out;             // plain outputs
  size_t out_stride;
  double *part;           // sgs plane partials [9][ny][y_parts()] or null
  const float *a32[4];
  const uint16_t *ahi[4], *alo[4];
  const int *rowband;
  const float *prof32;
  int nx, ny, nz, mpad, kpad, n16, nfield;
  uint32_t parity_mask;   // plain: bit f set = field f odd
};
hipError_t launch_y(const YArgs &a, bool sgs, int prec, hipStream_t s);
// Number of plane partials per (quantity, row) the stress y pass writes.
inline int y_parts(int nx, int n16) { return nx * ((n16 + kYWaves - 1) / kYWaves); }
hipError_t launch_stats(const double *part, double *stats, int ny, int nparts,
                        double inv_count, hipStream_t s);

}  // namespace eles
