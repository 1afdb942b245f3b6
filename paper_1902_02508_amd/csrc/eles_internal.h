// Internal declarations of the filter library: launch parameters shared by
// the host orchestration (eles_host.hip) and the kernel sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace eles {

constexpr int kXzThreads = 256;   // x/z pass block size (one column per thread)
constexpr int kXzTileX = 8;       // x outputs per x/z tile
constexpr int kXzRunZ = 4;        // z outputs per item of the z stage (one 16-byte store)
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

// Length of a zero-padded FP32 tap array of half-width m: entry e holds the
// tap of offset e - (kXzTileX - 1) - m, zero outside [kXzTileX - 1,
// kXzTileX - 1 + 2m]; the tail covers the widest window a stencil group
// reads (the z stage fetches 40 entries at a time).
__host__ __device__ inline int tap_pad_len(int m) { return 2 * m + 2 * kXzTileX + 40; }

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

// Stress x/z pass on the matrix cores, k_xzm.hip: persistent blocks, each
// taking an equal contiguous range of the z tiles of all (y, x group) rows;
// the waves of a block take the group's neighbouring 16-row x tiles.
constexpr int kXzmWaves = 4;   // waves per block of the matrix-core x/z pass
struct XzmPlan {
  int wide;   // 0: k_xzm (nine fields a wave); 1: k_xzw (three fields a wave)
  int ks;     // x stencil steps of four input rows (covers 16 + 2 mx rows)
  int h;      // z chunks on each side of a tile (covers mz)
  int vec;    // nz % 4 == 0: 16-byte stores
  int nxt;    // 16-row x tiles
  int nxg;    // k_xzm: groups of kXzmWaves x tiles (one per wave of a block);
              // k_xzw: block rows of kXzmWaves (x tile, field group) items
  int nct;    // 16-column z tiles
  int nrow;   // rows: ny * nxg
  int nblk;   // blocks of kXzmWaves waves
};
// False when the grid is outside what the kernel covers (the VALU kernel
// k_xz then runs instead).
bool xzm_plan(int nx, int ny, int nz, int mx, int mz, XzmPlan *p);
hipError_t launch_xzm(const XzArgs &a, const XzmPlan &p, hipStream_t s);

// Wide stencils (k_xzw.hip): x half-width up to 44, z up to 48, nz % 4 == 0.
// Each wave carries one group of three of the nine fields for one 16-row x
// tile; a block's four waves take four consecutive (x tile, group) items.
constexpr int kXzwMaxSteps = 26;   // x stencil steps of four rows
constexpr int kXzwMaxHalo = 3;     // z chunks on each side of a tile
bool xzw_plan(int nx, int ny, int nz, int mx, int mz, XzmPlan *p);
hipError_t launch_xzw(const XzArgs &a, const XzmPlan &p, hipStream_t s);

// y pass, k_y.hip.
struct YArgs {
  // element (x, k, z) of input field f sits at in[f*in_fs + x*in_xs + k*in_ks + z];
  // the stress mode reads the row-interleaved x/z-pass output
  const float *in;
  size_t in_fs, in_xs, in_ks;
  float *ubar, *tau;      // sgs outputs, planar [3][nx][ny][nz] / [6][...]
  float *out;             // plain outputs, element (x, i, z) of field f at
  size_t out_fs, out_xs, out_ks;   // out[f*out_fs + x*out_xs + i*out_ks + z]
  double *part;           // sgs plane partials [9][ny][parts] or null
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

// Stress y pass staged through LDS, k_ys.hip: persistent blocks, each
// keeping one group of consecutive 16-row output tiles (band rows
// [kb, kb + nrow)) and walking the (x, 16-column strip) pencils.
constexpr int kYsRow = 9 * kYTileN + 4;   // floats per staged row (9 fields x 16, + bank pad)
constexpr int kYsMaxTiles = 3;            // tiles per group
constexpr int kYsMaxGroups = 32;
constexpr int kYsMaxChunks = 384;         // chunk table entries over all groups
constexpr int kYsMaxGroupChunks = 24;     // chunks of one group (the walk is unrolled to this)
constexpr size_t kYsLdsMax = 163840;
struct YsPlan {
  int nblk;                               // persistent grid: a multiple of ngroup
  int ngroup;
  int lds_rows;                           // staged rows allocated per block
  int max_chunks;                         // most 16-column chunks of one group
  int tile0[kYsMaxGroups], ntile[kYsMaxGroups], kb[kYsMaxGroups], nrow[kYsMaxGroups];
  int chunk0[kYsMaxGroups], nchunk[kYsMaxGroups];
  // per chunk of a group, in walk order: first column | tile in group << 16
  // | (last chunk of its tile) << 24
  int chunk[kYsMaxChunks];
};
size_t ys_lds_bytes(const YsPlan &p);
int ys_grid(const YsPlan &p, int nz, int npencils);   // 0 if the kernel cannot run
hipError_t launch_ys(const YArgs &a, const YsPlan &p, hipStream_t s);
hipError_t launch_stats(const double *part, double *stats, int ny, int nparts,
                        double inv_count, hipStream_t s);

// ---- closure features: gradient operators of the grid (filter state)

// Spectral derivative along a periodic axis by fast transforms (k_sder.hip):
// the radices of n (16, 8, 4, 2, 3, 5; nrad = 0 when n has another prime
// factor or the lines do not fit a block, and the dense operator is used),
// P complex lines per block, division magics ceil(2^32 / d) of the pass
// geometry, the factor 2 pi / (L n) and the table exp(-2 pi i m / n).
constexpr int kSderMaxPass = 8;
struct SderAxis {
  int n, P, lp, E, T, nrad;      // E complex values per thread, T threads per block
  int rad[kSderMaxPass];
  uint32_t mnr[kSderMaxPass];    // of n / rad[s]
  uint32_t mns[kSderMaxPass];    // of the forward pass's Ns
  uint32_t imns[kSderMaxPass];   // of the inverse pass's Ns (radices reversed)
  float cfac;
  float2 *tw;                    // [n] in the filter state
};
struct SderArgs {
  SderAxis ax;
  const float *in;
  float *out;
  long in_fs, out_fs;
  int nx, ny, nz, zaxis;
  // z lines only: also d/dy of the three fields into dy + f * out_fs, the
  // three-point rows of D[parity] (row pitch kp; parity bit f of pmask), or
  // dy null
  float *dy;
  const float *D[2];
  int kp;
  unsigned pmask;
};
bool sder_plan(int n, double length, bool zaxis, SderAxis *a);
// Real forward / inverse transforms along x or z of nf fields in the folded
// layout of the differential filter (k_sder.hip): cosine k at position k,
// sine k at n/2 + k. prod: the x forward of the stress forms field f of the
// nine from u [3][...] (u1 shifted by prof[y]).
struct RfftArgs {
  SderAxis ax;
  const float *in;
  float *out;
  const float *prof;
  long in_fs, out_fs;
  int nx, ny, nz, nf, prod;
  unsigned zmask;   // x inverse: fields (bit f) whose wall rows are zero
};
hipError_t rfft_setup(const SderAxis &a, hipStream_t s);
hipError_t launch_rfft(const SderAxis &a, bool zaxis, bool inverse, const float *in, float *out, const float *prof,
                       long in_fs, long out_fs, int nx, int ny, int nz, int nf, bool prod, unsigned zmask,
                       hipStream_t s);
size_t sder_lds_bytes(const SderAxis &a);

struct GradView {
  int nx, ny, nz, mpx, kpx, mpz, kpz, mpy, kpy;
  double lx, lz;
  float *dx32;                 // spectral x derivative, padded [mpx][kpx]
  uint16_t *dxhi, *dxlo;
  int *dxband;                 // [mpx][2]
  uint16_t *dzhi, *dzlo;       // spectral z derivative, padded [mpz][kpz]
  float *dy32[2];              // y derivative of even / odd fields [mpy][kpy]
  uint16_t *dyhi[2], *dylo[2];
  int *dyband;                 // [mpy][2]
  SderAxis sx, sz;             // fast spectral derivatives along x and z
};
hipError_t launch_build_grad_ops(const GradView &v, const double *y64, hipStream_t s);
hipError_t launch_dz(const GradView &v, const float *ubar, float *out, long out_fstride, hipStream_t s);
// d/dy of the three fields at ubar (parities in pmask, bit f: odd) into
// out + f * out_fstride; needs ny >= 3
hipError_t launch_ddy(const GradView &v, const float *ubar, float *out, long out_fstride, unsigned pmask,
                      hipStream_t s);
// tables and LDS limit of the fast spectral derivatives
hipError_t sder_setup(const SderAxis &a, hipStream_t s);
// d/dx (zaxis false) or d/dz of the three fields at ubar into
// out + f * out_fstride by fast transforms; needs the axis's nrad > 0
hipError_t launch_sder(const GradView &v, bool zaxis, const float *ubar, float *out, long out_fstride,
                       hipStream_t s);
// d/dz as launch_sder, with d/dy of the three fields (odd fields in pmask)
// into dy + f * out_fstride from the same staged rows; needs ny >= 3
hipError_t launch_sder_zy(const GradView &v, const float *ubar, float *out, float *dy, long out_fstride,
                          unsigned pmask, hipStream_t s);
bool sder_zy_ok(const GradView &v);   // the fused kernel covers this grid
hipError_t launch_walldist(const double *y64, int nx, int ny, int nz, float *out, hipStream_t s);

// ---- the perceptron
constexpr int kMlpIn = 10, kMlpHidden = 64, kMlpOut = 6, kMlpInPad = 32;
constexpr int kMlpNParam = 10 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 * 6 + 6;
constexpr int kMlpOffB1 = 640, kMlpOffB2 = 640 + 64 + 4096, kMlpOffB3 = kMlpOffB2 + 64 + 4096,
              kMlpOffB4 = kMlpOffB3 + 64 + 384;
constexpr int kMlpChunk = 512;   // batch rows per split-K chunk of a weight gradient

struct ClosureView {
  float *theta, *m, *v;                         // FP32 master weights and Adam moments
  uint16_t *w1, *w2, *w3, *w4, *w2t, *w3t, *w4t;  // padded BF16 shadows
  const float *fsc, *fsh;                       // standardised feature = f * fsc + fsh
  const float *tsc, *tsh;                       // standardised target  = t * tsc + tsh
  const float *isc, *ish;                       // target = y * isc + ish
  // gradient-model term added to the prediction: G_ij = sum_k gmc[k]
  // g_ik g_jk over the raw features g_ik = feat[3 i + k]; gmc = 0 (and
  // use_gm = 0) leaves the plain network
  float gmc[3];
  int use_gm;
};
struct TrainData {
  const float *feat, *tau;   // [nsnap][10][npts], [nsnap][6][npts]
  int nsnap;
  long npts;
};
struct TrainWs {
  uint16_t *x0, *x0t;
  float *tb;
  uint16_t *h[3], *ht[3], *g[3], *dy, *dyt, *dz[3], *dzt[3];
  float *pw[4], *pb[4];
  double *lossp;
};
struct AdamArgs {
  float lr, b1, b2, eps, bc1, bc2;
  float *loss_out;
  const double *lossp;
  int nloss;
  long batch;
  int nchunks;
  const float *pw[4];
  const float *pb[4];
  int mrows[4], ncols[4];
};
hipError_t launch_sample(uint64_t seed, long step, int batch, uint64_t count, int64_t *out, hipStream_t s);
hipError_t launch_shadows(const ClosureView &c, hipStream_t s);
// the closure on features 0..8 of feat [10][nx ny nz] (the wall distance is
// taken from y64) into out [6][...]; with rows, the FP64 sums of each
// output over every (x, y) row into rows [6][nx ny]
hipError_t launch_infer(const ClosureView &c, const float *feat, int nx, int ny, int nz, const double *y64,
                        float *out, double *rows, hipStream_t s);
hipError_t launch_moments(const float *data, int nchan, int nsnap, long npts, double *part, int nchunks,
                          double *out, hipStream_t s);
// Plane means and the non-finite test (k_check.hip, built with IEEE
// semantics). part: FP64 scratch of plane_mean_parts(nq, ny) values.
inline long plane_mean_parts(int nq, int ny) { return (long)nq * ny * 16; }
// plane means out [nq][ny] from the row sums of launch_infer
hipError_t launch_row_means(const double *rows, int nq, int nx, int ny, int nz, double *out, hipStream_t s);
hipError_t launch_plane_mean(const float *f, int nq, int nx, int ny, int nz, double *part, double *out,
                             hipStream_t s);
// *flag (device) = 1 if any of v[0..n) (device FP64) is NaN or infinite.
hipError_t launch_nonfinite(const double *v, int n, int *flag, hipStream_t s);
hipError_t launch_train_step(const ClosureView &c, const TrainData &d, const TrainWs &w, uint64_t seed, long step,
                             int batch, AdamArgs adam, hipStream_t s);

// Differential filter (k_dfilt.hip): folded real Fourier transforms along
// x and z on the matrix cores, tridiagonal solves in y.
constexpr int kDFields = 9;   // fields filtered for the stress
constexpr int kDTS = 7;       // forward transform: 16-row coefficient tiles per wave
constexpr int kDTI = 4;       // inverse transform: 16-node output tiles per wave
constexpr int kDNT = 2;       // 16-wide data tiles per wave
// One periodic axis of n nodes in the folded real basis: cosines 0 .. h,
// sines 1 .. hs; the contraction runs over the index 1 .. h (folded node,
// or coefficient) in ks steps of four (ks4 groups of four steps), the
// index-0 term being added separately; qc cosine and qs sine tiles; gf
// forward tile groups per data tile (gc of them cosine, the rest sine) and
// gi inverse ones.
struct DAxis {
  int n, h, hs, ks, ks4, qc, qs, gf, gc, gi;
};
constexpr int kDMinN = 8;     // fewest nodes of a periodic axis
inline DAxis daxis(int n) {
  DAxis a;
  a.n = n;
  a.h = n / 2;
  a.hs = (n - 1) / 2;
  a.ks = (a.h + 3) / 4;
  a.ks4 = (a.ks + 3) / 4;
  a.qc = (a.h + 1 + 15) / 16;
  a.qs = (a.hs + 15) / 16;
  a.gc = (a.qc + kDTS - 1) / kDTS;
  a.gf = a.gc + (a.qs + kDTS - 1) / kDTS;
  a.gi = (a.qc + kDTI - 1) / kDTI;
  return a;
}
// floats of the pre-arranged forward and inverse tables of an axis
inline size_t dtab_fwd_floats(const DAxis &a) { return (size_t)a.gf * kDTS * a.ks4 * 256; }
inline size_t dtab_inv_floats(const DAxis &a) { return (size_t)2 * a.gi * kDTI * a.ks4 * 256; }
struct DView {
  int nx, ny, nz;
  int hx, hz;                   // nx / 2, nz / 2: wavenumber indices 0 .. h
  DAxis ax, az;
  double lx, lz, a;
  double *y64;                  // [ny]
  double *d64;                  // [even, odd][sub, main, super][ny] second difference
  double *p64;                  // [3][ny] sub-diagonal, 1/den, c' of the zero-wavenumber even system
  double *scratch64;            // [3][ny]
  float *fx, *ix, *fz, *iz;     // forward and inverse tables of x and z
  float *lo32;                  // [2][ny] system sub-diagonal -a^2 sub
  float *op32;                  // [2][3][ny] -a^2 (sub, main, super) of the y difference
  float *cp, *inv;              // [2][hx + 1][ny][hz + 1] elimination factors
  float *prof;                  // [3][ny] m, M = F(m), F(m^2) - M^2
  size_t ldsmax;                // largest table slice the LDS kernels may stage (bytes)
  SderAxis rx, rz;              // fast transforms along x and z (nrad 0: the table products)
};
hipError_t dfilter_lds_limit(DView &v);   // sets v.ldsmax for the current device
hipError_t launch_dsetup(const DView &v, hipStream_t s);
// timed passes (ev: 2 events per pass, or null)
enum { kDPassShift, kDPassXf, kDPassZf, kDPassY, kDPassZi, kDPassXi, kDPassEpi, kDPasses };
hipError_t launch_dfilter(const DView &v, const float *in, int nf, unsigned pmask, float *w0, float *w1, float *out,
                          hipStream_t s, const hipEvent_t *ev);
hipError_t launch_dsgs(const DView &v, const float *u, float *w0, float *w1, float *ubar, float *tau,
                       double *part, double *stats, hipStream_t s, const hipEvent_t *ev);
// the inverse filter u = (1 - a^2 lap) ubar with the same discretisation
hipError_t launch_dinverse(const DView &v, const float *in, int nf, unsigned pmask, float *w0, float *w1,
                           float *out, hipStream_t s, const hipEvent_t *ev);
// eq. (13)-(15) errors of les against dns ([3][nx][ny][nz] each) into
// out[5] (FP64, device); part: derr_parts doubles
hipError_t launch_derrors(const DView &v, const float *les, const float *dns, double utau_les, double utau_dns,
                          double *part, double *out, hipStream_t s);
long derr_parts(const DView &v);
long dsgs_parts(const DView &v);   // doubles of the statistics scratch of launch_dsgs

// LES-grid stress and commutation error (k_les.hip).
struct LesView {
  int nx, ny, nz;               // DNS grid
  int nxl, nyl, nzl;            // LES grid
  const int *ix, *iy, *iz;      // lower DNS node of every LES node, per direction
  const float *wx, *wy, *wz;    // weight of the upper DNS node
  const int *db;                // DNS y derivative: first node of the stencil of node j
  const double *dc;             //   its three coefficients [ny][3]
  const int *lb;                // LES y derivative, the same
  const double *lc;             //   [nyl][3]
  const double *lw;             // LES y trapezoid weights [nyl]
};
hipError_t launch_les_stress(const LesView &v, const float *ubar, const float *tau, float *ul, float *T,
                             hipStream_t s);
long les_comm_parts(const LesView &v);   // doubles of the commutation-error scratch
hipError_t launch_les_commutation(const LesView &v, const float *g, double *part, double *out, hipStream_t s);

}  // namespace eles
