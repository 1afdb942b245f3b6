// x/z pass: the periodic part of the separable filter of eq. (2).
//
// One block owns one wall-normal plane y, eight consecutive x rows and a
// strip of zt columns in z. Stage X: each thread owns one z column of the
// strip plus its periodic halo, streams the kXzTileX + 2 mx input rows that
// the eight outputs need straight from HBM (lanes along z, so every wave
// load is one contiguous segment), forms the fields in registers and keeps
// eight x-filtered outputs per field in registers. In the stress mode the
// fields are u1' = u1 - m(y), u2, u3 and their six products, so the raw
// velocity is read once and the products are never stored. The x-filtered
// strip goes to LDS. Stage Z: each thread takes runs of four z outputs of
// one (field, x) row and applies the z stencil from LDS, writing each run
// as one 16-byte store, so four neighbouring lanes fill a whole 64-byte
// segment (runs of eight as eight 4-byte stores cost four times the L2
// write requests). The nine outputs are interleaved by row, [x][y][f][z],
// so the y pass finds all fields of one (x, y) row side by side.
//
// Taps are read through uniform (scalar) loads from zero-padded tap arrays,
// so the per-output loops carry no bounds tests; each group of four inputs
// fetches its eleven taps at once.
#include "eles_internal.h"

namespace eles {
namespace {

constexpr int XT = kXzTileX;
constexpr int RZ = kXzRunZ;
constexpr int kZGroups = 8;  // z-stage input groups fetched at once
static_assert(RZ == 4, "the z stage stores runs of four");

__device__ inline int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

template <bool SGS>
struct Fields;

template <>
struct Fields<true> {
  static constexpr int NF = 9;
  __device__ static inline void form(const float (&c)[3], float (&v)[9]) {
    v[0] = c[0];
    v[1] = c[1];
    v[2] = c[2];
    v[3] = c[0] * c[0];
    v[4] = c[0] * c[1];
    v[5] = c[0] * c[2];
    v[6] = c[1] * c[1];
    v[7] = c[1] * c[2];
    v[8] = c[2] * c[2];
  }
};

template <>
struct Fields<false> {
  static constexpr int NF = 3;
  __device__ static inline void form(const float (&c)[3], float (&v)[3]) {
    v[0] = c[0];
    v[1] = c[1];
    v[2] = c[2];
  }
};

// Row-group modes of the streaming stencil loops. A group is four
// consecutive input rows r0..r0+3 feeding XT outputs o through tap r - o.
enum { G_HEAD = 0, G_FULL = 1, G_ANY = 2 };

// Does input row r reach output o through a kept tap (0 <= r - o <= m2)?
// HEAD groups start at a compile-time row below XT and never pass the far
// end (m2 >= 8); FULL groups are inside the band for every o. Groups past
// the band's far end also run as FULL: the padded tap arrays are zero
// beyond offset m2, which costs a few multiplications by zero instead of a
// branch per (row, output) pair. ANY tests both ends (narrow stencils).
template <int MODE>
__device__ inline bool reach(int r, int o, int m2) {
  if (MODE == G_HEAD) return o <= r;
  if (MODE == G_FULL) return true;
  return o <= r && r - o <= m2;
}

// The taps a group of four inputs b..b+3 and eight outputs uses: entries
// b .. b+10 of the padded tap array (input b+k reaches output o through
// entry b + k + 7 - o). b is a multiple of 4, so the window is three
// aligned 16-byte uniform loads, one wait per group instead of one per tap.
__device__ inline void tap_window(const float *__restrict__ w, int b, float (&t)[12]) {
  const float4 *p = reinterpret_cast<const float4 *>(w + b);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float4 q = p[i];
    t[4 * i] = q.x;
    t[4 * i + 1] = q.y;
    t[4 * i + 2] = q.z;
    t[4 * i + 3] = q.w;
  }
}

template <bool SGS, int MODE, int R0>
__device__ inline void x_group(float (&acc)[Fields<SGS>::NF][XT], const float (&cur)[4][3], float ms,
                               const float *__restrict__ wx, int r0, int m2) {
  constexpr int NF = Fields<SGS>::NF;
  const int rb = MODE == G_HEAD ? R0 : r0;
  float tw[12];
  tap_window(wx, rb, tw);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float c3[3] = {cur[k][0] - ms, cur[k][1], cur[k][2]};
    float v[NF];
    Fields<SGS>::form(c3, v);
    const int r = rb + k;
#pragma unroll
    for (int o = 0; o < XT; ++o) {
      if (!reach<MODE>(r, o, m2)) continue;
      const float wt = tw[k + XT - 1 - o];
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[f][o] = fmaf(wt, v[f], acc[f][o]);
    }
  }
}

// z stencil of one run of RZ = 4 outputs from its LDS row, kZGroups groups
// of four inputs at a time: the chunk's LDS values (one 16-byte read per
// group) and its 4 kZGroups + 8 taps (uniform 16-byte loads) are all
// requested before the first product, so a chunk waits once. Input t
// reaches output q through padded tap entry t + XT - 1 - q; entries past
// the stencil are zero, which also covers the first group's missing pairs
// and the groups past the row's end (they read a valid LDS address and
// meet only zero taps: their entries start at 4 ngz + XT - 4 > XT - 1 + 2m).
__device__ inline void z_run(float (&acc)[RZ], const float *src, const float *__restrict__ wz, int ngz) {
  for (int g0 = 0; g0 < ngz; g0 += kZGroups) {
    float4 v[kZGroups];
#pragma unroll
    for (int j = 0; j < kZGroups; ++j) {
      const int g = g0 + j < ngz ? g0 + j : ngz - 1;
      v[j] = *reinterpret_cast<const float4 *>(src + 4 * g);
    }
    float tw[4 * kZGroups + 8];
    {
      const float4 *p = reinterpret_cast<const float4 *>(wz + 4 * g0 + XT - RZ);
#pragma unroll
      for (int i = 0; i < kZGroups + 2; ++i) {
        const float4 q = p[i];
        tw[4 * i] = q.x;
        tw[4 * i + 1] = q.y;
        tw[4 * i + 2] = q.z;
        tw[4 * i + 3] = q.w;
      }
    }
    // every request above is issued before the first product (the fence
    // keeps the compiler from sinking the LDS reads to their uses)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < kZGroups; ++j) {
      const float vv[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < RZ; ++q) acc[q] = fmaf(tw[4 * j + k + RZ - 1 - q], vv[k], acc[q]);
    }
  }
}

template <bool SGS>
__global__ void __launch_bounds__(kXzThreads)
k_xz(XzArgs a, const float *__restrict__ gin, float *__restrict__ gout,
     const float *__restrict__ wx, const float *__restrict__ wz) {
  constexpr int NF = Fields<SGS>::NF;
  constexpr int NG = SGS ? 2 : 1;               // field groups staged through LDS
  constexpr int GF = (NF + NG - 1) / NG;        // fields per group
  extern __shared__ float tx[];                 // [GF][XT][zs]
  const int zh = a.zt + 2 * a.mz;
  const int zs = ((zh + 4 + 3) / 4) * 4;
  const int tid = threadIdx.x;
  const int mx2 = 2 * a.mx, mz2 = 2 * a.mz;

  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int xt = b % a.nxt;
  const int rest = b / a.nxt;
  const int ztile = rest % a.nzt;
  const int y = rest / a.nzt;
  const int x0 = xt * XT, z0 = ztile * a.zt;
  const size_t xstride = (size_t)a.ny * a.nz;

  // zero the row tails read by the last vector loads of stage Z
  for (int q = tid; q < GF * XT * (zs - zh); q += kXzThreads) {
    int row = q / (zs - zh), col = zh + q % (zs - zh);
    tx[row * zs + col] = 0.0f;
  }

  // ---- stage X: x-filtered values of every field for one column per thread
  float acc[NF][XT];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int o = 0; o < XT; ++o) acc[f][o] = 0.0f;
  if (tid < zh) {
    const int gz = wrap(z0 - a.mz + tid, a.nz);
    const float ms = SGS ? a.mshift[y] : 0.0f;
    const size_t plane = (size_t)y * a.nz + gz;
    // component bases; a missing component (plain mode, ncomp < 3) re-reads
    // the last one so that every load is unconditional
    const float *cb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) cb[c] = gin + (size_t)(c < a.ncomp ? c : a.ncomp - 1) * a.in_stride + plane;
    int gx = wrap(x0 - a.mx, a.nx);
    // rows arrive two groups ahead of their use
    float cur[4][3], nx1[4][3], nx2[4][3];
    auto load_group = [&](float (&dst)[4][3]) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const size_t off = (size_t)gx * xstride;
#pragma unroll
        for (int c = 0; c < 3; ++c) dst[k][c] = cb[c][off];
        gx = (gx + 1 == a.nx) ? 0 : gx + 1;
      }
    };
    auto advance = [&]() {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cur[k][c] = nx1[k][c];
          nx1[k][c] = nx2[k][c];
        }
    };
    const int rows = XT + mx2;
    load_group(cur);
    load_group(nx1);
    if (mx2 >= XT) {
      load_group(nx2);
      x_group<SGS, G_HEAD, 0>(acc, cur, ms, wx, 0, mx2);
      advance();
      load_group(nx2);
      x_group<SGS, G_HEAD, 4>(acc, cur, ms, wx, 4, mx2);
      advance();
      for (int r0 = XT; r0 < rows; r0 += 4) {
        load_group(nx2);
        x_group<SGS, G_FULL, 0>(acc, cur, ms, wx, r0, mx2);
        advance();
      }
    } else {
      for (int r0 = 0; r0 < rows; r0 += 4) {
        load_group(nx2);
        x_group<SGS, G_ANY, 0>(acc, cur, ms, wx, r0, mx2);
        advance();
      }
    }
  }

  // ---- stage Z, one LDS field group at a time
  const int nch = a.zt / RZ;
  const int zrows = RZ + mz2;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int f0 = g * GF;
    const int nfg = (NF - f0) < GF ? (NF - f0) : GF;
    if (g > 0) __syncthreads();   // the previous group's readers are done
    if (tid < zh) {
#pragma unroll
      for (int f = 0; f < GF; ++f)
        if (f < nfg)
#pragma unroll
          for (int o = 0; o < XT; ++o) tx[(f * XT + o) * zs + tid] = acc[f0 + f][o];
    }
    __syncthreads();
    const int items = nfg * XT * nch;
    const int ngz = (zrows + 3) / 4;
    for (int it = tid; it < items; it += kXzThreads) {
      const int c = it % nch;
      const int row = it / nch;
      const int f = f0 + row / XT, o = row % XT;
      const int xg = x0 + o;
      if (xg >= a.nx || f >= (SGS ? NF : a.ncomp)) continue;
      float zacc[RZ];
#pragma unroll
      for (int q = 0; q < RZ; ++q) zacc[q] = 0.0f;
      z_run(zacc, tx + row * zs + c * RZ, wz, ngz);
      // a run of RZ = 4 outputs leaves as one 16-byte store where it can
      // (four neighbouring lanes then fill a whole 64-byte segment)
      const int zl = c * RZ;
      float *dst = gout + (((size_t)xg * a.ny + y) * a.out_nf + f) * a.nz + z0 + zl;
      if ((a.nz & 3) == 0 && zl + 3 < a.zt && z0 + zl + 3 < a.nz) {
        *reinterpret_cast<float4 *>(dst) = make_float4(zacc[0], zacc[1], zacc[2], zacc[3]);
      } else {
#pragma unroll
        for (int q = 0; q < RZ; ++q)
          if (zl + q < a.zt && z0 + zl + q < a.nz) dst[q] = zacc[q];
      }
    }
  }
}

}  // namespace

int xz_tile_z(int nz, int mz) {
  const int zmax = ((kXzThreads - 2 * mz) / RZ) * RZ;
  const int ntile = (nz + zmax - 1) / zmax;
  const int per = (nz + ntile - 1) / ntile;
  return ((per + RZ - 1) / RZ) * RZ;
}

hipError_t launch_xz(const XzArgs &a, bool sgs, hipStream_t s) {
  const int zh = a.zt + 2 * a.mz;
  const int zs = ((zh + 4 + 3) / 4) * 4;
  const int gf = sgs ? 5 : 3;   // fields per LDS group
  const size_t lds = (size_t)gf * XT * zs * sizeof(float);
  const long nblk = (long)a.nxt * a.nzt * a.ny;
  if (lds > 65536) {
    hipError_t e = sgs ? hipFuncSetAttribute((const void *)k_xz<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                       : hipFuncSetAttribute((const void *)k_xz<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (sgs)
    k_xz<true><<<(unsigned)nblk, kXzThreads, lds, s>>>(a, a.in, a.out, a.wx, a.wz);
  else
    k_xz<false><<<(unsigned)nblk, kXzThreads, lds, s>>>(a, a.in, a.out, a.wx, a.wz);
  return hipGetLastError();
}

}  // namespace eles
