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
// strip goes to LDS. Stage Z: each thread takes runs of eight z outputs of
// one (field, x) row and applies the z stencil from LDS, writing coalesced
// rows back to HBM.
//
// Taps are read through uniform (scalar) loads from zero-padded tap arrays,
// so the per-output loops carry no bounds tests.
#include "eles_internal.h"

namespace eles {
namespace {

constexpr int XT = kXzTileX;
constexpr int RZ = kXzRunZ;

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

template <bool SGS>
__global__ void __launch_bounds__(kXzThreads)
k_xz(XzArgs a, const float *__restrict__ gin, float *__restrict__ gout,
     const float *__restrict__ wx, const float *__restrict__ wz) {
  constexpr int NF = Fields<SGS>::NF;
  extern __shared__ float tx[];   // [NF][XT][zs]
  const int zh = a.zt + 2 * a.mz;
  const int zs = ((zh + 4 + 3) / 4) * 4;
  const int tid = threadIdx.x;

  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int xt = b % a.nxt;
  const int rest = b / a.nxt;
  const int ztile = rest % a.nzt;
  const int y = rest / a.nzt;
  const int x0 = xt * XT, z0 = ztile * a.zt;

  // zero the row tails read by the last vector loads of stage Z
  for (int q = tid; q < NF * XT * (zs - zh); q += kXzThreads) {
    int row = q / (zs - zh), col = zh + q % (zs - zh);
    tx[row * zs + col] = 0.0f;
  }

  // ---- stage X
  if (tid < zh) {
    const int gz = wrap(z0 - a.mz + tid, a.nz);
    const float ms = SGS ? a.mshift[y] : 0.0f;
    const size_t plane = (size_t)y * a.nz + gz;
    const size_t xstride = (size_t)a.ny * a.nz;
    float acc[NF][XT];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int o = 0; o < XT; ++o) acc[f][o] = 0.0f;

    const int rows = ((XT + 2 * a.mx) + 3) / 4 * 4;
    int gx = wrap(x0 - a.mx, a.nx);
    float cur[4][3], nxt[4][3];
    auto load_group = [&](float (&dst)[4][3]) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const size_t off = (size_t)gx * xstride + plane;
#pragma unroll
        for (int c = 0; c < 3; ++c)
          dst[k][c] = (c < a.ncomp) ? gin[c * a.in_stride + off] : 0.0f;
        gx = (gx + 1 == a.nx) ? 0 : gx + 1;
      }
    };
    load_group(cur);
    for (int r0 = 0; r0 < rows; r0 += 4) {
      if (r0 + 4 < rows) load_group(nxt);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float c3[3] = {cur[k][0] - ms, cur[k][1], cur[k][2]};
        float v[NF];
        Fields<SGS>::form(c3, v);
        const float *w = wx + (r0 + k + XT - 1);
#pragma unroll
        for (int o = 0; o < XT; ++o) {
          const float wt = w[-o];
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[f][o] = fmaf(wt, v[f], acc[f][o]);
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) cur[k][c] = nxt[k][c];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int o = 0; o < XT; ++o) tx[(f * XT + o) * zs + tid] = acc[f][o];
  }
  __syncthreads();

  // ---- stage Z
  const int nch = a.zt / RZ;
  const int items = NF * XT * nch;
  const int zrows = ((RZ + 2 * a.mz) + 3) / 4 * 4;
  const size_t xstride = (size_t)a.ny * a.nz;
  for (int it = tid; it < items; it += kXzThreads) {
    const int c = it % nch;
    const int row = it / nch;
    const int f = row / XT, o = row % XT;
    const int xg = x0 + o;
    if (xg >= a.nx || f >= (SGS ? NF : a.ncomp)) continue;
    const float *src = tx + row * zs + c * RZ;
    float acc[RZ];
#pragma unroll
    for (int q = 0; q < RZ; ++q) acc[q] = 0.0f;
    for (int t4 = 0; t4 < zrows; t4 += 4) {
      const float4 v = *reinterpret_cast<const float4 *>(src + t4);
      const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float *w = wz + (t4 + k + RZ - 1);
#pragma unroll
        for (int q = 0; q < RZ; ++q) acc[q] = fmaf(w[-q], vv[k], acc[q]);
      }
    }
    float *dst = gout + f * a.out_stride + (size_t)xg * xstride + (size_t)y * a.nz + z0 + c * RZ;
#pragma unroll
    for (int q = 0; q < RZ; ++q)
      if (c * RZ + q < a.zt && z0 + c * RZ + q < a.nz) dst[q] = acc[q];
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
  const int nf = sgs ? 9 : 3;
  const size_t lds = (size_t)nf * XT * zs * sizeof(float);
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
