// y pass: the wall-normal part of the filter, as a product with the folded
// [ny x ny] operator of the reflected channel (Sec. 2.2, eq. (7)) applied to
// every (x, z) line, on the matrix cores, fused with the stress epilogue.
//
// For an x-slab the fields form a [ny x nz] matrix (z contiguous); the
// filtered slab is W^s times it. One wave computes a 16 x 16 output
// tile with v_mfma_f32_16x16x4_f32 (FP32) or
// v_mfma_f32_16x16x32_bf16 (BF16, and the three-product hi/lo split). The
// operator is banded: the K loop covers only the columns that are nonzero
// in the tile's 16 rows.
//
// Stress mode, for the nine x/z-filtered fields X = F_xz(u1', u2, u3,
// u1'u1', u1'u2, u1'u3, u2u2, u2u3, u3u3) with u1' = u1 - m(y):
//   ubar_1 = W^+ X_0 + M,  ubar_2 = W^- X_1,  ubar_3 = W^+ X_2,
//   tau_11 = W^+ X_3 + 2 C^+ X_0 - (W^+ X_0)^2 + s,
//   tau_12 = W^- X_4 + C^- X_1 - (W^+ X_0)(W^- X_1),
//   tau_13 = W^+ X_5 + C^+ X_2 - (W^+ X_0)(W^+ X_2),
//   tau_22, tau_23, tau_33 = W^(s_i s_j) X - ubar_i ubar_j,
// the exact expansion of F(u_i u_j) - F(u_i) F(u_j) about the profile m
// (products of a field of y alone commute with the x and z filters). The
// correction products share the B operand of X_0..X_2. Plane sums of the
// nine outputs are reduced per tile in FP64 for the averages over x and z.
#include "eles_internal.h"

namespace eles {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (unsigned short)(b >> 16);
}
__device__ inline float bf16_val(unsigned short h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ inline f4 mma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f4 mma16(us8 a, us8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b),
                                                 c, 0, 0, 0);
}

// BF16 operand of one lane: the plain rounding, or the hi/lo split.
template <int PREC>
struct Opd16 {
  us8 hi, lo;
};

template <int PREC>
__device__ inline f4 mma_b(const Opd16<PREC> &a, const Opd16<PREC> &b, f4 c) {
  if (PREC == 2) {
    c = mma16(a.lo, b.hi, c);
    c = mma16(a.hi, b.lo, c);
  }
  return mma16(a.hi, b.hi, c);
}

template <int PREC>
__device__ inline Opd16<PREC> load_a16(const uint16_t *__restrict__ hi, const uint16_t *__restrict__ lo,
                                       size_t o) {
  Opd16<PREC> r;
  r.hi = *reinterpret_cast<const us8 *>(hi + o);
  if (PREC == 2) r.lo = *reinterpret_cast<const us8 *>(lo + o);
  return r;
}

template <int PREC>
__device__ inline Opd16<PREC> split8(const float (&v)[8]) {
  Opd16<PREC> r;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    unsigned short h = bf16_rne(v[e]);
    r.hi[e] = h;
    if (PREC == 2) r.lo[e] = bf16_rne(v[e] - bf16_val(h));
  }
  return r;
}

// Union of the nonzero column ranges of rows i0..i0+15.
__device__ inline void tile_band(const int *__restrict__ rb, int i0, int &lo, int &hi) {
  lo = 1 << 30;
  hi = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int a = rb[2 * (i0 + r)], b = rb[2 * (i0 + r) + 1];
    if (b > a) {
      lo = min(lo, a);
      hi = max(hi, b);
    }
  }
  if (hi == 0) lo = 0;
}

template <bool SGS, int PREC>
__global__ void __launch_bounds__(64 * kYWaves)
k_y(YArgs a, const float *__restrict__ X, const int *__restrict__ rowband) {
  constexpr int NA = SGS ? 9 : 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int nib = a.mpad / kYBlockM;
  // items (x, i-block, z-tile) with z fastest; the tile count is padded to
  // a multiple of the block's waves so a block never straddles two rows
  const int nzt = (a.n16 + kYWaves - 1) / kYWaves * kYWaves;
  const long items = (long)a.nx * nib * nzt;
  const long item = (long)xcd_remap(blockIdx.x, gridDim.x) * kYWaves + wave;
  const int zt = (int)(item % nzt);
  const long rest = item / nzt;
  const int ib = (int)(rest % nib);
  const int x = (int)(rest / nib);
  const bool live = item < items && zt < a.n16;
  const int i0 = ib * kYBlockM, z0 = zt * kYTileN;
  const int field = SGS ? 0 : blockIdx.y;
  const int opsel = SGS ? 0 : (int)((a.parity_mask >> field) & 1u);
  const int zc = z0 + col;
  const bool zok = live && zc < a.nz;

  int klo = 0, khi = 0;
  if (live) tile_band(rowband, i0, klo, khi);

  f4 acc[NA];
#pragma unroll
  for (int f = 0; f < NA; ++f) acc[f] = f4{0.f, 0.f, 0.f, 0.f};

  const size_t slab = (size_t)x * a.ny;
  const float *Xf = X + (size_t)field * a.in_fs + (size_t)x * a.in_xs;

  if (PREC == 0) {
    // B fragments arrive two K steps ahead of the matrix instructions
    // that consume them.
    float b[NA], bn[NA], bnn[NA];
    auto load_b = [&](int k0, float (&dst)[NA]) {
      const int kk = k0 + grp;
      const bool ok = zok && kk < a.ny && k0 < khi;
      const size_t off = (size_t)(ok ? kk : 0) * a.in_ks + (ok ? zc : 0);
#pragma unroll
      for (int f = 0; f < NA; ++f) {
        const float t = Xf[(size_t)f * a.in_fs + off];
        dst[f] = ok ? t : 0.0f;
      }
    };
    const int kb0 = klo & ~3;
    load_b(kb0, b);
    load_b(kb0 + 4, bn);
    for (int k0 = kb0; k0 < khi; k0 += 4) {
      load_b(k0 + 8, bnn);
      const size_t ao = (size_t)(i0 + col) * a.kpad + k0 + grp;
      if (SGS) {
        const float ap = a.a32[0][ao], am = a.a32[1][ao];
        const float cp = a.a32[2][ao], cm = a.a32[3][ao];
        acc[0] = mma32(ap, b[0], acc[0]);
        acc[3] = mma32(2.0f * cp, b[0], acc[3]);
        acc[1] = mma32(am, b[1], acc[1]);
        acc[4] = mma32(cm, b[1], acc[4]);
        acc[2] = mma32(ap, b[2], acc[2]);
        acc[5] = mma32(cp, b[2], acc[5]);
        acc[3] = mma32(ap, b[3], acc[3]);
        acc[4] = mma32(am, b[4], acc[4]);
        acc[5] = mma32(ap, b[5], acc[5]);
        acc[6] = mma32(ap, b[6], acc[6]);
        acc[7] = mma32(am, b[7], acc[7]);
        acc[8] = mma32(ap, b[8], acc[8]);
      } else {
        acc[0] = mma32(a.a32[opsel][ao], b[0], acc[0]);
      }
#pragma unroll
      for (int f = 0; f < NA; ++f) {
        b[f] = bn[f];
        bn[f] = bnn[f];
      }
    }
  } else {
    for (int k0 = klo & ~31; k0 < khi; k0 += 32) {
      const int kb = k0 + 8 * grp;
      const size_t ao = (size_t)(i0 + col) * a.kpad + kb;
      auto load8 = [&](int f, float (&v)[8]) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = kb + e;
          v[e] = (zok && k < a.ny) ? Xf[(size_t)f * a.in_fs + (size_t)k * a.in_ks + zc] : 0.0f;
        }
      };
      if (SGS) {
        const Opd16<PREC> ap = load_a16<PREC>(a.ahi[0], a.alo[0], ao);
        const Opd16<PREC> am = load_a16<PREC>(a.ahi[1], a.alo[1], ao);
        const Opd16<PREC> cp = load_a16<PREC>(a.ahi[2], a.alo[2], ao);
        const Opd16<PREC> cm = load_a16<PREC>(a.ahi[3], a.alo[3], ao);
#pragma unroll
        for (int f = 0; f < 9; ++f) {
          float v[8];
          load8(f, v);
          const Opd16<PREC> bo = split8<PREC>(v);
          switch (f) {
            case 0:
              acc[0] = mma_b<PREC>(ap, bo, acc[0]);
              acc[3] = mma_b<PREC>(cp, bo, acc[3]);
              acc[3] = mma_b<PREC>(cp, bo, acc[3]);
              break;
            case 1:
              acc[1] = mma_b<PREC>(am, bo, acc[1]);
              acc[4] = mma_b<PREC>(cm, bo, acc[4]);
              break;
            case 2:
              acc[2] = mma_b<PREC>(ap, bo, acc[2]);
              acc[5] = mma_b<PREC>(cp, bo, acc[5]);
              break;
            case 4:
            case 7:
              acc[f] = mma_b<PREC>(am, bo, acc[f]);
              break;
            default:
              acc[f] = mma_b<PREC>(ap, bo, acc[f]);
          }
        }
      } else {
        const Opd16<PREC> w = load_a16<PREC>(a.ahi[opsel], a.alo[opsel], ao);
        float v[8];
        load8(0, v);
        acc[0] = mma_b<PREC>(w, split8<PREC>(v), acc[0]);
      }
    }
  }

  // ---- epilogue
  if (!SGS) {
    if (!zok) return;
    float *dst = a.out + (size_t)field * a.out_fs + (size_t)x * a.out_xs;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 4 * grp + r;
      if (i < a.ny) dst[(size_t)i * a.out_ks + zc] = acc[0][r];
    }
    return;
  }
  __shared__ double red[kYWaves][9][kYBlockM];
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  const float *Mp = a.prof32 + a.mpad;
  const float *Sp = a.prof32 + 2 * a.mpad;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 4 * grp + r;
    const bool ok = zok && i < a.ny;
    const float mi = (live && i < a.ny) ? Mp[i] : 0.0f;
    const float si = (live && i < a.ny) ? Sp[i] : 0.0f;
    const float f0 = acc[0][r], f1 = acc[1][r], f2 = acc[2][r];
    float o[9];
    o[0] = f0 + mi;
    o[1] = f1;
    o[2] = f2;
    o[3] = (acc[3][r] - f0 * f0) + si;
    o[4] = acc[4][r] - f0 * f1;
    o[5] = acc[5][r] - f0 * f2;
    o[6] = acc[6][r] - f1 * f1;
    o[7] = acc[7][r] - f1 * f2;
    o[8] = acc[8][r] - f2 * f2;
    if (ok) {
      const size_t off = (slab + i) * a.nz + zc;
#pragma unroll
      for (int q = 0; q < 3; ++q) a.ubar[q * N + off] = o[q];
#pragma unroll
      for (int q = 0; q < 6; ++q) a.tau[q * N + off] = o[3 + q];
    }
    if (a.part) {
      // FP64 sum over the tile's 16 columns of row i
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        double v = ok ? (double)o[q] : 0.0;
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        if (col == 0) red[wave][q][4 * grp + r] = v;
      }
    }
  }
  if (!a.part) return;
  __syncthreads();
  // the block's four tiles share (x, i-block): add them in a fixed order
  if (item - wave < items && threadIdx.x < 9 * kYBlockM) {
    const int q = threadIdx.x / kYBlockM, rr = threadIdx.x % kYBlockM;
    const int i = i0 + rr;
    if (i < a.ny) {
      double v = red[0][q][rr];
#pragma unroll
      for (int w = 1; w < kYWaves; ++w) v += red[w][q][rr];
      const size_t P = (size_t)a.nx * (nzt / kYWaves);
      const size_t p = (size_t)x * (nzt / kYWaves) + zt / kYWaves;
      a.part[((size_t)q * a.ny + i) * P + p] = v;
    }
  }
}

constexpr int kStatT = 256;

__global__ void __launch_bounds__(kStatT) k_stats(const double *__restrict__ part, double *__restrict__ stats,
                                                  int nparts, double inv) {
  __shared__ double red[kStatT];
  const double *src = part + (size_t)blockIdx.x * nparts;
  double s = 0.0;
  for (int p = threadIdx.x; p < nparts; p += kStatT) s += src[p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kStatT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) stats[blockIdx.x] = red[0] * inv;
}

template <bool SGS>
hipError_t launch_y_t(const YArgs &a, int prec, hipStream_t s) {
  const int nzt = (a.n16 + kYWaves - 1) / kYWaves * kYWaves;
  const long items = (long)a.nx * (a.mpad / kYBlockM) * nzt;
  const dim3 grid((unsigned)((items + kYWaves - 1) / kYWaves), SGS ? 1 : a.nfield);
  const dim3 block(64 * kYWaves);
  if (prec == 0)
    k_y<SGS, 0><<<grid, block, 0, s>>>(a, a.in, a.rowband);
  else if (prec == 1)
    k_y<SGS, 1><<<grid, block, 0, s>>>(a, a.in, a.rowband);
  else
    k_y<SGS, 2><<<grid, block, 0, s>>>(a, a.in, a.rowband);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_y(const YArgs &a, bool sgs, int prec, hipStream_t s) {
  return sgs ? launch_y_t<true>(a, prec, s) : launch_y_t<false>(a, prec, s);
}

hipError_t launch_stats(const double *part, double *stats, int ny, int nparts, double inv_count,
                        hipStream_t s) {
  k_stats<<<9 * ny, kStatT, 0, s>>>(part, stats, nparts, inv_count);
  return hipGetLastError();
}

}  // namespace eles
