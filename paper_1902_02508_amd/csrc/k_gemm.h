// Generic product C[M][N] = A[M][K] * B[N][K]^T on the matrix cores
// (v_mfma_f32_16x16x32_bf16), both operands with K contiguous. One wave owns
// 16 rows of C and NT tiles of 16 columns; the K range of a wave can be a
// chunk of a longer reduction (split K). A is BF16 or FP32 (rounded, or
// split into a hi/lo BF16 pair); B is BF16, optionally with its lo part.
// The epilogue receives the 16 x 16 accumulator tiles in the MFMA layout:
// lane (col = lane % 16, grp = lane / 16) holds rows 4 grp + r, r = 0..3.
#pragma once

#include "eles_internal.h"

namespace eles {

typedef float gf4 __attribute__((ext_vector_type(4)));
typedef __bf16 gbf8 __attribute__((ext_vector_type(8)));
typedef unsigned short gus8 __attribute__((ext_vector_type(8)));

__device__ inline unsigned short g_bf16(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (unsigned short)(b >> 16);
}
__device__ inline float g_f32(unsigned short h) { return __uint_as_float(((uint32_t)h) << 16); }

// Two FP32 values to two BF16 (round to nearest even, as g_bf16) in one
// instruction (v_cvt_pk_bf16_f32), packed low | high << 16.
typedef float gf2 __attribute__((ext_vector_type(2)));
typedef __bf16 gbf2 __attribute__((ext_vector_type(2)));
__device__ inline uint32_t g_bf16x2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(gf2{lo, hi}, gbf2));
}

__device__ inline gf4 g_mma(gus8 a, gus8 b, gf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(gbf8, a), __builtin_bit_cast(gbf8, b), c, 0,
                                                 0, 0);
}

struct NTArgs {
  const void *a;            // A rows, element (m, k) at a[m * lda + k]
  long lda;
  const uint16_t *bhi;      // B rows, element (n, k) at b[n * ldb + k]; rows
  const uint16_t *blo;      // >= N and columns >= K must hold zeros (lo may be null)
  long ldb;
  long M;
  int N, K;                 // N <= 16 * NT * gridDim.y
  int kchunk;               // K range of one wave (multiple of 32); K if no split
  long a_bstride;           // per blockIdx.z offsets (A elements, B elements)
  long b_bstride;
};

// AT: 0 = A is BF16 (bits); 1 = A is FP32, rounded to BF16; 2 = A is FP32,
// split into hi + lo with three products. BLO: use B's lo part (with AT 2).
// With FP32 A whose rows and K are multiples of 8 floats from a 16-byte
// aligned base (a8), a lane's eight values of a K chunk are two float4
// loads; else eight guarded scalar loads.
template <int AT, int NT, class Epi>
__device__ inline void nt_gemm_wave(const NTArgs &g, long m0, int n0, int kb, int ke, int z, Epi &epi) {
  const bool a8 = AT != 0 && g.K % 8 == 0 && g.lda % 8 == 0 && g.a_bstride % 8 == 0 &&
                  ((uintptr_t)g.a & 15u) == 0;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  gf4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = gf4{0.f, 0.f, 0.f, 0.f};
  const long m = m0 + col;
  const bool mok = m < g.M;
  float rowsum = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += 32) {
    const int ka = k0 + 8 * grp;
    gus8 ahi, alo;
    if (AT == 0) {
      const uint16_t *ap = (const uint16_t *)g.a + z * g.a_bstride + (mok ? m : 0) * g.lda + ka;
      gus8 t = *reinterpret_cast<const gus8 *>(ap);
      ahi = mok ? t : gus8{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int e = 0; e < 8; ++e) rowsum += g_f32(ahi[e]);
    } else {
      const float *ap = (const float *)g.a + z * g.a_bstride + (mok ? m : 0) * g.lda;
      float v[8];
      if (a8) {
        const bool ok = mok && ka < g.K;   // all eight or none
        const gf4 zero4 = gf4{0.f, 0.f, 0.f, 0.f};
        const gf4 v0 = ok ? *reinterpret_cast<const gf4 *>(ap + ka) : zero4;
        const gf4 v1 = ok ? *reinterpret_cast<const gf4 *>(ap + ka + 4) : zero4;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          v[e] = v0[e];
          v[4 + e] = v1[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (mok && ka + e < g.K) ? ap[ka + e] : 0.0f;
      }
      uint32_t hw[4], lw[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        hw[e] = g_bf16x2(v[2 * e], v[2 * e + 1]);
        if (AT == 2)
          lw[e] = g_bf16x2(v[2 * e] - __uint_as_float(hw[e] << 16), v[2 * e + 1] - __uint_as_float(hw[e] & 0xffff0000u));
      }
      ahi = __builtin_bit_cast(gus8, hw);
      if (AT == 2) alo = __builtin_bit_cast(gus8, lw);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int nrow = n0 + 16 * t + col;
      const bool nok = nrow < g.N;
      const long boff = z * g.b_bstride + (long)(nok ? nrow : 0) * g.ldb + ka;
      const gus8 zero8 = gus8{0, 0, 0, 0, 0, 0, 0, 0};
      const gus8 bh = nok ? *reinterpret_cast<const gus8 *>(g.bhi + boff) : zero8;
      if (AT == 2) {
        const gus8 bl = nok ? *reinterpret_cast<const gus8 *>(g.blo + boff) : zero8;
        acc[t] = g_mma(alo, bh, acc[t]);
        acc[t] = g_mma(ahi, bl, acc[t]);
      }
      acc[t] = g_mma(ahi, bh, acc[t]);
    }
  }
  epi(m0, n0, acc, rowsum, z);
}

}  // namespace eles
