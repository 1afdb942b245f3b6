// x/z pass of the stress on the matrix cores for wide stencils.
//
// Same arithmetic as k_xzm.hip (the periodic x and z parts of the separable
// filter of eq. (2) as banded 16 x 16 products on v_mfma_f32_16x16x4f32,
// the nine fields of the stress formed in registers from the shifted
// velocity), for x stencils up to 2 * 44 + 1 taps and z stencils up to
// 2 * 48 + 1 taps. A z tile then reads its own 16-column chunk and up to
// three on each side, and nine fields of that window do not fit in
// registers; so each wave carries three of the nine fields:
//   group 0: u1', u2, u3;   group 1: u1'u1', u1'u2, u1'u3;   group 2: u2u2, u2u3, u3u3
// The (16-row x tile, group) items of a wall-normal plane y, group fastest,
// are cut into rows of four, one item per wave of a four-wave block (one
// wave per SIMD, so every SIMD carries the same work); the block's waves
// walk the same z tiles together and share the velocity rows they load
// through the compute unit's cache.
//
// Along a piece of a row the wave walks 16-column chunks in z: the x
// stencil of a chunk (the three fields' products as the A operand, the taps
// as the B operand; rows of the A tile in the order z = 4 (row % 4) +
// row / 4, so accumulator register r of lane group j holds column 4 r + j),
// then the z stencil of the tile whose window the chunk completes, from a
// ring of 2H + 1 x-filtered chunks in registers. While step s of a chunk
// forms its products, the velocities of step s of the next chunk are
// requested into the same registers.
#include <type_traits>

#include "eles_internal.h"

#define XZW_INLINE __attribute__((always_inline))

namespace eles {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
// word 3 of a raw buffer descriptor on gfx9-family parts (32-bit data
// format, no swizzle)
constexpr int kBufWord3 = 0x00020000;
constexpr int kNF = 9;                 // fields of the stress
constexpr int kTapBase = kXzTileX - 1;   // padded-tap entry of offset -m

__device__ inline int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

__device__ inline f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Tap of offset d (|d| <= m) from the padded FP32 array; zero outside.
__device__ inline float tap(const float *__restrict__ w, int m, int d) {
  return (d >= -m && d <= m) ? w[d + kTapBase + m] : 0.0f;
}

template <int I, int N, class F>
__device__ XZW_INLINE inline void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <int KS, int H, bool VEC>
__global__ void __launch_bounds__(kXzmWaves * 64) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_xzw(XzArgs a, XzmPlan p) {
  constexpr int NW = 2 * H + 1;   // chunks one z tile reads
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, j = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gb = xcd_remap(blockIdx.x, gridDim.x);
  const int total = p.nrow * p.nct;
  const int start = (int)((long)gb * total / gridDim.x), end = (int)((long)(gb + 1) * total / gridDim.x);
  if (start >= end) return;
  const int nx = a.nx, nz = a.nz, mx = a.mx, mz = a.mz;
  const int plane = a.ny * nz;

  // x stencil, B operand of step s: lane (k-slot j, output column i) holds
  // tx(x_in - x_out) with x_in = x0 - mx + 4 s + j, x_out = x0 + i
  float bx[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) bx[s] = tap(a.wx, mx, 4 * s + j - i - mx);
  // z stencil, A operand of window chunk c (relative -H..H) and register r:
  // lane (output row i, k-slot j) holds tz(z_in - z_out), z_in = 16 c + 4 r + j
  float az[NW][4];
#pragma unroll
  for (int c = 0; c < NW; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) az[c][r] = tap(a.wz, mz, 16 * (c - H) + 4 * r + j - i);

  // the item of block row br: x tile and field group, and whether it lies
  // past the plane's items (last row of a plane when 3 nxt % 4 != 0: the
  // wave then runs item (4 br + w) mod 3 nxt with its stores dropped)
  auto item = [&](int br, int &xt, int &grp) XZW_INLINE {
    int it = 4 * br + wave;
    const bool drop = it >= 3 * p.nxt;
    it = drop ? it - 3 * p.nxt : it;
    xt = it / 3;
    grp = it - 3 * xt;
    return drop;
  };

  const int nbytes = (int)((unsigned)a.nx * a.ny * a.nz * 4u);
  const __amdgpu_buffer_rsrc_t u0 = __builtin_amdgcn_make_buffer_rsrc((void *)a.in, 0, nbytes, kBufWord3);
  const __amdgpu_buffer_rsrc_t u1 =
      __builtin_amdgcn_make_buffer_rsrc((void *)(a.in + a.in_stride), 0, nbytes, kBufWord3);
  const __amdgpu_buffer_rsrc_t u2 =
      __builtin_amdgcn_make_buffer_rsrc((void *)(a.in + 2 * a.in_stride), 0, nbytes, kBufWord3);
  const int zrow = 4 * (i & 3) + (i >> 2);   // chunk column of A row i
  const unsigned row_bytes = (unsigned)a.ny * kNF * nz * 4;   // one x row of the output

  // where the next chunk's velocities come from: first x row of this lane
  // (wrapped), plane offset y nz, chunk index
  int nxs, nyz, nk;
  auto target_row = [&](int y, int xt) XZW_INLINE {
    nxs = wrapi(16 * xt - mx + j, nx);
    nyz = y * nz;
  };
  auto first = [&]() XZW_INLINE -> unsigned {
    int zc = 16 * nk + zrow;
    if (nk < 0 || 16 * nk + 16 > nz) zc = wrapi(zc, nz);
    return (unsigned)(nxs * plane + nyz + zc);
  };
  float b[KS][3];
  auto load_step = [&](int s, int &xi, unsigned &e) XZW_INLINE {
    b[s][0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(u0, e * 4, 0, 0));
    b[s][1] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(u1, e * 4, 0, 0));
    b[s][2] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(u2, e * 4, 0, 0));
    // nx >= 4: one subtraction wraps; selects, not a branch
    xi += 4;
    e += 4 * plane;
    const bool w = xi >= nx;
    xi = w ? xi - nx : xi;
    e = w ? e - nx * plane : e;
  };

  f4 win[NW][3];
  // x stencil of the chunk whose velocities are in b, into ring slot S,
  // requesting the velocities of the current target into b step by step
  // the group's three products q_c of the shifted velocity (v0, v1, v2):
  // group 0 (1 v0, 1 v1, 1 v2), group 1 (v0 v0, v0 v1, v0 v2), group 2
  // (v1 v1, v1 v2, v2 v2)
  auto xfilter = [&](auto slot, float ms, int grp) XZW_INLINE {
    constexpr int S = decltype(slot)::value;
    const bool g0 = grp == 0, g1 = grp == 1;
    int xi = nxs;
    unsigned e = first();
#pragma unroll
    for (int f = 0; f < 3; ++f) win[S][f] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const float v0 = b[s][0] - ms, v1 = b[s][1], v2 = b[s][2];
      const float A = g0 ? 1.0f : (g1 ? v0 : v1);
      const float C = g0 ? 1.0f : (g1 ? v0 : v2);
      const float q[3] = {A * (g0 || g1 ? v0 : v1), A * (g0 || g1 ? v1 : v2), C * v2};
      load_step(s, xi, e);
      // keep this step's loads here, a whole chunk ahead of their use
      __builtin_amdgcn_sched_barrier(0);
      const float w = bx[s];
#pragma unroll
      for (int f = 0; f < 3; ++f) win[S][f] = mma(q[f], w, win[S][f]);
    }
  };
  // z stencil of tile t of row (y, x0) whose newest chunk sits in slot S,
  // stored as fields 3 grp .. 3 grp + 2. With nz % 4 == 0 the stores go
  // through a buffer descriptor whose range ends at the last x row: lanes
  // past nx fall outside it, lanes past nz get an offset outside it, and
  // the hardware drops both, so each tile issues the same three stores.
  auto zfilter = [&](auto slot, int t, int y, int x0, int grp, bool drop) XZW_INLINE {
    constexpr int S = decltype(slot)::value;
    f4 acc[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) acc[f] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NW; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int f = 0; f < 3; ++f) acc[f] = mma(az[c][r], win[(S + 1 + c) % NW][f][r], acc[f]);
    const int zo = 16 * t + 4 * j;
    const int xo = x0 + i;
    if constexpr (VEC) {
      const size_t rem = (size_t)(nx - x0) * row_bytes;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          a.out + (size_t)x0 * (row_bytes / 4), 0, (int)(rem < 0x7fffffffu ? rem : 0x7fffffffu), kBufWord3);
      const unsigned off =
          zo < nz && !drop ? (unsigned)(i * row_bytes + (y * kNF * nz + 3 * grp * nz + zo) * 4) : 0x80000000u;
#pragma unroll
      for (int f = 0; f < 3; ++f)
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, acc[f]), rs, off + f * nz * 4, 0, 0);
    } else if (xo < nx && !drop) {
      float *dst = a.out + ((size_t)xo * a.ny + y) * (size_t)(kNF * nz) + 3 * grp * nz + zo;
#pragma unroll
      for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (zo + r < nz) dst[(size_t)f * nz + r] = acc[f][r];
    }
  };

  // the block's range starts in block row (y, br) at tile ta; every later
  // piece starts a new block row at tile 0
  int y, br, ta;
  {
    const int row = start / p.nct;
    ta = start - row * p.nct;
    y = row / p.nxg;
    br = row - y * p.nxg;
  }
  int left = end - start;
  {
    int xt0, g0;
    item(br, xt0, g0);
    target_row(y, xt0);
  }
  nk = ta - H;
  {
    int xi = nxs;
    unsigned e = first();
#pragma unroll
    for (int s = 0; s < KS; ++s) load_step(s, xi, e);
  }
  while (left > 0) {
    // piece: tiles [ta, tb) of block row (y, br), chunks [ta - H, tb + H)
    const int tb = left < p.nct - ta ? ta + left : p.nct;
    left -= tb - ta;
    int xt, grp;
    const bool drop = item(br, xt, grp);
    const int x0 = 16 * xt;
    const float ms = a.mshift[y];
    const int ke = tb + H;
    int k = ta - H;
    // the chunk after k: the next one of this piece, else the first one of
    // the next block row, else k again (a harmless reload)
    auto aim = [&]() XZW_INLINE {
      if (k + 1 < ke) {
        nk = k + 1;
      } else if (left > 0) {
        const bool wrap = br + 1 == p.nxg;
        int xn, gn;
        item(wrap ? 0 : br + 1, xn, gn);
        target_row(wrap ? y + 1 : y, xn);
        nk = -H;
      } else {
        nk = k;
      }
    };
    // chunks ta - H .. ta + H into slots 0 .. 2H
    static_for<0, NW>([&](auto q) XZW_INLINE {
      aim();
      xfilter(q, ms, grp);
      ++k;
    });
    // each step: z stencil of the tile whose last chunk is the newest one,
    // then the x stencil of the next chunk. Every step ends with the next
    // chunk's loads, also on entry, so the waits for them count the same
    // stores on every path.
    bool done = false;
    while (!done) {
      static_for<0, NW>([&](auto q) XZW_INLINE {
        constexpr int S = (2 * H + decltype(q)::value) % NW;
        if (done) return;
        zfilter(std::integral_constant<int, S>{}, k - 1 - H, y, x0, grp, drop);
        if (k == ke) {
          done = true;
          return;
        }
        aim();
        xfilter(std::integral_constant<int, (S + 1) % NW>{}, ms, grp);
        ++k;
      });
    }
    if (++br == p.nxg) {
      br = 0;
      ++y;
    }
    ta = 0;
  }
}

using KernelFn = void (*)(XzArgs, XzmPlan);

// instances: x stencil steps rounded up to an even count (the extra steps
// multiply zero taps), z halo chunks 1..3, 16-byte stores (nz % 4 == 0)
template <int H>
KernelFn pick_ks(int ks) {
  switch ((ks + 1) & ~1) {
    case 14: return k_xzw<14, H, true>;
    case 16: return k_xzw<16, H, true>;
    case 18: return k_xzw<18, H, true>;
    case 20: return k_xzw<20, H, true>;
    case 22: return k_xzw<22, H, true>;
    case 24: return k_xzw<24, H, true>;
    case 26: return k_xzw<26, H, true>;
    default: return nullptr;
  }
}

KernelFn pick(const XzmPlan &p) {
  if (!p.vec) return nullptr;
  switch (p.h) {
    case 1: return pick_ks<1>(p.ks);
    case 2: return pick_ks<2>(p.ks);
    case 3: return pick_ks<3>(p.ks);
    default: return nullptr;
  }
}

}  // namespace

bool xzw_plan(int nx, int ny, int nz, int mx, int mz, XzmPlan *p) {
  const int ks = (16 + 2 * mx + 3) / 4;
  const int h = (mz + 15) / 16;
  if (ks > kXzwMaxSteps || h > kXzwMaxHalo || nx < 4) return false;
  if ((long)nx * ny * nz >= (1L << 29)) return false;   // byte offsets below 2^31
  if (16L * ny * 9 * nz * 4 >= (1L << 31)) return false;
  if ((nz & 3) != 0) return false;   // 16-byte stores only
  p->wide = 1;
  p->ks = ks < 13 ? 14 : (ks + 1) & ~1;
  p->h = h < 1 ? 1 : h;
  p->vec = (nz & 3) == 0;
  p->nxt = (nx + 15) / 16;
  p->nxg = (3 * p->nxt + kXzmWaves - 1) / kXzmWaves;   // block rows per plane
  p->nct = (nz + 15) / 16;
  p->nrow = p->nxg * ny;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return false;
  const KernelFn fn = pick(*p);
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kXzmWaves * 64, 0) != hipSuccess)
    return false;
  if (per_cu < 1 || ncu < 1) return false;
  const long tiles = (long)p->nrow * p->nct;
  const long want = (tiles + 1) / 2;
  const long cap = (long)per_cu * ncu;
  p->nblk = (int)(want < cap ? want : cap);
  return true;
}

hipError_t launch_xzw(const XzArgs &a, const XzmPlan &p, hipStream_t s) {
  const KernelFn fn = pick(p);
  if (!fn) return hipErrorInvalidValue;
  fn<<<(unsigned)p.nblk, kXzmWaves * 64, 0, s>>>(a, p);
  return hipGetLastError();
}

}  // namespace eles
