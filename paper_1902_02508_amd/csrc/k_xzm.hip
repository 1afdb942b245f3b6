// x/z pass of the stress on the matrix cores.
//
// The periodic x and z parts of the separable filter of eq. (2) are banded
// Toeplitz operators. On a tile of 16 x 16 outputs each is a dense product
// with a band 16 + 2m inputs wide, which the FP32 MFMA v_mfma_f32_16x16x4f32
// evaluates four inputs at a time.
//
// Work: the x/z outputs of one wall-normal plane y and sixteen consecutive
// x (a "row" (y, x tile)) form nct tiles of 16 z columns. The rows' tiles,
// laid end to end, are cut into one contiguous range per wave (persistent
// waves, equal shares), so every wave does the same amount of work; a range
// covers one or two pieces of rows.
//
// Along a piece the wave walks 16-column input chunks in z. For each chunk
// it forms the nine fields of the stress (u1' = u1 - m(y), u2, u3 and their
// six products) from the raw velocity in registers and applies the x
// stencil as
//     X[z][x_out] = sum over x_in of P[x_in][z] tx(x_in - x_out),
// the products as the A operand (one value per lane, loaded straight from
// HBM: sixteen lanes read one 64-byte row segment) and the taps as the B
// operand, constant for the whole wave. The rows of the A tile are the 16
// columns of the chunk in the order z = 4 (row % 4) + row / 4, so that
// accumulator register r of lane group j holds column 4 r + j: the four
// lane groups hold four consecutive columns, which is the B operand of the
// z stencil
//     Y[z_out][x] = sum over z_in of tz(z_in - z_out) X[z_in][x]
// for four consecutive inputs. The x-filtered chunks feed the z product
// from registers, with no exchange. The z stencil half-width is at most 16,
// so a z tile reads its own chunk and one on each side.
//
// Chunks go in pairs, requested together. A piece's pairs start at the
// chunk before its first tile, so the pairs of a whole row (first tile 0)
// start at odd chunks: where rows start on 128-byte boundaries a pair
// covers the second half of one 128-byte line and the first half of the
// next, and the two halves of a line are requested one pair apart; by
// then the line has usually left L2 (evicted mostly by the kernel's own
// output stores), and it is fetched again. Starting pairs at even chunks
// costs a pair per cut inside a row. The wave keeps four x-filtered chunks
// in a ring of register slots (the pair just filtered and the one before);
// after each pair it filters the two z tiles that became complete. The pair
// loop is unrolled by two, so every slot is static.
//
// Loads: while step s of a pair forms its products, the velocities of step
// s of the next pair are requested into the same registers, so each load
// has a whole pair of matrix work to arrive.
//
// Each lane of a finished z tile holds four consecutive z outputs of one x,
// stored as one 16-byte store into the row-interleaved [x][y][f][z] layout.
#include <type_traits>

#include "eles_internal.h"

#define XZM_INLINE __attribute__((always_inline))

namespace eles {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
// word 3 of a raw buffer descriptor on gfx9-family parts (32-bit data
// format, no swizzle)
constexpr int kBufWord3 = 0x00020000;
constexpr int kNF = 9;          // fields of the stress
constexpr int kWaves = kXzmWaves;
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
__device__ XZM_INLINE inline void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <int KS, bool VEC>
__global__ void __launch_bounds__(kWaves * 64) __attribute__((amdgpu_waves_per_eu(1, 1))) k_xzm(XzArgs a, XzmPlan p) {
  constexpr int NR = 4;   // ring slots: two pairs of chunks
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, j = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // the block's range of (y, x group, z tile) positions; wave w takes x
  // tile 4 g + w of group g, so the four waves walk the same z positions of
  // neighbouring x tiles together and share their x-halo rows in cache
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
  // z stencil, A operand of window chunk c (relative -1..1) and register r:
  // lane (output row i, k-slot j) holds tz(z_in - z_out), z_in = 16 c + 4 r + j
  float az[3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) az[c][r] = tap(a.wz, mz, 16 * (c - 1) + 4 * r + j - i);

  // velocity components through buffer descriptors: 32-bit byte offsets,
  // no per-lane 64-bit addresses
  const int nbytes = (int)((unsigned)a.nx * a.ny * a.nz * 4u);
  const __amdgpu_buffer_rsrc_t u0 = __builtin_amdgcn_make_buffer_rsrc((void *)a.in, 0, nbytes, kBufWord3);
  const __amdgpu_buffer_rsrc_t u1 =
      __builtin_amdgcn_make_buffer_rsrc((void *)(a.in + a.in_stride), 0, nbytes, kBufWord3);
  const __amdgpu_buffer_rsrc_t u2 =
      __builtin_amdgcn_make_buffer_rsrc((void *)(a.in + 2 * a.in_stride), 0, nbytes, kBufWord3);
  const int zrow = 4 * (i & 3) + (i >> 2);   // chunk column of A row i
  const unsigned row_bytes = (unsigned)a.ny * kNF * nz * 4;   // one x row of the output

  // where the next pair's velocities come from: first x row of this lane
  // (wrapped), plane offset y nz, first chunk of the pair
  int nxs, nyz, nk;
  auto target_row = [&](int y, int xt) XZM_INLINE {
    nxs = wrapi(16 * xt - mx + j, nx);
    nyz = y * nz;
  };
  // element offset of chunk k's first row; the modulo runs only for chunks
  // that wrap around the periodic z direction
  auto first = [&](int k) XZM_INLINE -> unsigned {
    int zc = 16 * k + zrow;
    if (k < 0 || 16 * k + 16 > nz) zc = wrapi(zc, nz);
    return (unsigned)(nxs * plane + nyz + zc);
  };
  float b[2][KS][3];
  auto load_step = [&](int s, int &xi, unsigned (&e)[2]) XZM_INLINE {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      b[h][s][0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(u0, e[h] * 4, 0, 0));
      b[h][s][1] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(u1, e[h] * 4, 0, 0));
      b[h][s][2] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(u2, e[h] * 4, 0, 0));
    }
    // nx >= 4: one subtraction wraps; selects, not a branch
    xi += 4;
    const bool w = xi >= nx;
    xi = w ? xi - nx : xi;
    const unsigned de = w ? 4 * plane - nx * plane : 4 * plane;
    e[0] += de;
    e[1] += de;
  };

  f4 win[NR][kNF];
  // x stencil of the pair whose velocities are in b, into ring slots S and
  // S + 1, requesting the velocities of the target pair into b step by step
  auto xfilter = [&](auto slot, float ms) XZM_INLINE {
    constexpr int S = decltype(slot)::value;
    int xi = nxs;
    unsigned e[2] = {first(nk), first(nk + 1)};
#pragma unroll
    for (int f = 0; f < kNF; ++f) {
      win[S][f] = f4{0.f, 0.f, 0.f, 0.f};
      win[S + 1][f] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      float q[2][kNF];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float v0 = b[h][s][0] - ms, v1 = b[h][s][1], v2 = b[h][s][2];
        q[h][0] = v0, q[h][1] = v1, q[h][2] = v2;
        q[h][3] = v0 * v0, q[h][4] = v0 * v1, q[h][5] = v0 * v2;
        q[h][6] = v1 * v1, q[h][7] = v1 * v2, q[h][8] = v2 * v2;
      }
      load_step(s, xi, e);
      // keep this step's loads here, a whole pair ahead of their use
      __builtin_amdgcn_sched_barrier(0);
      const float w = bx[s];
#pragma unroll
      for (int f = 0; f < kNF; ++f) {
        win[S][f] = mma(q[0][f], w, win[S][f]);
        win[S + 1][f] = mma(q[1][f], w, win[S + 1][f]);
      }
    }
  };
  // z stencil of tile t of row (y, x0) from ring slots S0, S0 + 1, S0 + 2
  // (mod 4). With nz % 4 == 0 every lane's four outputs are all inside or
  // all outside the grid, and the stores go through a buffer descriptor
  // whose range ends at the last x row: lanes past nx fall outside it, lanes
  // past nz get an offset outside it, and the hardware drops both. Each
  // tile then issues the same nine stores on every path, with no branch
  // around them.
  auto zfilter = [&](auto slot, int t, int y, int x0, bool drop) XZM_INLINE {
    constexpr int S0 = decltype(slot)::value;
    f4 acc[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f) acc[f] = f4{0.f, 0.f, 0.f, 0.f};
    const int zo = 16 * t + 4 * j;
    const int xo = x0 + i;
    __amdgpu_buffer_rsrc_t rs;
    unsigned off = 0;
    float *dst = nullptr;
    if constexpr (VEC) {
      const size_t rem = (size_t)(nx - x0) * row_bytes;
      rs = __builtin_amdgcn_make_buffer_rsrc(a.out + (size_t)x0 * (row_bytes / 4), 0,
                                             (int)(rem < 0x7fffffffu ? rem : 0x7fffffffu), kBufWord3);
      off = zo < nz && !drop ? (unsigned)(i * row_bytes + (y * kNF * nz + zo) * 4) : 0x80000000u;
    } else {
      dst = a.out + ((size_t)xo * a.ny + y) * (size_t)(kNF * nz) + zo;
    }
    // three fields at a time, each group stored as soon as it is done
#pragma unroll
    for (int g = 0; g < 3; ++g) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int f = 3 * g; f < 3 * g + 3; ++f) acc[f] = mma(az[c][r], win[(S0 + c) % NR][f][r], acc[f]);
      if constexpr (VEC) {
#pragma unroll
        for (int f = 3 * g; f < 3 * g + 3; ++f)
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, acc[f]), rs, off + f * nz * 4, 0, 0);
      } else if (xo < nx && !drop) {
#pragma unroll
        for (int f = 3 * g; f < 3 * g + 3; ++f)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (zo + r < nz) dst[(size_t)f * nz + r] = acc[f][r];
      }
    }
  };

  // the range starts in row (y, x group xg) at tile ta; every later piece
  // starts a new row at tile 0. A wave whose x tile 4 xg + w lies past the
  // grid (last group when nxt % 4 != 0) runs the tile (4 xg + w) mod nxt
  // with all its stores dropped: its loads stay in bounds and its memory
  // operations keep their count.
  int y, xg, ta;
  {
    const int row = start / p.nct;
    ta = start - row * p.nct;
    y = row / p.nxg;
    xg = row - y * p.nxg;
  }
  auto xtile = [&](int g) XZM_INLINE { return 4 * g + wave < p.nxt ? 4 * g + wave : (4 * g + wave) % p.nxt; };
  int left = end - start;
  target_row(y, xtile(xg));
  nk = ta - 1;
  {
    int xi = nxs;
    unsigned e[2] = {first(nk), first(nk + 1)};
#pragma unroll
    for (int s = 0; s < KS; ++s) load_step(s, xi, e);
  }
  while (left > 0) {
    // piece: tiles [ta, tb) of row (y, xt); pairs of chunks from ta - 1,
    // the last one possibly reaching one chunk past tb
    const int tb = left < p.nct - ta ? ta + left : p.nct;
    left -= tb - ta;
    const int xt = xtile(xg);
    const bool drop = 4 * xg + wave >= p.nxt;
    const int x0 = 16 * xt;
    const float ms = a.mshift[y];
    int k = ta - 1;   // first chunk of the pair in b
    // the pair after k: the next one of this piece, else the first one of
    // the next row, else k again (a harmless reload)
    auto aim = [&]() XZM_INLINE {
      if (k + 2 <= tb) {
        nk = k + 2;
      } else if (left > 0) {
        const bool wrap = xg + 1 == p.nxg;
        target_row(wrap ? y + 1 : y, xtile(wrap ? 0 : xg + 1));
        nk = -1;
      } else {
        nk = k;
      }
    };
    // pair 0 (chunks ta - 1, ta) into slots 0, 1
    aim();
    xfilter(std::integral_constant<int, 0>{}, ms);
    k += 2;
    // pair n (chunks ta - 1 + 2n, ta + 2n) completes tiles ta + 2n - 2 and
    // ta + 2n - 1: the first reads slots 2n - 2 .. 2n, the second 2n - 1 ..
    // 2n + 1 (mod 4)
    bool done = false;
    while (!done) {
      static_for<0, 2>([&](auto q) XZM_INLINE {
        constexpr int S = 2 * ((decltype(q)::value + 1) % 2);   // slots of this pair: S, S + 1
        if (done) return;
        aim();
        xfilter(std::integral_constant<int, S>{}, ms);
        const int t = k - 1;   // first tile this pair completes
        k += 2;
        zfilter(std::integral_constant<int, (S + 2) % NR>{}, t, y, x0, drop);
        if (t + 1 < tb) zfilter(std::integral_constant<int, (S + 3) % NR>{}, t + 1, y, x0, drop);
        if (t + 2 >= tb) done = true;
      });
    }
    if (++xg == p.nxg) {
      xg = 0;
      ++y;
    }
    ta = 0;
  }
}

using KernelFn = void (*)(XzArgs, XzmPlan);

// instances for x stencil steps 5..12, with and without 16-byte stores
template <int KS, bool VEC>
constexpr KernelFn kernel_of() {
  return k_xzm<KS, VEC>;
}
template <bool VEC>
KernelFn pick(int ks) {
  switch (ks) {
    case 5: return kernel_of<5, VEC>();
    case 6: return kernel_of<6, VEC>();
    case 7: return kernel_of<7, VEC>();
    case 8: return kernel_of<8, VEC>();
    case 9: return kernel_of<9, VEC>();
    case 10: return kernel_of<10, VEC>();
    case 11: return kernel_of<11, VEC>();
    case 12: return kernel_of<12, VEC>();
    default: return nullptr;
  }
}
KernelFn pick(int ks, bool vec) { return vec ? pick<true>(ks) : pick<false>(ks); }

}  // namespace

bool xzm_plan(int nx, int ny, int nz, int mx, int mz, XzmPlan *p) {
  const int ks = (16 + 2 * mx + 3) / 4;
  if (mz > 16 || ks > 12) return xzw_plan(nx, ny, nz, mx, mz, p);
  if (nx < 4) return false;
  p->wide = 0;
  if ((long)nx * ny * nz >= (1L << 29)) return false;   // byte offsets below 2^31
  // byte offsets of sixteen output x rows below 2^31 (buffer stores)
  if (16L * ny * 9 * nz * 4 >= (1L << 31)) return false;
  p->ks = ks < 5 ? 5 : ks;
  p->h = 1;
  p->vec = (nz & 3) == 0;
  p->nxt = (nx + 15) / 16;
  p->nxg = (p->nxt + kWaves - 1) / kWaves;
  p->nct = (nz + 15) / 16;
  p->nrow = p->nxg * ny;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return false;
  const KernelFn fn = pick(p->ks, p->vec);
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWaves * 64, 0) != hipSuccess) return false;
  if (per_cu < 1 || ncu < 1) return false;
  // every resident block takes an equal share, at least two positions each
  const long tiles = (long)p->nrow * p->nct;
  const long want = (tiles + 1) / 2;
  const long cap = (long)per_cu * ncu;
  p->nblk = (int)(want < cap ? want : cap);
  return true;
}

hipError_t launch_xzm(const XzArgs &a, const XzmPlan &p, hipStream_t s) {
  if (p.wide) return launch_xzw(a, p, s);
  const KernelFn fn = pick(p.ks, p.vec);
  if (!fn) return hipErrorInvalidValue;
  fn<<<(unsigned)p.nblk, kWaves * 64, 0, s>>>(a, p);
  return hipGetLastError();
}

}  // namespace eles
