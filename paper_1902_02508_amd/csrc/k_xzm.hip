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
// from registers, with no exchange. The wave keeps the 2H + 1 chunks that
// one z tile reads (H = ceil(mz / 16)) in a ring of register slots; the
// chunk loop is unrolled by the ring length, so every slot is static.
//
// Loads: while step s of a chunk forms its products, the velocities of
// step s of the next chunk are requested into the same registers, so each
// load has a whole chunk of matrix work to arrive.
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

template <int KS, int H, bool VEC>
__global__ void __launch_bounds__(kWaves * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) k_xzm(XzArgs a, XzmPlan p) {
  constexpr int NW = 2 * H + 1;   // chunks one z tile reads
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, j = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gw = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave;
  const int nw = gridDim.x * kWaves;
  const int total = p.nrow * p.nct;
  const int start = (int)((long)gw * total / nw), end = (int)((long)(gw + 1) * total / nw);
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

  // where the next chunk's velocities come from: first x row of this lane
  // (wrapped), plane offset y nz, chunk index
  int nxs, nyz, nk;
  auto target_row = [&](int y, int xt) XZM_INLINE {
    nxs = wrapi(16 * xt - mx + j, nx);
    nyz = y * nz;
  };
  // element offset of the target chunk's first row; the modulo runs only
  // for chunks that wrap around the periodic z direction
  auto first = [&]() XZM_INLINE -> unsigned {
    int zc = 16 * nk + zrow;
    if (nk < 0 || 16 * nk + 16 > nz) zc = wrapi(zc, nz);
    return (unsigned)(nxs * plane + nyz + zc);
  };
  float b[KS][3];
  auto load_step = [&](int s, int &xi, unsigned &e) XZM_INLINE {
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

  f4 win[NW][kNF];
  // x stencil of the chunk whose velocities are in b, into ring slot S,
  // requesting the velocities of the current target into b step by step
  auto xfilter = [&](auto slot, float ms) XZM_INLINE {
    constexpr int S = decltype(slot)::value;
    int xi = nxs;
    unsigned e = first();
#pragma unroll
    for (int f = 0; f < kNF; ++f) win[S][f] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const float v0 = b[s][0] - ms, v1 = b[s][1], v2 = b[s][2];
      const float q[kNF] = {v0, v1, v2, v0 * v0, v0 * v1, v0 * v2, v1 * v1, v1 * v2, v2 * v2};
      load_step(s, xi, e);
      // keep this step's loads here, a whole chunk ahead of their use
      __builtin_amdgcn_sched_barrier(0);
      const float w = bx[s];
#pragma unroll
      for (int f = 0; f < kNF; ++f) win[S][f] = mma(q[f], w, win[S][f]);
    }
  };
  // z stencil of tile t of row (y, x0) whose newest chunk sits in slot S.
  // With nz % 4 == 0 every lane's four outputs are all inside or all outside
  // the grid, and the stores go through a buffer descriptor whose range ends
  // at the last x row: lanes past nx fall outside it, lanes past nz get an
  // offset outside it, and the hardware drops both. Each tile then issues
  // the same nine stores on every path, with no branch around them.
  auto zfilter = [&](auto slot, int t, int y, int x0) XZM_INLINE {
    constexpr int S = decltype(slot)::value;
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
      off = zo < nz ? (unsigned)(i * row_bytes + (y * kNF * nz + zo) * 4) : 0x80000000u;
    } else {
      dst = a.out + ((size_t)xo * a.ny + y) * (size_t)(kNF * nz) + zo;
    }
    // three fields at a time, each group stored as soon as it is done
#pragma unroll
    for (int g = 0; g < 3; ++g) {
#pragma unroll
      for (int c = 0; c < NW; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int f = 3 * g; f < 3 * g + 3; ++f) acc[f] = mma(az[c][r], win[(S + 1 + c) % NW][f][r], acc[f]);
      if constexpr (VEC) {
#pragma unroll
        for (int f = 3 * g; f < 3 * g + 3; ++f)
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, acc[f]), rs, off + f * nz * 4, 0, 0);
      } else if (xo < nx) {
#pragma unroll
        for (int f = 3 * g; f < 3 * g + 3; ++f)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (zo + r < nz) dst[(size_t)f * nz + r] = acc[f][r];
      }
    }
  };

  // the wave's range starts in row (y, xt) at tile ta; every later piece
  // starts a new row at tile 0
  int y, xt, ta;
  {
    const int row = start / p.nct;
    ta = start - row * p.nct;
    y = row / p.nxt;
    xt = row - y * p.nxt;
  }
  int left = end - start;
  target_row(y, xt);
  nk = ta - H;
  {
    int xi = nxs;
    unsigned e = first();
#pragma unroll
    for (int s = 0; s < KS; ++s) load_step(s, xi, e);
  }
  while (left > 0) {
    // piece: tiles [ta, tb) of row (y, xt), chunks [ta - H, tb + H)
    const int tb = left < p.nct - ta ? ta + left : p.nct;
    left -= tb - ta;
    const int x0 = 16 * xt;
    const float ms = a.mshift[y];
    const int ke = tb + H;
    int k = ta - H;
    // the chunk after k: the next one of this piece, else the first one of
    // the next row, else k again (a harmless reload)
    auto aim = [&]() XZM_INLINE {
      if (k + 1 < ke) {
        nk = k + 1;
      } else if (left > 0) {
        const bool wrap = xt + 1 == p.nxt;
        target_row(wrap ? y + 1 : y, wrap ? 0 : xt + 1);
        nk = -H;
      } else {
        nk = k;
      }
    };
    // chunks ta - H .. ta + H into slots 0 .. 2H
    static_for<0, NW>([&](auto q) XZM_INLINE {
      aim();
      xfilter(q, ms);
      ++k;
    });
    // each step: z stencil of the tile whose last chunk is the newest one,
    // then the x stencil of the next chunk. Every step ends with the next
    // chunk's loads, also on entry, so the waits for them count the same
    // stores on every path.
    bool done = false;
    while (!done) {
      static_for<0, NW>([&](auto q) XZM_INLINE {
        constexpr int S = (2 * H + decltype(q)::value) % NW;
        if (done) return;
        zfilter(std::integral_constant<int, S>{}, k - 1 - H, y, x0);
        if (k == ke) {
          done = true;
          return;
        }
        aim();
        xfilter(std::integral_constant<int, (S + 1) % NW>{}, ms);
        ++k;
      });
    }
    if (++xt == p.nxt) {
      xt = 0;
      ++y;
    }
    ta = 0;
  }
}

using KernelFn = void (*)(XzArgs, XzmPlan);

// instances for x stencil steps 5..12 (H = 1), with and without 16-byte stores
template <int KS, bool VEC>
constexpr KernelFn kernel_of() {
  return k_xzm<KS, 1, VEC>;
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
  if (mz > 16 || ks > 12 || nx < 4) return false;
  if ((long)nx * ny * nz >= (1L << 29)) return false;   // byte offsets below 2^31
  // byte offsets of sixteen output x rows below 2^31 (buffer stores)
  if (16L * ny * 9 * nz * 4 >= (1L << 31)) return false;
  p->ks = ks < 5 ? 5 : ks;
  p->h = 1;
  p->vec = (nz & 3) == 0;
  p->nxt = (nx + 15) / 16;
  p->nct = (nz + 15) / 16;
  p->nrow = p->nxt * ny;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return false;
  const KernelFn fn = pick(p->ks, p->vec);
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWaves * 64, 0) != hipSuccess) return false;
  if (per_cu < 1 || ncu < 1) return false;
  // every resident wave takes an equal share, at least two tiles each
  const long tiles = (long)p->nrow * p->nct;
  const long want = (tiles + 2 * kWaves - 1) / (2 * kWaves);
  const long cap = (long)per_cu * ncu;
  p->nblk = (int)(want < cap ? want : cap);
  return true;
}

hipError_t launch_xzm(const XzArgs &a, const XzmPlan &p, hipStream_t s) {
  const KernelFn fn = pick(p.ks, p.vec);
  if (!fn) return hipErrorInvalidValue;
  fn<<<(unsigned)p.nblk, kWaves * 64, 0, s>>>(a, p);
  return hipGetLastError();
}

}  // namespace eles
