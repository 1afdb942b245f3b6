// y pass of the stress mode, staged through LDS, with persistent blocks.
//
// The wall-normal rows are split into groups of consecutive 16-row output
// tiles. A block keeps one group for its whole life and walks (x, 16-column
// z strip) pencils. For each pencil the rows of the nine x/z-filtered
// fields that the group's band needs are staged from HBM into LDS (16-byte
// loads; every input element crosses HBM once) and the twelve matrix-core
// products of the stress expansion (the relations are listed in k_y.hip)
// are split evenly over four waves, three each:
//   wave 0: W+ X0 -> Y0;  C+ X0, W+ X3 -> Y3 = 2 (C+ X0) + W+ X3
//   wave 1: W- X1 -> Y1;  C- X1, W- X4 -> Y4
//   wave 2: W+ X2 -> Y2;  C+ X2, W+ X5 -> Y5
//   wave 3: W+ X6 -> Y6;  W- X7 -> Y7;  W+ X8 -> Y8
// with FP32 accumulators in registers.
//
// Roles. Waves 0-3 only compute: LDS reads and matrix instructions, no
// global memory operation, so they never wait on HBM. Waves 4-7 do all the
// HBM traffic: they form ubar and tau of the previous pencil from its
// products in LDS and store them (16-byte stores), request the next
// pencil's rows into registers, and move those rows to LDS while the
// compute waves publish the current products. On this hardware a wave that
// reuses the registers of a pending store, or waits for a load issued
// after stores, waits for those stores too (one in-order counter), so
// keeping the stores away from the matrix waves is what lets the two
// streams overlap. Per pencil n, between two block barriers:
//   phase 1: compute waves: products of n from X; I/O waves: load n+1
//            into registers, epilogue of n-1 from Y;
//   phase 2: compute waves: products of n to Y; I/O waves: rows of n+1
//            to X.
// The group's operator tiles and mean-shift profiles are copied to LDS once.
//
// Plane sums: each I/O thread keeps FP64 sums of its (row, 4-column) slot
// over all pencils of its block (quad DPP exchanges add the four slots of a
// row) and the block writes them once at the end: partials are
// [quantity][row][block of the group], reduced over blocks by k_stats in a
// fixed order.
//
// K order inside the matrix products: a tile's columns are walked in
// chunks of 16 from a 4-aligned start chosen on the host (the walk ends by
// ny rounded up to 4 where it can, so the staged rows cover every chunk);
// within a chunk, lane group g supplies columns kc + 4g + s to the product
// of slice s = 0..3: a lane's four operator values of the chunk are one
// float4 (stored in lane order in LDS), its field values come from staged
// rows kc + 4g + s. The staged row stride (nine fields of 16 columns plus 4
// pad floats) puts the four lane groups on disjoint banks. Operator columns
// outside a tile's band are zero, so the chunk padding adds nothing.
#include "eles_internal.h"

namespace eles {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
// word 3 of a raw buffer descriptor on gfx9-family parts (32-bit data
// format, no swizzle)
constexpr int kBufWord3 = 0x00020000;

constexpr int RS = kYsRow;
constexpr int kSlots = 36;        // float4 slots per staged row: 9 fields x 4
constexpr int kIo = 256;          // I/O threads (waves 4..7)
constexpr int kBlock = 512;
constexpr int kMaxT = 3;          // tiles per group
// staged float4 slots per I/O thread held in registers (KR, a template
// parameter): the smallest instantiated count that covers the widest group,
// so the commit normally needs no load of its own
constexpr int kKRs[] = {10, 14, 18};
static_assert(16 * kMaxT * 4 <= kIo, "one epilogue slot per I/O thread");
static_assert(kMaxT <= kYsMaxTiles, "tile bound");

__device__ inline f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Lane exchange of an FP64 value inside each quad (DPP quad_perm CTRL).
template <int CTRL>
__device__ inline double quad_perm(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the four lanes of a quad, FP64; every lane gets the total.
__device__ inline double quad_sum(double v) {
  v += quad_perm<0xB1>(v);   // lanes [1,0,3,2]
  v += quad_perm<0x4E>(v);   // lanes [2,3,0,1]
  return v;
}

struct Pencil {
  int x, strip;
};

// Float4 slot q of a pencil's staged rows [kb, kb + nrow): the load is
// unconditional (a clamped, valid address); *zero reports that the slot is
// past ny, past nz or past the last slot, so that the caller can replace
// the value by zeros when it writes LDS. Applying that select right after
// the load would make every load wait for its data before the next issues.
template <bool VEC>
__device__ inline f4 load_slot(const YArgs &a, Pencil m, int kb, int nrow, int q, bool *zero) {
  const int nq = nrow * kSlots;
  const bool qok = q < nq;
  q = qok ? q : nq - 1;
  const int row = q / kSlots, rem = q - row * kSlots;
  const int f = rem >> 2, zl = 4 * (rem & 3);
  const int z0 = m.strip * kYTileN;
  const bool rok = kb + row < a.ny;
  if (VEC) {
    // through a buffer descriptor of the pencil's x slab: 32-bit offsets,
    // and rows past ny or columns past nz read as zeros (offset outside)
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(a.in + (size_t)m.x * a.in_xs), 0, (int)(a.in_xs * 4), kBufWord3);
    const bool ok = qok && rok && z0 + zl < a.nz;
    const unsigned off = ok ? (unsigned)(((kb + row) * a.in_ks + f * a.in_fs + z0 + zl) * 4) : 0x80000000u;
    *zero = false;
    return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
  }
  const float *p = a.in + (size_t)m.x * a.in_xs + (size_t)(kb + (rok ? row : 0)) * a.in_ks +
                   (size_t)f * a.in_fs + z0;
  // ragged z: four scalar loads, columns past nz zeroed here (rare shape)
  f4 v;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const bool ok = rok && z0 + zl + e < a.nz;
    const float t = p[ok ? zl + e : 0];
    v[e] = ok ? t : 0.0f;
  }
  *zero = !rok;
  return v;
}

__device__ inline void store_slot(float *sx, int q, const f4 &v) {
  const int row = q / kSlots, rem = q - row * kSlots;
  *reinterpret_cast<f4 *>(sx + row * RS + (rem >> 2) * 16 + 4 * (rem & 3)) = v;
}

template <bool VEC, int KR>
__device__ inline unsigned prefetch(const YArgs &a, Pencil m, int kb, int nrow, int io, f4 (&r)[KR]) {
  unsigned zmask = 0;
#pragma unroll
  for (int u = 0; u < KR; ++u) {
    bool z;
    r[u] = load_slot<VEC>(a, m, kb, nrow, u * kIo + io, &z);
    zmask |= (unsigned)z << u;
  }
  return zmask;
}

// Registers to LDS, then any slots past the register window straight from HBM.
template <bool VEC, int KR>
__device__ inline void commit(const YArgs &a, Pencil m, int kb, int nrow, int io, const f4 (&r)[KR],
                              unsigned zmask, float *sx) {
  const int nq = nrow * kSlots;
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < KR; ++u) {
    const int q = u * kIo + io;
    if (q < nq) store_slot(sx, q, (zmask >> u) & 1u ? zero : r[u]);
  }
  for (int base = KR * kIo; base < nq; base += KR * kIo) {
    f4 v[KR];
    unsigned zm = 0;
#pragma unroll
    for (int u = 0; u < KR; ++u) {
      bool z;
      v[u] = load_slot<VEC>(a, m, kb, nrow, base + u * kIo + io, &z);
      zm |= (unsigned)z << u;
    }
#pragma unroll
    for (int u = 0; u < KR; ++u) {
      const int q = base + u * kIo + io;
      if (q < nq) store_slot(sx, q, (zm >> u) & 1u ? zero : v[u]);
    }
  }
}

// LDS layout of a block: operator tiles [4 ops][group chunks][64 lanes][4],
// staged rows X [lds_rows][RS], products Y [16 kMaxT][RS], then M and S of
// the group's rows [2][16 kMaxT].
template <bool VEC, int KR>
__global__ void __launch_bounds__(kBlock, 1) k_ys(YArgs a, YsPlan pl) {
  extern __shared__ float lds[];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool iow = wave >= 4;
  const int io = tid - kIo;                   // I/O thread index (I/O waves)
  const int lane = tid & 63, col = lane & 15, grp = lane >> 4;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int g = lb % pl.ngroup, bg = lb / pl.ngroup;
  const int nbg = gridDim.x / pl.ngroup;   // the host launches a multiple of ngroup blocks
  const int npen = a.nx * a.n16;
  const int kb = pl.kb[g], nrow = pl.nrow[g], t0 = pl.tile0[g], nt = pl.ntile[g];
  const int ch0 = pl.chunk0[g], nch = pl.nchunk[g];
  float *sa = lds;
  float *sx = sa + (size_t)4 * pl.max_chunks * 256;
  float *sy = sx + (size_t)pl.lds_rows * RS;
  float *sm = sy + (size_t)16 * kMaxT * RS;
  const int ybase = t0 * 16;
  const int yrows = min(16 * nt, a.ny - ybase);
  if (bg >= npen) return;   // uniform: more blocks than pencils

  // ---- operator tiles (lane order) and profiles of the group
  for (int q0 = 0; q0 < 4 * nch * 64; q0 += 4 * kBlock) {
    f4 v[4];
    int dst[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int q = q0 + u * kBlock + tid;
      dst[u] = q < 4 * nch * 64 ? q : -1;
      q = q < 4 * nch * 64 ? q : 0;
      const int L = q & 63, j = (q >> 6) % nch, op = (q >> 6) / nch;
      const int e = pl.chunk[ch0 + j];
      const int kc = e & 0xffff, t = (e >> 16) & 0xff;
      v[u] = *reinterpret_cast<const f4 *>(a.a32[op] + (size_t)((t0 + t) * 16 + (L & 15)) * a.kpad + kc +
                                           4 * (L >> 4));
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (dst[u] >= 0) *reinterpret_cast<f4 *>(sa + 4 * dst[u]) = v[u];
  }
  for (int r = tid; r < 16 * kMaxT; r += kBlock) {
    const int i = ybase + r;
    sm[r] = r < yrows ? a.prof32[a.mpad + i] : 0.0f;
    sm[16 * kMaxT + r] = r < yrows ? a.prof32[2 * a.mpad + i] : 0.0f;
  }

  int p = bg;
  if (!iow) {
    // ===== compute waves: products of each pencil, X -> Y
    int op0, op1, op2, f0, f1, f2;
    if (wave == 3) {
      op0 = 0, f0 = 6, op1 = 1, f1 = 7, op2 = 0, f2 = 8;
    } else {
      const int wo = wave == 1 ? 1 : 0;   // W- for the odd fields u2 and u1 u2
      op0 = wo, f0 = wave, op1 = 2 + wo, f1 = wave, op2 = wo, f2 = wave + 3;
    }
    const float *Aop[3] = {sa + ((size_t)op0 * nch * 64 + lane) * 4, sa + ((size_t)op1 * nch * 64 + lane) * 4,
                           sa + ((size_t)op2 * nch * 64 + lane) * 4};

    const float *B0 = sx + (4 * grp - kb) * RS + f0 * 16 + col;
    const float *B1 = sx + (4 * grp - kb) * RS + f1 * 16 + col;
    const float *B2 = sx + (4 * grp - kb) * RS + f2 * 16 + col;
    __syncthreads();   // operator tiles and profiles are in LDS
    __syncthreads();   // the first pencil's rows are in LDS
    while (true) {
      const bool more = p + nbg < npen;
      // ---- phase 1: products, a flat walk over the group's chunks,
      // software pipelined one chunk deep (the next chunk's LDS fragments
      // are requested before the current chunk's products; fences keep
      // that order)
      f4 acct[kMaxT][3];
#pragma unroll
      for (int t = 0; t < kMaxT; ++t)
#pragma unroll
        for (int q = 0; q < 3; ++q) acct[t][q] = f4{0.f, 0.f, 0.f, 0.f};
      f4 acc[3] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
      auto fetch = [&](f4 (&w)[3], float (&bv)[12], int j) {
        const int kc = pl.chunk[ch0 + j] & 0xffff;
#pragma unroll
        for (int k = 0; k < 3; ++k) w[k] = *reinterpret_cast<const f4 *>(Aop[k] + (size_t)j * 256);
        const int r = kc * RS;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          bv[3 * s] = B0[r + s * RS];
          bv[3 * s + 1] = B1[r + s * RS];
          bv[3 * s + 2] = B2[r + s * RS];
        }
      };
      auto mmas = [&](const f4 (&w)[3], const float (&bv)[12]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          acc[0] = mma(w[0][s], bv[3 * s], acc[0]);
          acc[1] = mma(w[1][s], bv[3 * s + 1], acc[1]);
          acc[2] = mma(w[2][s], bv[3 * s + 2], acc[2]);
        }
      };
      // after chunk j: a finished tile moves to its accumulators (register
      // selects, not an indexed store, which would live in scratch)
      auto retire = [&](int j) {
        const int e = pl.chunk[ch0 + j];
        if (e >> 24) {
          const int t = (e >> 16) & 0xff;
#pragma unroll
          for (int q = 0; q < kMaxT; ++q)
#pragma unroll
            for (int k = 0; k < 3; ++k) acct[q][k] = q == t ? acc[k] : acct[q][k];
#pragma unroll
          for (int k = 0; k < 3; ++k) acc[k] = f4{0.f, 0.f, 0.f, 0.f};
        }
      };
      {
        f4 wa[3], wb[3];
        float ba[12], bb[12];
        fetch(wa, ba, 0);
        int j = 0;
        while (true) {
          fetch(wb, bb, j + 1 < nch ? j + 1 : j);
          __builtin_amdgcn_sched_barrier(0);
          mmas(wa, ba);
          __builtin_amdgcn_sched_barrier(0);
          retire(j);
          if (++j == nch) break;
          fetch(wa, ba, j + 1 < nch ? j + 1 : j);
          __builtin_amdgcn_sched_barrier(0);
          mmas(wb, bb);
          __builtin_amdgcn_sched_barrier(0);
          retire(j);
          if (++j == nch) break;
        }
      }
      __syncthreads();
      // ---- phase 2: products to Y, [row - ybase][f][16]
#pragma unroll
      for (int tt = 0; tt < kMaxT; ++tt) {
        if (tt < nt) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rr = 16 * tt + 4 * grp + r;
            if (rr < yrows) {
              float *d = sy + rr * RS + col;
              if (wave == 3) {
                d[6 * 16] = acct[tt][0][r];
                d[7 * 16] = acct[tt][1][r];
                d[8 * 16] = acct[tt][2][r];
              } else {
                const float c1 = wave == 0 ? 2.0f * acct[tt][1][r] : acct[tt][1][r];
                d[wave * 16] = acct[tt][0][r];
                d[(wave + 3) * 16] = c1 + acct[tt][2][r];
              }
            }
          }
        }
      }
      __syncthreads();
      if (!more) break;
      p += nbg;
    }
    return;
  }

  // ===== I/O waves: HBM in (rows of the next pencil) and out (ubar, tau)
  // epilogue slot: row lr of the group, columns 4 n4 .. 4 n4 + 3
  const int lr = io >> 2, n4 = io & 3;
  const bool slot = lr < yrows;
  double psum[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) psum[q] = 0.0;
  const size_t N = (size_t)a.nx * a.ny * a.nz;

  // epilogue of pencil m from Y: ubar, tau and this slot's plane sums
  auto epilogue = [&](Pencil m) {
    if (!slot) return;
    const int i = ybase + lr;
    const int z = m.strip * kYTileN + 4 * n4;
    const float *yp = sy + lr * RS + 4 * n4;
    f4 y[9];
#pragma unroll
    for (int f = 0; f < 9; ++f) y[f] = *reinterpret_cast<const f4 *>(yp + 16 * f);
    const float mi = sm[lr], si = sm[16 * kMaxT + lr];
    f4 o[9];
    o[0] = y[0] + mi;
    o[1] = y[1];
    o[2] = y[2];
    o[3] = (y[3] - y[0] * y[0]) + si;
    o[4] = y[4] - y[0] * y[1];
    o[5] = y[5] - y[0] * y[2];
    o[6] = y[6] - y[1] * y[1];
    o[7] = y[7] - y[1] * y[2];
    o[8] = y[8] - y[2] * y[2];
    const int nc = min(4, a.nz - z);   // valid columns of this slot (may be <= 0)
    const size_t off = ((size_t)m.x * a.ny + i) * a.nz + z;
    if (VEC) {
      if (nc > 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) *reinterpret_cast<f4 *>(a.ubar + q * N + off) = o[q];
#pragma unroll
        for (int q = 0; q < 6; ++q) *reinterpret_cast<f4 *>(a.tau + q * N + off) = o[3 + q];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (e < nc) {
#pragma unroll
          for (int q = 0; q < 3; ++q) a.ubar[q * N + off + e] = o[q][e];
#pragma unroll
          for (int q = 0; q < 6; ++q) a.tau[q * N + off + e] = o[3 + q][e];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      double s = 0.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) s += e < nc ? (double)o[q][e] : 0.0;
      psum[q] += quad_sum(s);
    }
  };

  Pencil cur{p / a.n16, p % a.n16};
  f4 rv[KR];
  unsigned zm = prefetch<VEC, KR>(a, cur, kb, nrow, io, rv);
  __syncthreads();   // operator tiles and profiles are in LDS
  commit<VEC, KR>(a, cur, kb, nrow, io, rv, zm, sx);
  __syncthreads();
  bool have_prev = false;
  Pencil prev = cur;
  while (true) {
    const int pn = p + nbg;
    const bool more = pn < npen;
    const Pencil nxt = more ? Pencil{pn / a.n16, pn % a.n16} : cur;
    // ---- phase 1: next rows in flight, epilogue of the previous pencil
    // (unconditional: the last pencil re-reads itself, which keeps the
    // compiler's count of outstanding memory operations exact)
    zm = prefetch<VEC, KR>(a, nxt, kb, nrow, io, rv);
    if (have_prev) epilogue(prev);
    __syncthreads();
    // ---- phase 2: next rows to X
    if (more) commit<VEC, KR>(a, nxt, kb, nrow, io, rv, zm, sx);
    __syncthreads();
    prev = cur;
    have_prev = true;
    if (!more) break;
    p = pn;
    cur = nxt;
  }
  epilogue(prev);
  if (a.part && slot && n4 == 0) {
#pragma unroll
    for (int q = 0; q < 9; ++q) a.part[((size_t)q * a.ny + ybase + lr) * nbg + bg] = psum[q];
  }
}

template <bool VEC>
const void *ys_fn(int kr) {
  if (!VEC) return (const void *)k_ys<false, 10>;
  switch (kr) {
    case 10: return (const void *)k_ys<true, 10>;
    case 14: return (const void *)k_ys<true, 14>;
    default: return (const void *)k_ys<true, 18>;
  }
}

// register window of the plan: the smallest instantiated KR with
// KR * kIo >= the widest group's staged slots (else the largest; the commit
// then loads the remainder itself)
int ys_kr(const YsPlan &p) {
  int slots = 0;
  for (int g = 0; g < p.ngroup; ++g) slots = max(slots, p.nrow[g] * kSlots);
  for (int kr : kKRs)
    if (kr * kIo >= slots) return kr;
  return kKRs[2];
}

// ragged nz (scalar loads, rare shapes) keeps the smallest window
int ys_kr(const YsPlan &p, int nz) { return nz % 4 == 0 ? ys_kr(p) : kKRs[0]; }

const void *ys_pick(const YsPlan &p, int nz) {
  const int kr = ys_kr(p, nz);
  return (nz % 4) == 0 ? ys_fn<true>(kr) : ys_fn<false>(kr);
}

}  // namespace

int ys_max_tiles() { return kMaxT; }

size_t ys_lds_bytes(const YsPlan &p) {
  return ((size_t)4 * p.max_chunks * 256 + (size_t)(p.lds_rows + 16 * kMaxT) * kYsRow + 2 * 16 * kMaxT) *
         sizeof(float);
}

int ys_grid(const YsPlan &p, int nz, int npencils) {
  const size_t lds = ys_lds_bytes(p);
  const void *fn = ys_pick(p, nz);
  if (lds > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  int per = 0, dev = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kBlock, lds) != hipSuccess || per < 1) return 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
    return 0;
  long perg = (long)per * ncu / p.ngroup;   // blocks per group
  if (perg > npencils) perg = npencils;
  return perg < 1 ? 0 : (int)(perg * p.ngroup);
}

hipError_t launch_ys(const YArgs &a, const YsPlan &p, hipStream_t s) {
  const size_t lds = ys_lds_bytes(p);
  if (p.nblk < p.ngroup || p.nblk % p.ngroup) return hipErrorInvalidValue;
  const int kr = ys_kr(p, a.nz);
  if (a.nz % 4 == 0) {
    switch (kr) {
      case 10: k_ys<true, 10><<<(unsigned)p.nblk, kBlock, lds, s>>>(a, p); break;
      case 14: k_ys<true, 14><<<(unsigned)p.nblk, kBlock, lds, s>>>(a, p); break;
      default: k_ys<true, 18><<<(unsigned)p.nblk, kBlock, lds, s>>>(a, p); break;
    }
  } else {
    k_ys<false, 10><<<(unsigned)p.nblk, kBlock, lds, s>>>(a, p);
  }
  return hipGetLastError();
}

}  // namespace eles
