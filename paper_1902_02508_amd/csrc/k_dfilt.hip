// The paper's differential filter (Sec. 3, eq. (12)): ubar solves
// (1 - a^2 lap) ubar = u, with spectral second derivatives in the periodic
// x and z directions and the three-point second difference on the
// non-uniform wall-normal nodes of the flow reflected across both walls as
// in eq. (7).
//
// The operator is diagonal in the real Fourier basis of x and z (cosines
// and sines of the grid wavenumbers share the eigenvalue -k^2), so a field
// is transformed along x and along z, every (x coefficient, z coefficient)
// column is then a tridiagonal system in y, solved by elimination with
// factors built once per grid, and the result is transformed back.
//
// Transforms. Node k and node n - k share cos(2 pi s k / n) and carry
// opposite sines, so with e_k = x_k + x_{n-k} and o_k = x_k - x_{n-k}
// (k = 0 .. n/2, index n - k taken mod n) the cosine coefficients are a
// product with e and the sine coefficients a product with o, each about
// half the size of the full transform; the inverse is folded the same way
// (x_k = P_k + Q_k, x_{n-k} = P_k - Q_k with P the cosine and Q the sine
// sum). The products run on the FP32 matrix cores (16x16x4 MFMA) with the
// tables pre-arranged in the A-operand lane order, so one 16-byte load
// gives a lane its table entries of four K steps; the data is the B
// operand, read straight from memory through buffer loads whose count per
// K group is fixed, and the next group is fetched while the current one
// is multiplied.
//
// Stress: u1 is shifted by its plane-mean profile m(y); the nine fields
// u1', u2, u3 and their six products are filtered. Because m depends on y
// alone, the x/z coefficients of m u_j are m times those of u_j, so the
// terms the shift leaves are formed in the solve:
//   F(u1'u_j) + c_j (F(m u_j) - M F(u_j)) = S^-1(p_j + c_j m u_j) - c_j M S^-1(u_j)
// (hats on the right: coefficients; c_1 = 2, c_2 = c_3 = 1; M = F(m)), and
//   ubar_1 = F(u1') + M,  tau_11 = [..]_1 - F(u1')^2 + F(m^2) - M^2,
//   tau_1j = [..]_j - F(u1') F(u_j),  tau_ij = F(u_i u_j) - F(u_i) F(u_j),
// the expansion of u1 = u1' + m, exact for any profile.
#include "eles_internal.h"

namespace eles {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kBufWord3 = 0x00020000;
constexpr unsigned kOOB = 0x80000000u;   // offset past every range: loads 0, stores dropped

__device__ inline f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const float *p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)p, 0, (int)(bytes < 0x7fffffffu ? bytes : 0x7fffffffu),
                                           kBufWord3);
}
__device__ inline float bload(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
}

// |wavenumber| index of real-basis coefficient q of an n-point axis:
// q = 0 .. n/2 are cosines of index q, the rest sines of index q - n/2
__device__ __host__ inline int widx(int q, int n) {
  const int h = n / 2;
  return q <= h ? q : q - h;
}

// ---------------------------------------------------------------- setup

// K index of table column (g, s4) of lane row j. MID order (data read one
// value per lane and step): 1 + 4 (4 g + s4) + j. LAST order (a lane reads
// four consecutive values with one load): 1 + 16 g + 4 j + s4, and the
// sine coefficients of the inverse from the top, hs - (16 g + 4 j + s4),
// so that no group holding a valid index reaches past either end of a row.
__device__ inline int kcol(bool last, int g, int s4, int j) {
  return last ? 1 + 16 * g + 4 * j + s4 : 1 + 4 * (4 * g + s4) + j;
}

// Pre-arranged tables of one axis, entry [tile][g][lane][s4] = M[16 tile +
// lane % 16][kcol(g, s4, lane / 16)], built in FP64 and rounded to FP32.
// Forward (row = coefficient, column = folded node k = 1 .. h), in groups of
// kDTS tiles, the cosine groups first, then the sine groups:
//   cosine s:  w_s cos(2 pi s k / n), halved at k = n/2 (there e_k = 2 x_k),
//              w_s = 1/n at s = 0 and s = n/2, else 2/n;
//   sine s+1:  (2/n) sin(2 pi (s+1) k / n).
// Inverse (row = output node k = 0 .. h, column = coefficient 1 .. h), per
// tile group its P tiles, then its Q tiles: cos(2 pi k s / n) and
// sin(2 pi k s / n).
// The index-0 terms (node x_0 of the forward sums, coefficient C_0 of the
// inverse) are added by the kernels.
__global__ void k_dtab(DAxis ax, bool last, float *fwd, float *inv) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)ax.ks4 * 256;
  const long nf = (long)ax.gf * kDTS * per, ni = 2L * ax.gi * kDTI * per;
  if (e >= nf + ni) return;
  const bool f = e < nf;
  const long e2 = f ? e : e - nf;
  const int tile = (int)(e2 / per);
  const int r = (int)(e2 - (long)tile * per);
  const int g = r >> 8, lane = (r & 255) >> 2, s4 = r & 3;
  const int i = lane & 15, j = lane >> 4;
  const int col = kcol(last, g, s4, j);
  const int n = ax.n, h = ax.h, hs = ax.hs;
  double val = 0.0;
  // angle 2 pi p q / n in units of pi, reduced exactly
  auto angle = [n](long p, long q) { return (double)((2L * p * q) % (2L * n)) / n; };
  if (f) {
    // tile group tg < gc holds cosine tiles tg kDTS + r, the others sine tiles
    const int tg = tile / kDTS, r = tile - tg * kDTS;
    const int ct = tg < ax.gc ? tg * kDTS + r : ax.qc;                // cosine tile, or none
    const int st = tg < ax.gc ? ax.qs : (tg - ax.gc) * kDTS + r;      // sine tile, or none
    if (ct < ax.qc) {
      const int q = 16 * ct + i;
      if (q <= h && col <= h) {
        const double w = (q == 0 || 2 * q == n) ? 1.0 / n : 2.0 / n;
        const double half = 2 * col == n ? 0.5 : 1.0;
        val = w * half * cospi(angle(q, col));
      }
    } else if (st < ax.qs) {
      const int q = 16 * st + i;
      if (q < hs && col <= h) val = (2.0 / n) * sinpi(angle(q + 1, col));
    }
  } else {
    // tile group tg holds its kDTI P tiles, then its kDTI Q tiles
    const int tg = tile / (2 * kDTI), r = tile - tg * 2 * kDTI;
    if (r < kDTI) {
      const int k = 16 * (tg * kDTI + r) + i;
      if (k <= h && col <= h) val = cospi(angle(k, col));
    } else {
      const int k = 16 * (tg * kDTI + r - kDTI) + i;
      const int sc = last ? hs - (16 * g + 4 * j + s4) : col;
      if (k <= h && sc >= 1 && sc <= hs) val = sinpi(angle(k, sc));
    }
  }
  (f ? fwd : inv)[e2] = (float)val;
}

// Second difference on the reflected nodes: d64 [parity 0 = even, 1 = odd]
// [sub, main, super][ny]. Even: every node, the wall's mirror neighbour
// folded onto its reflected twin. Odd: nodes 1 .. ny-2, the wall values
// (zero) dropped.
__global__ void k_dsecond(DView v) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int ny = v.ny;
  if (j >= ny) return;
  const double *y = v.y64;
  double hm, hp;
  if (j == 0) {
    hp = y[1] - y[0];
    hm = hp;
  } else if (j == ny - 1) {
    hm = y[j] - y[j - 1];
    hp = hm;
  } else {
    hm = y[j] - y[j - 1];
    hp = y[j + 1] - y[j];
  }
  const double s = 2.0 / (hm + hp);
  double lo = s / hm, di = -s / hm - s / hp, hi = s / hp;
  double *ev = v.d64, *od = v.d64 + 3 * ny;
  // even
  double el = lo, eh = hi;
  if (j == 0) {
    eh += el;
    el = 0.0;
  }
  if (j == ny - 1) {
    el += eh;
    eh = 0.0;
  }
  ev[j] = el;
  ev[ny + j] = di;
  ev[2 * ny + j] = eh;
  // odd (rows 1 .. ny-2)
  od[j] = (j <= 1) ? 0.0 : lo;
  od[ny + j] = (j == 0 || j == ny - 1) ? 0.0 : di;
  od[2 * ny + j] = (j >= ny - 2) ? 0.0 : hi;
}

// Factors of (1 + a^2 (kx^2 + kz^2)) I - a^2 D for every wavenumber pair
// (sx, sz) and parity: c'_j and 1/den_j of the elimination, and the scaled
// sub-diagonal -a^2 lo_j (FP64 arithmetic, FP32 storage, layout
// [p][sx][y][sz] so that neighbouring z coefficients are adjacent). The
// zero-wavenumber even system is also kept in FP64 for the mean profile.
__global__ void k_dfactor(DView v) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long ncol = (long)(v.hx + 1) * (v.hz + 1);
  if (t >= 2 * ncol) return;
  const int p = (int)(t / ncol);
  const long col = t - p * ncol;
  const int sx = (int)(col / (v.hz + 1)), sz = (int)(col % (v.hz + 1));
  const int ny = v.ny, nzc = v.hz + 1;
  const double a2 = v.a * v.a;
  const double kx = 2.0 * M_PI * sx / v.lx, kz = 2.0 * M_PI * sz / v.lz;
  const double c = 1.0 + a2 * (kx * kx + kz * kz);
  const double *d = v.d64 + (size_t)p * 3 * ny;
  const int j0 = p ? 1 : 0, j1 = p ? ny - 2 : ny - 1;
  const size_t base = ((size_t)p * (v.hx + 1) + sx) * ny * nzc + sz;
  float *cp = v.cp + base;
  float *inv = v.inv + base;
  const bool keep64 = p == 0 && col == 0;
  double cprev = 0.0;
  for (int j = 0; j < ny; ++j) {
    if (j < j0 || j > j1) {
      cp[(size_t)j * nzc] = 0.0f;
      inv[(size_t)j * nzc] = 0.0f;
      continue;
    }
    const double L = -a2 * d[j], Dg = c - a2 * d[ny + j], U = -a2 * d[2 * ny + j];
    const double den = j == j0 ? Dg : Dg - L * cprev;
    const double cj = U / den;
    cp[(size_t)j * nzc] = (float)cj;
    inv[(size_t)j * nzc] = (float)(1.0 / den);
    if (keep64) {
      v.p64[j] = L;
      v.p64[ny + j] = 1.0 / den;
      v.p64[2 * ny + j] = cj;
    }
    cprev = cj;
  }
  if (col == 0)
    for (int j = 0; j < ny; ++j) {
      v.lo32[(size_t)p * ny + j] = (float)(-a2 * d[j]);
      for (int r = 0; r < 3; ++r) v.op32[((size_t)p * 3 + r) * ny + j] = (float)(-a2 * d[r * ny + j]);
    }
}

// ---------------------------------------------------------------- per call

// Shift profile m(y): the mean of u1 over kMeanSlabs evenly spaced x
// planes of each y (FP64 sums). Any profile leaves the stress exact; this
// one removes the bulk of u1 before the products are formed.
__global__ void __launch_bounds__(256) k_dmean(DView v, const float *__restrict__ u1) {
  __shared__ double red[4];
  const int j = blockIdx.x, nz = v.nz;
  const int cnt = kMeanSlabs * nz;
  double sum = 0.0;
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int sl = e / nz, z = e - sl * nz;
    const int x = (int)((long)v.nx * sl / kMeanSlabs);
    sum += (double)u1[((size_t)x * v.ny + j) * nz + z];
  }
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) v.scratch64[j] = ((red[0] + red[1]) + (red[2] + red[3])) / cnt;
}

// M = F(m) and F(m^2) - M^2 from m in scratch64[0 .. ny) (the
// zero-wavenumber even system, FP64); m itself is rounded to FP32 once and
// that value is used everywhere. One thread runs the elimination; for
// ny <= kDProfLds the block first stages m and the FP64 factors in LDS and
// the elimination keeps its intermediate values there (r1 over m, r2 over
// the sub-diagonal, both read once before being overwritten).
constexpr int kDProfLds = 2048;
__device__ inline void dprof_solve(int ny, double *__restrict__ m, double *__restrict__ L,
                                   const double *__restrict__ iv, const double *__restrict__ cp,
                                   float *__restrict__ Mo, float *__restrict__ So) {
  double r1 = 0.0, r2 = 0.0;
  for (int j = 0; j < ny; ++j) {
    const double mj = m[j], lj = L[j], ij = iv[j];
    r1 = (mj - lj * r1) * ij;
    r2 = (mj * mj - lj * r2) * ij;
    m[j] = r1;
    L[j] = r2;
  }
  double x1 = 0.0, x2 = 0.0;
  for (int j = ny - 1; j >= 0; --j) {
    x1 = m[j] - cp[j] * x1;
    x2 = L[j] - cp[j] * x2;
    Mo[j] = (float)x1;
    So[j] = (float)(x2 - x1 * x1);
  }
}
__global__ void __launch_bounds__(256) k_dprof(DView v) {
  extern __shared__ double sd[];   // [4][ny]: m, sub-diagonal, 1/den, c'
  const int ny = v.ny;
  const bool staged = ny <= kDProfLds;
  for (int j = threadIdx.x; j < ny; j += blockDim.x) {
    const float mf = (float)v.scratch64[j];
    v.prof[j] = mf;
    if (staged) {
      sd[j] = (double)mf;
      sd[ny + j] = v.p64[j];
      sd[2 * ny + j] = v.p64[ny + j];
      sd[3 * ny + j] = v.p64[2 * ny + j];
    } else {
      v.scratch64[j] = (double)mf;   // m as used, in FP64
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (staged) {
    dprof_solve(ny, sd, sd + ny, sd + 2 * ny, sd + 3 * ny, v.prof + ny, v.prof + 2 * ny);
  } else {
    // m in scratch64[0 ..), the sub-diagonal copied to scratch64[ny ..)
    for (int j = 0; j < ny; ++j) v.scratch64[ny + j] = v.p64[j];
    dprof_solve(ny, v.scratch64, v.scratch64 + ny, v.p64 + ny, v.p64 + 2 * ny, v.prof + ny, v.prof + 2 * ny);
  }
}

// Arguments of the transform kernels. MID: fields [nb][n][C] transformed
// along the middle axis (columns c contiguous, C = ny nz); LAST: R rows of
// n contiguous values transformed along the row.
struct DT {
  size_t ldsmax;       // LDS-table kernels: largest slice (bytes)
  const float *tab;
  const float *in;
  float *out;
  const float *prof;   // m(y), products only
  DAxis ax;
  int nb;              // MID: fields
  int ny, nz;          // MID products: y of column c is c / nz
  long C;              // MID: columns per field
  long R;              // LAST: rows
  size_t fs;           // MID: field stride (elements)
};

// the two factors of stress field b (0 .. 8): u1', u2, u3, then the
// products u1'u1', u1'u2, u1'u3, u2u2, u2u3, u3u3
__device__ inline void dfield(int b, int &ca, int &cb) {
  ca = b < 3 ? b : (b < 6 ? 0 : (b < 8 ? 1 : 2));
  cb = b < 3 ? b : (b < 6 ? b - 3 : (b == 6 ? 1 : 2));
}

typedef unsigned u4 __attribute__((ext_vector_type(4)));
__device__ inline void bstore4(f4 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, off, 0, 0);
}
__device__ inline f4 bload4(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// table operand: lane offset in a VGPR, tile/group offset in an SGPR
__device__ inline f4 tload(__amdgpu_buffer_rsrc_t r, unsigned lane_off, int soff) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, lane_off, soff, 0));
}

// Lane addressing of the transform kernels: the value of K index k and data
// tile t of this lane is at byte offset k * kstride + loff[t] of the
// descriptor (MID: k is the row of a column; LAST: the position in a row);
// lanes past the data (lv false) use kOOB.
struct Lanes {
  unsigned loff[kDNT];
  bool lv[kDNT];
  unsigned kstride;
};

// What a wave needs of one data group: descriptors of its input (sa; sb
// the second factor of a product) and output, and the lane addressing.
struct Ctx {
  __amdgpu_buffer_rsrc_t sa, sb, dst;
  Lanes L;
  int b, ca, cb;       // MID: field; products: its factors
  float msh[kDNT];     // products: the shift m(y) of each of the lane's columns
};

template <bool LAST, bool PROD>
__device__ __attribute__((always_inline)) inline void make_ctx(const DT &a, long dg, Ctx &c) {
  const int i = threadIdx.x & 15;
  const int n = a.ax.n;
  c.b = c.ca = c.cb = 0;
#pragma unroll
  for (int t = 0; t < kDNT; ++t) c.msh[t] = 0.0f;
  if (LAST) {
    const long r0 = dg * 16 * kDNT;
    const long rows = min((long)16 * kDNT, a.R - r0);
    c.sa = rsrc(a.in + (size_t)r0 * n, (size_t)rows * n * 4);
    c.sb = c.sa;
    c.dst = rsrc(a.out + (size_t)r0 * n, (size_t)rows * n * 4);
    c.L.kstride = 4;
#pragma unroll
    for (int t = 0; t < kDNT; ++t) {
      c.L.lv[t] = 16 * t + i < rows;
      c.L.loff[t] = (unsigned)((16 * t + i) * n * 4);
    }
  } else {
    // data-group indices stay below 2^31 (columns / 16 times fields)
    const int cg = (int)dg / a.nb;
    c.b = (int)dg - cg * a.nb;
    const long c0 = (long)cg * 16 * kDNT;
    const size_t bytes = ((size_t)(n - 1) * a.C + (a.C - c0)) * 4;
    if (PROD) {
      dfield(c.b, c.ca, c.cb);
      c.sa = rsrc(a.in + (size_t)c.ca * a.fs + c0, bytes);
      c.sb = rsrc(a.in + (size_t)c.cb * a.fs + c0, bytes);
    } else {
      c.sa = rsrc(a.in + (size_t)c.b * a.fs + c0, bytes);
      c.sb = c.sa;
    }
    c.dst = rsrc(a.out + (size_t)c.b * a.fs + c0, bytes);
    c.L.kstride = (unsigned)(a.C * 4);
#pragma unroll
    for (int t = 0; t < kDNT; ++t) {
      c.L.lv[t] = c0 + 16 * t + i < a.C;
      c.L.loff[t] = (unsigned)((16 * t + i) * 4);
      // a lane's column (y nz + z) is fixed for the data group, and so is
      // its y (columns past the data take the last row's shift; their
      // values are zero and stay zero)
      if (PROD) c.msh[t] = a.prof[(int)min(c0 + 16 * t + i, (long)a.C - 1) / a.nz];
    }
  }
}

// A wave streams through nd data groups d0, d0 + dstep, ..: the K groups
// of all of them form one sequence, and the loads of the next K group
// (possibly the first of the next data group) are issued before the
// current one is multiplied and, at a data group's end, before its stores
// (stores share the memory counter with loads).
template <class Grp, class LoadF, class CompF>
__device__ __attribute__((always_inline)) inline void stream(long nz, LoadF &load, CompF &compute) {
  Grp G0, G1;
  load(G0);
  __builtin_amdgcn_sched_barrier(0);
  for (long z = 0; z < nz; z += 2) {
    load(G1);
    __builtin_amdgcn_sched_barrier(0);
    compute(G0);
    if (z + 1 >= nz) break;
    load(G0);
    __builtin_amdgcn_sched_barrier(0);
    compute(G1);
  }
}

// Forward transform. Per data group: kDNT data tiles (16 columns or rows
// each) x kDTS coefficient tiles of tile group tg; accumulators start from
// the node-0 term w_q x_0 of the cosines.
// PROD: MID only, the field is formed from u (stress fields, shifted u1).
template <bool LAST, bool PROD, class Tab>
__device__ __attribute__((always_inline)) inline void fwd_stream(const DT &a, long d0, long dstep, long nd, int tg,
                                                                 const Tab &T) {
  const int lane = threadIdx.x & 63, j = lane >> 4;
  const DAxis ax = a.ax;
  const int n = ax.n, h = ax.h, ks4 = ax.ks4;
  const bool cs = tg < ax.gc;   // cosine group (sums x_k + x_{n-k}), else sine group (differences)
  const int tb = cs ? tg * kDTS : (tg - ax.gc) * kDTS;   // first tile of the group in its half
  const int nt = min(kDTS, (cs ? ax.qc : ax.qs) - tb);
  const float sg = cs ? 1.0f : -1.0f;
  const long nz = nd * ks4;

  // the field value from the loaded factor(s) (products: shift u1, multiply)
  auto field = [&](const Ctx &c, float x, float xb, float sh) __attribute__((always_inline)) {
    if (!PROD) return x;
    const float xa = c.ca == 0 ? x - sh : x;
    const float xc = c.cb == 0 ? xb - sh : xb;
    return c.b >= 3 ? xa * xc : xa;
  };

  struct Grp {
    f4 A[Tab::kPre ? kDTS : 1];
    float x[4][kDNT], p[4][kDNT], xb[4][kDNT], pb[4][kDNT];
    float x0[kDNT], x0b[kDNT], msh[kDNT];
  };
  Ctx cl, cc;   // load and multiply cursors
  long kl = 0, kc = 0;
  int gl = 0, gcur = 0;
  make_ctx<LAST, PROD>(a, d0, cl);
  cc = cl;
  f4 acc[kDTS][kDNT];

  auto load = [&](Grp &G) __attribute__((always_inline)) {
    const bool live = kl < nd;
    const Ctx &c = cl;
    if constexpr (Tab::kPre) {
#pragma unroll
      for (int tt = 0; tt < kDTS; ++tt) G.A[tt] = T.get(tt * ks4 + gl);
    }
#pragma unroll
    for (int t = 0; t < kDNT; ++t) {
      const unsigned o0 = live && c.L.lv[t] ? c.L.loff[t] : kOOB;
      G.x0[t] = bload(c.sa, o0);
      G.x0b[t] = PROD ? bload(c.sb, o0) : 0.0f;
      G.msh[t] = c.msh[t];
    }
    if (LAST) {
      // four consecutive nodes k0 .. k0+3 and their partners n-k0-3 .. n-k0
      const int k0 = 1 + 16 * gl + 4 * j;
#pragma unroll
      for (int t = 0; t < kDNT; ++t) {
        const bool ok = live && c.L.lv[t] && k0 <= h;
        const f4 X = bload4(c.sa, ok ? (unsigned)k0 * 4 + c.L.loff[t] : kOOB);
        const f4 P = bload4(c.sa, ok ? (unsigned)(n - k0 - 3) * 4 + c.L.loff[t] : kOOB);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          G.x[s4][t] = X[s4];
          G.p[s4][t] = P[3 - s4];
        }
      }
    } else {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = 1 + 4 * (4 * gl + s4) + j;
#pragma unroll
        for (int t = 0; t < kDNT; ++t) {
          const bool ok = live && c.L.lv[t] && k <= h;
          const unsigned ox = ok ? (unsigned)k * c.L.kstride + c.L.loff[t] : kOOB;
          const unsigned op = ok ? (unsigned)(n - k) * c.L.kstride + c.L.loff[t] : kOOB;
          G.x[s4][t] = bload(c.sa, ox);
          G.p[s4][t] = bload(c.sa, op);
          if (PROD) {
            G.xb[s4][t] = bload(c.sb, ox);
            G.pb[s4][t] = bload(c.sb, op);
          }
        }
      }
    }
    if (++gl == ks4) {
      gl = 0;
      ++kl;
      if (kl < nd) make_ctx<LAST, PROD>(a, d0 + kl * dstep, cl);
    }
  };

  auto compute = [&](Grp &G) __attribute__((always_inline)) {
    const Ctx &c = cc;
    const int g = gcur;
    if (g == 0) {
      // node 0: cosine q gains w_q x_0
#pragma unroll
      for (int t = 0; t < kDNT; ++t) {
        const float x0 = c.L.lv[t] ? field(c, G.x0[t], G.x0b[t], G.msh[t]) : 0.0f;
#pragma unroll
        for (int tt = 0; tt < kDTS; ++tt)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int q = 16 * (tb + tt) + 4 * j + e;
            const float wq = !cs || q > h ? 0.0f : (q == 0 || 2 * q == n) ? 1.0f / n : 2.0f / n;
            acc[tt][t][e] = wq * x0;
          }
      }
    }
    f4 A[kDTS];
#pragma unroll
    for (int tt = 0; tt < kDTS; ++tt) {
      if constexpr (Tab::kPre)
        A[tt] = G.A[tt];
      else
        A[tt] = T.get(tt * ks4 + g);
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      // LAST: a group spans sixteen K indices over lanes and steps; run it whole
      if (!LAST && 4 * g + s4 >= ax.ks) break;
      float bv[kDNT];   // e_k (cosine group) or o_k (sine group)
#pragma unroll
      for (int t = 0; t < kDNT; ++t) {
        float x = G.x[s4][t], p = G.p[s4][t];
        if (PROD) {
          // entries past the data read 0 and must stay 0 after the shift
          const float sh = c.L.lv[t] && kcol(false, g, s4, j) <= h ? G.msh[t] : 0.0f;
          x = field(c, x, G.xb[s4][t], sh);
          p = field(c, p, G.pb[s4][t], sh);
        }
        bv[t] = fmaf(sg, p, x);
      }
#pragma unroll
      for (int tt = 0; tt < kDTS; ++tt) {
        if (tt >= nt) break;
#pragma unroll
        for (int t = 0; t < kDNT; ++t) acc[tt][t] = mma(A[tt][s4], bv[t], acc[tt][t]);
      }
    }
    if (g == ks4 - 1) {
      // coefficient rows: cosine q at q (q <= h), sine q+1 at h + 1 + q (q < hs)
      const int qend = cs ? h + 1 : ax.hs;   // valid q < qend
      const int rb = cs ? 0 : h + 1;
#pragma unroll
      for (int tt = 0; tt < kDTS; ++tt) {
        if (tt >= nt) break;
        const int q0 = 16 * (tb + tt) + 4 * j;
        if (LAST && 16 * (tb + tt) + 16 <= qend) {
          // LAST, whole tile valid: a lane's four outputs are adjacent
#pragma unroll
          for (int t = 0; t < kDNT; ++t)
            bstore4(acc[tt][t], c.dst, c.L.lv[t] ? (unsigned)(rb + q0) * 4 + c.L.loff[t] : kOOB);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int q = q0 + e;
#pragma unroll
            for (int t = 0; t < kDNT; ++t) {
              const unsigned off = q < qend && c.L.lv[t] ? (unsigned)(rb + q) * c.L.kstride + c.L.loff[t] : kOOB;
              bstore(acc[tt][t][e], c.dst, off);
            }
          }
        }
      }
    }
    if (++gcur == ks4) {
      gcur = 0;
      ++kc;
      if (kc < nd) make_ctx<LAST, PROD>(a, d0 + kc * dstep, cc);
    }
  };
  stream<Grp>(nz, load, compute);
}

// Inverse transform. Per data group: kDNT data tiles x kDTI output node
// tiles, each with a cosine (P) and a sine (Q) accumulator; P starts from
// the coefficient C_0.
template <bool LAST, class Tab>
__device__ __attribute__((always_inline)) inline void inv_stream(const DT &a, long d0, long dstep, long nd, int tg,
                                                                 const Tab &T) {
  const int lane = threadIdx.x & 63, j = lane >> 4;
  const DAxis ax = a.ax;
  const int n = ax.n, h = ax.h, hs = ax.hs, ks4 = ax.ks4;
  const int t0 = tg * kDTI;
  const int nt = min(kDTI, ax.qc - t0);
  const long nz = nd * ks4;

  struct Grp {
    f4 AP[Tab::kPre ? kDTI : 1], AQ[Tab::kPre ? kDTI : 1];
    float c[4][kDNT], s[4][kDNT];
    float c0[kDNT];
  };
  Ctx cl, cc;
  long kl = 0, kc = 0;
  int gl = 0, gcur = 0;
  make_ctx<LAST, false>(a, d0, cl);
  cc = cl;
  f4 P[kDTI][kDNT], Q[kDTI][kDNT];

  auto load = [&](Grp &G) __attribute__((always_inline)) {
    const bool live = kl < nd;
    const Ctx &c = cl;
    if constexpr (Tab::kPre) {
#pragma unroll
      for (int tt = 0; tt < kDTI; ++tt) {
        G.AP[tt] = T.get(tt * ks4 + gl);
        G.AQ[tt] = T.get((kDTI + tt) * ks4 + gl);
      }
    }
#pragma unroll
    for (int t = 0; t < kDNT; ++t) G.c0[t] = bload(c.sa, live && c.L.lv[t] ? c.L.loff[t] : kOOB);
    if (LAST) {
      // cosines s0 .. s0+3 upward, sines s1 .. s1-3 downward (row h + s)
      const int s0 = 1 + 16 * gl + 4 * j, s1 = hs - 16 * gl - 4 * j;
#pragma unroll
      for (int t = 0; t < kDNT; ++t) {
        const bool ok = live && c.L.lv[t];
        const f4 C = bload4(c.sa, ok && s0 <= h ? (unsigned)s0 * 4 + c.L.loff[t] : kOOB);
        const f4 S = bload4(c.sa, ok && s1 >= 1 ? (unsigned)(h + s1 - 3) * 4 + c.L.loff[t] : kOOB);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          G.c[s4][t] = C[s4];
          G.s[s4][t] = S[3 - s4];
        }
      }
    } else {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int sidx = 1 + 4 * (4 * gl + s4) + j;   // cosine s (row s), sine s (row h + s)
#pragma unroll
        for (int t = 0; t < kDNT; ++t) {
          const bool ok = live && c.L.lv[t];
          const unsigned oc = ok && sidx <= h ? (unsigned)sidx * c.L.kstride + c.L.loff[t] : kOOB;
          const unsigned os = ok && sidx <= hs ? (unsigned)(h + sidx) * c.L.kstride + c.L.loff[t] : kOOB;
          G.c[s4][t] = bload(c.sa, oc);
          G.s[s4][t] = bload(c.sa, os);
        }
      }
    }
    if (++gl == ks4) {
      gl = 0;
      ++kl;
      if (kl < nd) make_ctx<LAST, false>(a, d0 + kl * dstep, cl);
    }
  };

  auto compute = [&](Grp &G) __attribute__((always_inline)) {
    const Ctx &c = cc;
    const int g = gcur;
    if (g == 0) {
#pragma unroll
      for (int t = 0; t < kDNT; ++t)
#pragma unroll
        for (int tt = 0; tt < kDTI; ++tt) {
          P[tt][t] = f4{G.c0[t], G.c0[t], G.c0[t], G.c0[t]};
          Q[tt][t] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    f4 AP[kDTI], AQ[kDTI];
#pragma unroll
    for (int tt = 0; tt < kDTI; ++tt) {
      if constexpr (Tab::kPre) {
        AP[tt] = G.AP[tt];
        AQ[tt] = G.AQ[tt];
      } else {
        AP[tt] = T.get(tt * ks4 + g);
        AQ[tt] = T.get((kDTI + tt) * ks4 + g);
      }
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      // LAST: a group spans sixteen K indices over lanes and steps; run it whole
      if (!LAST && 4 * g + s4 >= ax.ks) break;
#pragma unroll
      for (int tt = 0; tt < kDTI; ++tt) {
        if (tt >= nt) break;
#pragma unroll
        for (int t = 0; t < kDNT; ++t) {
          P[tt][t] = mma(AP[tt][s4], G.c[s4][t], P[tt][t]);
          Q[tt][t] = mma(AQ[tt][s4], G.s[s4][t], Q[tt][t]);
        }
      }
    }
    if (g == ks4 - 1) {
      // node k = P + Q, node n - k = P - Q
#pragma unroll
      for (int tt = 0; tt < kDTI; ++tt) {
        if (tt >= nt) break;
        const int kt = 16 * (t0 + tt);
        if (LAST && kt >= 1 && kt + 16 <= hs + 1) {
          // LAST, whole tile valid for both halves: k0 .. k0+3 upward and
          // n-k0-3 .. n-k0 downward are adjacent
          const int k0 = kt + 4 * j;
#pragma unroll
          for (int t = 0; t < kDNT; ++t) {
            const f4 sp = P[tt][t] + Q[tt][t], sm = P[tt][t] - Q[tt][t];
            bstore4(sp, c.dst, c.L.lv[t] ? (unsigned)k0 * 4 + c.L.loff[t] : kOOB);
            bstore4(f4{sm[3], sm[2], sm[1], sm[0]}, c.dst,
                    c.L.lv[t] ? (unsigned)(n - k0 - 3) * 4 + c.L.loff[t] : kOOB);
          }
          continue;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = 16 * (t0 + tt) + 4 * j + e;
#pragma unroll
          for (int t = 0; t < kDNT; ++t) {
            const float pv = P[tt][t][e], qv = Q[tt][t][e];
            const unsigned o1 = c.L.lv[t] && k <= h ? (unsigned)k * c.L.kstride + c.L.loff[t] : kOOB;
            const unsigned o2 =
                c.L.lv[t] && k >= 1 && k <= hs ? (unsigned)(n - k) * c.L.kstride + c.L.loff[t] : kOOB;
            bstore(pv + qv, c.dst, o1);
            bstore(pv - qv, c.dst, o2);
          }
        }
      }
    }
    if (++gcur == ks4) {
      gcur = 0;
      ++kc;
      if (kc < nd) make_ctx<LAST, false>(a, d0 + kc * dstep, cc);
    }
  };
  stream<Grp>(nz, load, compute);
}

// Table accessors: the slice of one tile group (forward: kDTS tiles;
// inverse: kDTI P tiles then kDTI Q tiles), tile-major, 1 KB per (tile, K
// group); get(tile * ks4 + g) gives this lane's four entries.
struct TabG {   // from memory through a descriptor: fetched with the data
  static constexpr bool kPre = true;
  __amdgpu_buffer_rsrc_t r;
  unsigned lane_off;
  __device__ f4 get(int tg) const { return tload(r, lane_off, tg * 1024); }
};
struct TabL {   // from LDS: read when the group is multiplied
  static constexpr bool kPre = false;
  const float *p;   // slice + lane * 4
  __device__ f4 get(int tg) const { return *(const f4 *)(p + tg * 256); }
};

__device__ inline long data_groups(const DT &a, bool last) {
  return last ? (a.R + 16 * kDNT - 1) / (16 * kDNT) : (a.C + 16 * kDNT - 1) / (16 * kDNT) * a.nb;
}

// One wave per (data group, tile group), the table read from memory.
template <bool LAST, bool PROD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_dfwd(DT a) {
  const long w = (long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int ngr = a.ax.gf;
  if (w >= data_groups(a, LAST) * ngr) return;
  const long dg = w / ngr;
  const int tg = (int)(w - dg * ngr);
  const TabG T{rsrc(a.tab + (size_t)tg * kDTS * a.ax.ks4 * 256, (size_t)kDTS * a.ax.ks4 * 1024),
               (unsigned)(threadIdx.x & 63) * 16};
  fwd_stream<LAST, PROD>(a, dg, 1, 1, tg, T);
}
template <bool LAST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_dinv(DT a) {
  const long w = (long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int ngr = a.ax.gi;
  if (w >= data_groups(a, LAST) * ngr) return;
  const long dg = w / ngr;
  const int tg = (int)(w - dg * ngr);
  const TabG T{rsrc(a.tab + (size_t)tg * 2 * kDTI * a.ax.ks4 * 256, (size_t)2 * kDTI * a.ax.ks4 * 1024),
               (unsigned)(threadIdx.x & 63) * 16};
  inv_stream<LAST>(a, dg, 1, 1, tg, T);
}

// Persistent blocks of kDWaves waves, nbt blocks per tile group: the
// block's table slice is staged in LDS once and its waves walk a
// contiguous range of data groups.
constexpr int kDWaves = 8;
__device__ inline void stage_table(const float *src, int nfloat, float *lds) {
  const f4 *s4 = (const f4 *)src;
  f4 *d4 = (f4 *)lds;
  for (int e = threadIdx.x; e < nfloat / 4; e += blockDim.x) d4[e] = s4[e];
  __syncthreads();
}
template <bool LAST, bool PROD>
__global__ void __launch_bounds__(64 * kDWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_dfwd_lds(DT a, int nbt) {
  extern __shared__ float tl[];
  const int tg = blockIdx.x / nbt, bi = blockIdx.x - tg * nbt;
  if (tg >= a.ax.gf) return;   // whole block
  const int nfl = kDTS * a.ax.ks4 * 256;
  stage_table(a.tab + (size_t)tg * nfl, nfl, tl);
  const long ndg = data_groups(a, LAST);
  const long d0 = ndg * bi / nbt, d1 = ndg * (bi + 1) / nbt;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const TabL T{tl + (threadIdx.x & 63) * 4};
  if (d0 + wave < d1) fwd_stream<LAST, PROD>(a, d0 + wave, kDWaves, (d1 - d0 - wave + kDWaves - 1) / kDWaves, tg, T);
}
template <bool LAST>
__global__ void __launch_bounds__(64 * kDWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_dinv_lds(DT a, int nbt) {
  extern __shared__ float tl[];
  const int tg = blockIdx.x / nbt, bi = blockIdx.x - tg * nbt;
  if (tg >= a.ax.gi) return;   // whole block
  const int nfl = 2 * kDTI * a.ax.ks4 * 256;
  stage_table(a.tab + (size_t)tg * nfl, nfl, tl);
  const long ndg = data_groups(a, LAST);
  const long d0 = ndg * bi / nbt, d1 = ndg * (bi + 1) / nbt;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const TabL T{tl + (threadIdx.x & 63) * 4};
  if (d0 + wave < d1) inv_stream<LAST>(a, d0 + wave, kDWaves, (d1 - d0 - wave + kDWaves - 1) / kDWaves, tg, T);
}

// Tridiagonal solves in y, out of place: in, out [f][qx][y][qz]. Thread
// per (system, qx, qz). Plain: system f of parity (pmask >> f) & 1 (1:
// odd). SGS: six systems over the nine stress fields; systems 0 .. 2 carry
// field g (u_j) and field 3 + g (u1'u_j) with the shift terms folded in.
constexpr int kCH = 8;   // y values loaded together
template <bool SGS>
__global__ void __launch_bounds__(256) k_dsolve(DView v, const float *__restrict__ in, float *__restrict__ out,
                                                int nf, unsigned pmask) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nx = v.nx, ny = v.ny, nz = v.nz;
  const long ncolf = (long)nx * nz;
  const int ns = SGS ? 6 : nf;
  if (t >= ns * ncolf) return;
  const int g = (int)(t / ncolf);
  const long col = t - g * ncolf;
  const int qx = (int)(col / nz), qz = (int)(col - (long)qx * nz);
  int fa, fb = -1, p;
  float cj = 0.0f;
  if (SGS) {
    fa = g < 3 ? g : g + 3;
    if (g < 3) fb = g + 3;
    p = (g == 1 || g == 4) ? 1 : 0;
    cj = g == 0 ? 2.0f : 1.0f;
  } else {
    fa = g;
    p = (pmask >> g) & 1;
  }
  const bool two = fb >= 0;
  const int nzc = v.hz + 1;
  const size_t fbase = ((size_t)p * (v.hx + 1) + widx(qx, nx)) * ny * nzc + widx(qz, nz);
  const float *__restrict__ cp = v.cp + fbase;
  const float *__restrict__ iv = v.inv + fbase;
  const float *__restrict__ lo = v.lo32 + (size_t)p * ny;
  const float *__restrict__ m = v.prof;
  const float *__restrict__ M = v.prof + ny;
  const size_t fs = (size_t)nx * ny * nz;
  const size_t cbase = (size_t)qx * ny * nz + qz;
  const float *__restrict__ xa = in + (size_t)fa * fs + cbase;
  const float *__restrict__ xb = in + (size_t)(two ? fb : fa) * fs + cbase;
  float *ya = out + (size_t)fa * fs + cbase;
  float *yb = out + (size_t)(two ? fb : fa) * fs + cbase;
  const int j0 = p, j1 = ny - 1 - p;
  // forward elimination: r_j = (d_j - lo_j r_{j-1}) / den_j (lo_{j0} = 0);
  // the next chunk of y values is requested before this one is eliminated
  struct FC {
    float da[kCH], db[kCH], iv[kCH], l[kCH], m[kCH];
  };
  auto fload = [&](int jb, FC &c) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < kCH; ++k) {
      const int jj = min(jb + k, j1);
      c.da[k] = xa[(size_t)jj * nz];
      c.db[k] = two ? xb[(size_t)jj * nz] : 0.0f;
      c.iv[k] = iv[(size_t)jj * nzc];
      c.l[k] = lo[jj];
      c.m[k] = m[jj];
    }
  };
  float ra = 0.0f, rb = 0.0f;
  auto fstep = [&](int jb, const FC &c) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < kCH; ++k) {
      if (jb + k > j1) break;
      const int jj = jb + k;
      ra = (c.da[k] - c.l[k] * ra) * c.iv[k];
      ya[(size_t)jj * nz] = ra;
      if (two) {
        rb = ((c.db[k] + cj * c.m[k] * c.da[k]) - c.l[k] * rb) * c.iv[k];
        yb[(size_t)jj * nz] = rb;
      }
    }
  };
  {
    FC A, B;
    fload(j0, A);
    for (int jb = j0; jb <= j1; jb += 2 * kCH) {
      fload(jb + kCH, B);
      fstep(jb, A);
      if (jb + kCH > j1) break;
      fload(jb + 2 * kCH, A);
      fstep(jb + kCH, B);
    }
  }
  // back substitution: x_j = r_j - c'_j x_{j+1} (c'_{j1} = 0); a chunk's
  // r values are read before the rows below it are overwritten
  struct BC {
    float r1[kCH], r2[kCH], cp[kCH], M[kCH];
  };
  auto bload = [&](int jt, BC &c) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < kCH; ++k) {
      const int jj = max(jt - k, j0);
      c.r1[k] = ya[(size_t)jj * nz];
      c.r2[k] = two ? yb[(size_t)jj * nz] : 0.0f;
      c.cp[k] = cp[(size_t)jj * nzc];
      c.M[k] = M[jj];
    }
  };
  float xa1 = 0.0f, xb1 = 0.0f;
  auto bstep = [&](int jt, const BC &c) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < kCH; ++k) {
      if (jt - k < j0) break;
      const int jj = jt - k;
      xa1 = c.r1[k] - c.cp[k] * xa1;
      ya[(size_t)jj * nz] = xa1;
      if (two) {
        xb1 = c.r2[k] - c.cp[k] * xb1;
        yb[(size_t)jj * nz] = xb1 - cj * c.M[k] * xa1;
      }
    }
  };
  {
    BC A, B;
    bload(j1, A);
    for (int jt = j1; jt >= j0; jt -= 2 * kCH) {
      bload(jt - kCH, B);
      bstep(jt, A);
      if (jt - kCH < j0) break;
      bload(jt - 2 * kCH, A);
      bstep(jt - kCH, B);
    }
  }
  if (p) {
    ya[0] = 0.0f;
    ya[(size_t)(ny - 1) * nz] = 0.0f;
    if (two) {
      yb[0] = 0.0f;
      yb[(size_t)(ny - 1) * nz] = 0.0f;
    }
  }
}

constexpr int kDXC = 16;   // x planes per block of the plane-sum kernels

// The operator itself in the coefficient space, out of place: for every
// (field, qx, qz) column, out_j = (1 + a^2 (kx^2 + kz^2)) x_j - a^2 (D x)_j
// with the reflected three-point difference D of the field's parity; odd
// fields are zero on the wall rows. FP64 wavenumber term, FP32 products.
__global__ void __launch_bounds__(256) k_dapply(DView v, const float *__restrict__ in, float *__restrict__ out,
                                                int nf, unsigned pmask) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nx = v.nx, ny = v.ny, nz = v.nz;
  const long ncolf = (long)nx * nz;
  if (t >= nf * ncolf) return;
  const int f = (int)(t / ncolf);
  const long col = t - f * ncolf;
  const int qx = (int)(col / nz), qz = (int)(col - (long)qx * nz);
  const int p = (pmask >> f) & 1;
  const double kx = 2.0 * M_PI * widx(qx, nx) / v.lx, kz = 2.0 * M_PI * widx(qz, nz) / v.lz;
  const float c = (float)(1.0 + v.a * v.a * (kx * kx + kz * kz));
  const float *__restrict__ lo = v.op32 + (size_t)p * 3 * ny;
  const float *__restrict__ mi = lo + ny;
  const float *__restrict__ hi = lo + 2 * ny;
  const size_t base = (size_t)f * nx * ny * nz + (size_t)qx * ny * nz + qz;
  const float *__restrict__ x = in + base;
  float *__restrict__ y = out + base;
  const int j0 = p, j1 = ny - 1 - p;
  // sliding window x_{j-1}, x_j, x_{j+1}; neighbours outside j0 .. j1 carry
  // zero coefficients
  float xm = 0.0f, x0 = x[(size_t)j0 * nz];
  for (int jb = j0; jb <= j1; jb += kCH) {
    float nxt[kCH];
#pragma unroll
    for (int c8 = 0; c8 < kCH; ++c8) nxt[c8] = x[(size_t)min(jb + c8 + 1, j1) * nz];
#pragma unroll
    for (int c8 = 0; c8 < kCH; ++c8) {
      const int j = jb + c8;
      if (j > j1) break;
      const float xp = j < j1 ? nxt[c8] : 0.0f;
      y[(size_t)j * nz] = (c + mi[j]) * x0 + (lo[j] * xm + hi[j] * xp);
      xm = x0;
      x0 = xp;
    }
  }
  if (p) {
    y[0] = 0.0f;
    y[(size_t)(ny - 1) * nz] = 0.0f;
  }
}

// Errors of eqs. (13)-(15), partial sums. Block (xc, y) over kDXC x planes:
// q = 0: sum (a1/ut_a - b1/ut_d)^2; 1: sum (b1/ut_d)^2; 2 + 4 i + (0 .. 3):
// sums of a_i, a_i^2, b_i, b_i^2 (FP64), part[(q ny + y) nxc + xc].
constexpr int kEQ = 14;
__global__ void __launch_bounds__(256) k_eparts(DView v, const float *__restrict__ la, const float *__restrict__ db,
                                                double inv_ua, double inv_ud, double *__restrict__ part) {
  __shared__ double red[4][kEQ];
  const int xc = blockIdx.x, y = blockIdx.y, nxc = gridDim.x;
  const int nz = v.nz, ny = v.ny;
  const int x0 = xc * kDXC, x1 = min(v.nx, x0 + kDXC);
  const size_t n = (size_t)v.nx * ny * nz;
  double s[kEQ];
#pragma unroll
  for (int q = 0; q < kEQ; ++q) s[q] = 0.0;
  const int cnt = (x1 - x0) * nz;
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int xo = e / nz, z = e - xo * nz;
    const size_t t = ((size_t)(x0 + xo) * ny + y) * nz + z;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double a = la[i * n + t], b = db[i * n + t];
      if (i == 0) {
        const double d = a * inv_ua - b * inv_ud;
        s[0] += d * d;
        s[1] += (b * inv_ud) * (b * inv_ud);
      }
      s[2 + 4 * i] += a;
      s[3 + 4 * i] += a * a;
      s[4 + 4 * i] += b;
      s[5 + 4 * i] += b * b;
    }
  }
#pragma unroll
  for (int q = 0; q < kEQ; ++q)
    for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < kEQ; ++q) red[threadIdx.x >> 6][q] = s[q];
  __syncthreads();
  if (threadIdx.x < kEQ) {
    const int q = threadIdx.x;
    part[((size_t)q * ny + y) * nxc + xc] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  }
}

// The partial sums over x chunks in order, the profiles, and the trapezoid
// integrals over y (bounded trapezoid on the nodes used); threads take y
// nodes, a block reduction adds their terms: out[0] eq. (13) over the
// channel; out[1] eq. (14) and out[2 .. 4] eq. (15) for u1, u2, u3 over the
// lower half, y <= 0 (wall to centreline).
constexpr int kET = 10;   // integral terms
__global__ void __launch_bounds__(256) k_efinal(DView v, const double *__restrict__ part, int nxc, double inv_ua,
                                                double inv_ud, double *__restrict__ out) {
  __shared__ double red[4][kET];
  const int ny = v.ny;
  const double *y = v.y64;
  const double cnt = (double)v.nx * v.nz;
  double acc[kET];   // n13, d13, n14, d14, n15[3], d15[3]
#pragma unroll
  for (int q = 0; q < kET; ++q) acc[q] = 0.0;
  for (int j = threadIdx.x; j < ny; j += blockDim.x) {
    double sm[kEQ];
#pragma unroll
    for (int q = 0; q < kEQ; ++q) {
      double t = 0.0;
      for (int c = 0; c < nxc; ++c) t += part[((size_t)q * ny + j) * nxc + c];
      sm[q] = t;
    }
    const double lo = j > 0 ? y[j] - y[j - 1] : 0.0;
    const double hi = j < ny - 1 ? y[j + 1] - y[j] : 0.0;
    const double w = 0.5 * (lo + hi);
    acc[0] += w * sm[0];
    acc[1] += w * sm[1];
    if (y[j] <= 0.0) {
      // half-channel trapezoid: the upper neighbour only if it is in the half
      const double wh = 0.5 * (lo + (j < ny - 1 && y[j + 1] <= 0.0 ? hi : 0.0));
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double ma = sm[2 + 4 * i] / cnt, qa = sm[3 + 4 * i] / cnt;
        const double mb = sm[4 + 4 * i] / cnt, qb = sm[5 + 4 * i] / cnt;
        const double ra = sqrt(fmax(qa - ma * ma, 0.0)) * inv_ua, rb = sqrt(fmax(qb - mb * mb, 0.0)) * inv_ud;
        if (i == 0) {
          const double d = ma * inv_ua - mb * inv_ud;
          acc[2] += wh * d * d;
          acc[3] += wh * (mb * inv_ud) * (mb * inv_ud);
        }
        acc[4 + i] += wh * (ra - rb) * (ra - rb);
        acc[7 + i] += wh * rb * rb;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kET; ++q)
    for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < kET; ++q) red[threadIdx.x >> 6][q] = acc[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[kET];
    for (int q = 0; q < kET; ++q) t[q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    out[0] = sqrt(t[0] / t[1]);
    out[1] = sqrt(t[2] / t[3]);
    for (int i = 0; i < 3; ++i) out[2 + i] = sqrt(t[4 + i] / t[7 + i]);
  }
}

// ubar and tau from the nine filtered fields g. Block (xc, y): the points
// of kDXC x planes at wall-normal index y; with part, also the FP64 sums of
// the nine outputs over those points, part[(q ny + y) nxc + xc].
__global__ void __launch_bounds__(256) k_depi(DView v, const float *__restrict__ g, float *__restrict__ ubar,
                                              float *__restrict__ tau, double *__restrict__ part) {
  __shared__ double red[4][kDFields];
  const int xc = blockIdx.x, y = blockIdx.y, nxc = gridDim.x;
  const int nz = v.nz, ny = v.ny;
  const int x0 = xc * kDXC, x1 = min(v.nx, x0 + kDXC);
  const size_t n = (size_t)v.nx * ny * nz;
  const float M = v.prof[ny + y], S = v.prof[2 * ny + y];
  double sum[kDFields];
#pragma unroll
  for (int q = 0; q < kDFields; ++q) sum[q] = 0.0;
  const int cnt = (x1 - x0) * nz;
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int xo = e / nz, z = e - xo * nz;
    const size_t t = ((size_t)(x0 + xo) * ny + y) * nz + z;
    float G[kDFields];
#pragma unroll
    for (int f = 0; f < kDFields; ++f) G[f] = g[f * n + t];
    float o[kDFields];
    o[0] = G[0] + M;
    o[1] = G[1];
    o[2] = G[2];
    o[3] = (G[3] - G[0] * G[0]) + S;
    o[4] = G[4] - G[0] * G[1];
    o[5] = G[5] - G[0] * G[2];
    o[6] = G[6] - G[1] * G[1];
    o[7] = G[7] - G[1] * G[2];
    o[8] = G[8] - G[2] * G[2];
#pragma unroll
    for (int q = 0; q < 3; ++q) ubar[q * n + t] = o[q];
#pragma unroll
    for (int q = 0; q < 6; ++q) tau[q * n + t] = o[3 + q];
#pragma unroll
    for (int q = 0; q < kDFields; ++q) sum[q] += (double)o[q];
  }
  if (!part) return;   // uniform over the grid
#pragma unroll
  for (int q = 0; q < kDFields; ++q)
    for (int off = 32; off > 0; off >>= 1) sum[q] += __shfl_xor(sum[q], off);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < kDFields; ++q) red[threadIdx.x >> 6][q] = sum[q];
  __syncthreads();
  if (threadIdx.x < kDFields) {
    const int q = threadIdx.x;
    part[((size_t)q * ny + y) * nxc + xc] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  }
}

// stats[q][y] = (sum over chunks of part) / (nx nz), chunks in order
__global__ void k_dstat(const double *__restrict__ part, int nqy, int nxc, double inv, double *__restrict__ stats) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nqy) return;
  double s = 0.0;
  for (int c = 0; c < nxc; ++c) s += part[(size_t)i * nxc + c];
  stats[i] = s * inv;
}

unsigned grid_of(long work, int per) { return (unsigned)((work + per - 1) / per); }

DT targs(const DView &v, bool x, const float *tab, const float *in, float *out, int nb) {
  DT a;
  a.ldsmax = v.ldsmax;
  a.tab = tab;
  a.in = in;
  a.out = out;
  a.prof = v.prof;
  a.ax = x ? v.ax : v.az;
  a.nb = nb;
  a.ny = v.ny;
  a.nz = v.nz;
  a.C = (long)v.ny * v.nz;
  a.R = (long)nb * v.nx * v.ny;
  a.fs = (size_t)v.nx * v.ny * v.nz;
  return a;
}

size_t fwd_slice_bytes(const DAxis &ax) { return (size_t)kDTS * ax.ks4 * 1024; }
size_t inv_slice_bytes(const DAxis &ax) { return (size_t)2 * kDTI * ax.ks4 * 1024; }
long host_data_groups(const DT &a, bool last) {
  return last ? (a.R + 16 * kDNT - 1) / (16 * kDNT) : (a.C + 16 * kDNT - 1) / (16 * kDNT) * a.nb;
}
// blocks per tile group of the persistent kernels: one block per CU in all
int blocks_per_group(int ngroups) { return max(1, 256 / ngroups); }

template <bool LAST, bool PROD>
void fwd(const DT &a, hipStream_t s) {
  const size_t lds = fwd_slice_bytes(a.ax);
  if (lds <= a.ldsmax) {
    const int nbt = blocks_per_group(a.ax.gf);
    k_dfwd_lds<LAST, PROD><<<nbt * a.ax.gf, 64 * kDWaves, lds, s>>>(a, nbt);
  } else {
    k_dfwd<LAST, PROD><<<grid_of(host_data_groups(a, LAST) * a.ax.gf, 4), 256, 0, s>>>(a);
  }
}
template <bool LAST>
void inv(const DT &a, hipStream_t s) {
  const size_t lds = inv_slice_bytes(a.ax);
  if (lds <= a.ldsmax) {
    const int nbt = blocks_per_group(a.ax.gi);
    k_dinv_lds<LAST><<<nbt * a.ax.gi, 64 * kDWaves, lds, s>>>(a, nbt);
  } else {
    k_dinv<LAST><<<grid_of(host_data_groups(a, LAST) * a.ax.gi, 4), 256, 0, s>>>(a);
  }
}

// the four transforms and the solve: in -> out through w0, w1 (x forward
// in -> w1, z forward w1 -> w0, solve w0 -> w1, z inverse w1 -> w0, x
// inverse w0 -> out; out may be w1)
// Timing events of one call: ev[2 p] before and ev[2 p + 1] after pass p
// (DPass), or null; a null entry leaves that pass untimed.
void mark(const hipEvent_t *ev, int idx, hipStream_t s) {
  if (ev && ev[idx]) (void)hipEventRecord(ev[idx], s);
}

template <bool SGS, bool APPLY = false>
hipError_t run_filter(const DView &v, const float *in, int nf, unsigned pmask, float *w0, float *w1, float *out,
                      hipStream_t s, const hipEvent_t *ev) {
  const int nb = SGS ? kDFields : nf;
  // fast transforms (k_sder.hip) where both lengths allow, else the folded
  // table products on the matrix cores
  const bool fast = v.rx.nrad && v.rz.nrad;   // odd stress fields: u2, u1'u2, u2u3 (mask 0x92)
  const long fs = (long)v.nx * v.ny * v.nz;
  mark(ev, 2 * kDPassXf, s);
  if (fast)
    launch_rfft(v.rx, false, false, in, w1, v.prof, fs, fs, v.nx, v.ny, v.nz, nb, SGS, 0u, s);
  else
    fwd<false, SGS>(targs(v, true, v.fx, in, w1, nb), s);
  mark(ev, 2 * kDPassXf + 1, s);
  mark(ev, 2 * kDPassZf, s);
  if (fast)
    launch_rfft(v.rz, true, false, w1, w0, nullptr, fs, fs, v.nx, v.ny, v.nz, nb, false, 0u, s);
  else
    fwd<true, false>(targs(v, false, v.fz, w1, w0, nb), s);
  mark(ev, 2 * kDPassZf + 1, s);
  const int ns = SGS ? 6 : nf;
  mark(ev, 2 * kDPassY, s);
  if (APPLY)
    k_dapply<<<grid_of((long)nf * v.nx * v.nz, 256), 256, 0, s>>>(v, w0, w1, nf, pmask);
  else
    k_dsolve<SGS><<<grid_of((long)ns * v.nx * v.nz, 256), 256, 0, s>>>(v, w0, w1, nf, pmask);
  mark(ev, 2 * kDPassY + 1, s);
  mark(ev, 2 * kDPassZi, s);
  if (fast)
    launch_rfft(v.rz, true, true, w1, w0, nullptr, fs, fs, v.nx, v.ny, v.nz, nb, false, 0u, s);
  else
    inv<true>(targs(v, false, v.iz, w1, w0, nb), s);
  mark(ev, 2 * kDPassZi + 1, s);
  mark(ev, 2 * kDPassXi, s);
  if (fast)
    launch_rfft(v.rx, false, true, w0, out, nullptr, fs, fs, v.nx, v.ny, v.nz, nb, false, SGS ? 0x92u : pmask, s);
  else
    inv<false>(targs(v, true, v.ix, w0, out, nb), s);
  mark(ev, 2 * kDPassXi + 1, s);
  return hipGetLastError();
}

}  // namespace

// The LDS-table kernels stage up to the device's per-block LDS: the
// dynamic-LDS limit of each instance is raised to it (64 KB without).
hipError_t dfilter_lds_limit(DView &v) {
  int dev = 0, bytes = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return hipErrorUnknown;
  v.ldsmax = 65536;
  if (bytes > 65536) {
    const void *k[] = {(const void *)k_dfwd_lds<false, false>, (const void *)k_dfwd_lds<false, true>,
                       (const void *)k_dfwd_lds<true, false>, (const void *)k_dinv_lds<false>,
                       (const void *)k_dinv_lds<true>};
    for (const void *f : k)
      if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
        return hipSuccess;   // keep 64 KB
    v.ldsmax = (size_t)bytes;
  }
  return hipSuccess;
}

hipError_t launch_dsetup(const DView &v, hipStream_t s) {
  for (int x = 0; x < 2; ++x) {
    const DAxis &ax = x ? v.ax : v.az;
    const long ne = (long)dtab_fwd_floats(ax) + (long)dtab_inv_floats(ax);
    k_dtab<<<grid_of(ne, 256), 256, 0, s>>>(ax, x == 0, x ? v.fx : v.fz, x ? v.ix : v.iz);
  }
  k_dsecond<<<grid_of(v.ny, 256), 256, 0, s>>>(v);
  const long ncol = 2L * (v.hx + 1) * (v.hz + 1);
  k_dfactor<<<grid_of(ncol, 64), 64, 0, s>>>(v);
  return hipGetLastError();
}

// fields [nf][nx][ny][nz] in `in` -> filtered in `out`; w0, w1: workspaces
// of nf fields, distinct from in and out
hipError_t launch_dfilter(const DView &v, const float *in, int nf, unsigned pmask, float *w0, float *w1, float *out,
                          hipStream_t s, const hipEvent_t *ev) {
  return run_filter<false>(v, in, nf, pmask, w0, w1, out, s, ev);
}

hipError_t launch_dinverse(const DView &v, const float *in, int nf, unsigned pmask, float *w0, float *w1,
                           float *out, hipStream_t s, const hipEvent_t *ev) {
  return run_filter<false, true>(v, in, nf, pmask, w0, w1, out, s, ev);
}

long derr_parts(const DView &v) { return (long)kEQ * v.ny * ((v.nx + kDXC - 1) / kDXC); }

hipError_t launch_derrors(const DView &v, const float *les, const float *dns, double utau_les, double utau_dns,
                          double *part, double *out, hipStream_t s) {
  const int nxc = (v.nx + kDXC - 1) / kDXC;
  k_eparts<<<dim3(nxc, v.ny), 256, 0, s>>>(v, les, dns, 1.0 / utau_les, 1.0 / utau_dns, part);
  k_efinal<<<1, 256, 0, s>>>(v, part, nxc, 1.0 / utau_les, 1.0 / utau_dns, out);
  return hipGetLastError();
}

// u [3][nx][ny][nz] -> ubar [3], tau [6]; w0, w1: workspaces of nine
// fields; part: dsgs_parts doubles; stats: FP64 [9][ny] plane means of
// ubar and tau, or null
hipError_t launch_dsgs(const DView &v, const float *u, float *w0, float *w1, float *ubar, float *tau,
                       double *part, double *stats, hipStream_t s, const hipEvent_t *ev) {
  mark(ev, 2 * kDPassShift, s);
  k_dmean<<<v.ny, 256, 0, s>>>(v, u);
  const size_t lds = v.ny <= kDProfLds ? (size_t)4 * v.ny * sizeof(double) : 0;
  k_dprof<<<1, 256, lds, s>>>(v);
  mark(ev, 2 * kDPassShift + 1, s);
  hipError_t e = run_filter<true>(v, u, kDFields, 0u, w0, w1, w1, s, ev);
  if (e != hipSuccess) return e;
  const int nxc = (v.nx + kDXC - 1) / kDXC;
  mark(ev, 2 * kDPassEpi, s);
  k_depi<<<dim3(nxc, v.ny), 256, 0, s>>>(v, w1, ubar, tau, stats ? part : nullptr);
  if (stats) {
    const int nqy = kDFields * v.ny;
    k_dstat<<<grid_of(nqy, 256), 256, 0, s>>>(part, nqy, nxc, 1.0 / ((double)v.nx * v.nz), stats);
  }
  mark(ev, 2 * kDPassEpi + 1, s);
  return hipGetLastError();
}

long dsgs_parts(const DView &v) { return (long)kDFields * v.ny * ((v.nx + kDXC - 1) / kDXC); }

}  // namespace eles
