// Spectral derivatives of the closure features along the periodic x and z
// directions, by fast Fourier transforms.
//
// The feature is the derivative of the trigonometric interpolant of a line
// of n nodes with period L: transform, multiply coefficient m by i k_m with
// k_m = 2 pi m / L for m < n/2 and 2 pi (m - n) / L for m > n/2 (zero for
// the Nyquist mode of even n), transform back. The operator is real, so two
// real lines travel as the real and imaginary parts of one complex line and
// come back as their two derivatives.
//
// The transforms are the self-sorting (Stockham) mixed-radix factorisation
// of n into radices 16, 8, 4, 2, 3, 5. A pass of radix R, with Ns the
// product of the radices before it, takes for every j < n/R the inputs
// j + r n/R (r < R), turns input r by w^(r k n/(Ns R)) with k = j mod Ns and
// w = exp(-+2 pi i/n), applies the R-point DFT and writes output q to
// (j - k) R + k + q Ns. After the last pass the coefficients are in natural
// order, and item j of that pass holds coefficients j + q n/R: exactly the
// inputs of item j of an inverse pass of the same radix with Ns = 1, so the
// derivative factors are applied in registers and the inverse transform
// (radices in reverse order) starts there without an exchange.
//
// One block holds P complex lines (2P real lines) in LDS, P n <= 8192, each
// thread up to 32 complex values in registers; the first forward pass reads
// the lines from HBM and the last inverse pass writes them, every other
// exchange goes through LDS (in place: all reads of a pass complete before
// its writes). x lines: the block takes 2P consecutive z columns of one
// (field, y) row, LDS element (x, p) at x P + p with lanes running over p
// first, so each x row is one contiguous 8P-byte piece; consecutive blocks
// of one XCD take neighbouring z pieces, which share cache lines. z lines:
// the block takes 2P consecutive (x, y) rows of one field, element (p, x)
// at p n + x with lanes running over the position first. LDS offsets are
// swizzled within aligned groups of 32 elements (e ^ (e / 32 mod 32)) so
// that the strided writes of the first passes spread over the banks.
#include "eles_internal.h"

namespace eles {
namespace {


struct cpx {
  float re, im;
};

__device__ inline cpx cadd(cpx a, cpx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cpx csub(cpx a, cpx b) { return {a.re - b.re, a.im - b.im}; }
// a (c + S i s)
template <int S>
__device__ inline cpx crot(cpx a, float c, float s) {
  return S > 0 ? cpx{a.re * c - a.im * s, a.re * s + a.im * c} : cpx{a.re * c + a.im * s, a.im * c - a.re * s};
}
// a (S i)
template <int S>
__device__ inline cpx cmuli(cpx a) {
  return S > 0 ? cpx{-a.im, a.re} : cpx{a.im, -a.re};
}

// cos and sin of 2 pi m / 16
__device__ constexpr float c16(int m) {
  m &= 15;
  return m == 0 ? 1.0f
         : m == 1 || m == 15 ? 0.923879532511286756f
         : m == 2 || m == 14 ? 0.707106781186547524f
         : m == 3 || m == 13 ? 0.382683432365089772f
         : m == 4 || m == 12 ? 0.0f
         : m == 5 || m == 11 ? -0.382683432365089772f
         : m == 6 || m == 10 ? -0.707106781186547524f
         : m == 7 || m == 9  ? -0.923879532511286756f
                             : -1.0f;
}
__device__ constexpr float s16(int m) { return c16(m - 4); }

// a exp(S 2 pi i m / R) for R dividing 16; the quarter turns exactly
template <int S, int R>
__device__ inline cpx twist(cpx a, int m) {
  const int e = (m * (16 / R)) & 15;
  if (e == 0) return a;
  if (e == 4) return cmuli<S>(a);
  if (e == 8) return cpx{-a.re, -a.im};
  if (e == 12) return cmuli<-S>(a);
  return crot<S>(a, c16(e), s16(e));
}

// v[q] <- sum_r v[r] exp(S 2 pi i r q / R), in place on R registers
template <int R, int S>
struct Dft;

template <int S>
struct Dft<2, S> {
  __device__ __attribute__((always_inline)) static void run(cpx *v) {
    const cpx a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int S>
struct Dft<3, S> {
  __device__ __attribute__((always_inline)) static void run(cpx *v) {
    const float h = 0.866025403784438647f;   // sin(2 pi / 3)
    const cpx s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const cpx m = {v[0].re - 0.5f * s.re, v[0].im - 0.5f * s.im};
    const cpx e = cmuli<S>(cpx{h * d.re, h * d.im});
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, e);
    v[2] = csub(m, e);
  }
};

template <int S>
struct Dft<4, S> {
  __device__ __attribute__((always_inline)) static void run(cpx *v) {
    const cpx t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const cpx t2 = cadd(v[1], v[3]), t3 = cmuli<S>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <int S>
struct Dft<5, S> {
  __device__ __attribute__((always_inline)) static void run(cpx *v) {
    const float c1 = 0.309016994374947424f, c2 = -0.809016994374947424f;   // cos(2 pi/5), cos(4 pi/5)
    const float s1 = 0.951056516295153572f, s2 = 0.587785252292473129f;   // sin(2 pi/5), sin(4 pi/5)
    const cpx t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const cpx t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    const cpx b1 = {v[0].re + c1 * t1.re + c2 * t2.re, v[0].im + c1 * t1.im + c2 * t2.im};
    const cpx b2 = {v[0].re + c2 * t1.re + c1 * t2.re, v[0].im + c2 * t1.im + c1 * t2.im};
    const cpx d1 = cmuli<S>(cpx{s1 * t3.re + s2 * t4.re, s1 * t3.im + s2 * t4.im});
    const cpx d2 = cmuli<S>(cpx{s2 * t3.re - s1 * t4.re, s2 * t3.im - s1 * t4.im});
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(b1, d1);
    v[4] = csub(b1, d1);
    v[2] = cadd(b2, d2);
    v[3] = csub(b2, d2);
  }
};

// R = R1 R2: input r = R2 r1 + r2, output q = q1 + R1 q2; R1-point DFTs
// over r1, turns exp(S 2 pi i r2 q1 / R), R2-point DFTs over r2
template <int R1, int R2, int S>
struct DftSplit {
  __device__ __attribute__((always_inline)) static void run(cpx *v) {
    constexpr int R = R1 * R2;
    cpx b[R];
#pragma unroll
    for (int r2 = 0; r2 < R2; ++r2) {
      cpx t[R1];
#pragma unroll
      for (int r1 = 0; r1 < R1; ++r1) t[r1] = v[R2 * r1 + r2];
      Dft<R1, S>::run(t);
#pragma unroll
      for (int q1 = 0; q1 < R1; ++q1) b[r2 * R1 + q1] = twist<S, R>(t[q1], r2 * q1);
    }
#pragma unroll
    for (int q1 = 0; q1 < R1; ++q1) {
      cpx t[R2];
#pragma unroll
      for (int r2 = 0; r2 < R2; ++r2) t[r2] = b[r2 * R1 + q1];
      Dft<R2, S>::run(t);
#pragma unroll
      for (int q2 = 0; q2 < R2; ++q2) v[q1 + R1 * q2] = t[q2];
    }
  }
};
template <int S>
struct Dft<8, S> : DftSplit<2, 4, S> {};
template <int S>
struct Dft<16, S> : DftSplit<4, 4, S> {};

__device__ inline int swz(int e) { return e ^ ((e >> 5) & 31); }

__device__ inline uint32_t divm(uint32_t w, uint32_t d, uint32_t mag) { return d == 1 ? w : __umulhi(w, mag); }

// The block's lines. x lines: element (x, p) at x * xs + 2 p (real) and
// + 1 (imaginary); z lines: element (x, p) at 2 p * xs + x and + xs. Real
// line 2 p + h exists while 2 p + h < lim.
struct Tile {
  const float *in;
  float *out;
  int P, lp, n;
  long xs;
  int lim;
  bool vec;   // x lines: the pairs are 8-byte aligned
};

// item w of a pass with nR = n / R items per line: line p, position j
template <bool Z>
__device__ inline void item(const Tile &t, int w, int nR, uint32_t mag, int &p, int &j) {
  if (!Z) {
    p = w & (t.P - 1);
    j = w >> t.lp;
  } else {
    p = (int)divm((uint32_t)w, (uint32_t)nR, mag);
    j = w - p * nR;
  }
}

template <bool Z>
__device__ inline int lds_at(const Tile &t, int x, int p) {
  return swz(Z ? p * t.n + x : x * t.P + p);
}

template <bool Z>
__device__ inline cpx gload(const Tile &t, int x, int p) {
  cpx v{0.0f, 0.0f};
  const int h = 2 * p;
  if (!Z) {
    const float *a = t.in + (long)x * t.xs + h;
    if (t.vec && h + 1 < t.lim) {
      const float2 q = *reinterpret_cast<const float2 *>(a);
      v = cpx{q.x, q.y};
    } else {
      if (h < t.lim) v.re = a[0];
      if (h + 1 < t.lim) v.im = a[1];
    }
  } else {
    const float *a = t.in + (long)h * t.xs + x;
    if (h < t.lim) v.re = a[0];
    if (h + 1 < t.lim) v.im = a[t.xs];
  }
  return v;
}

template <bool Z>
__device__ inline void gstore(const Tile &t, int x, int p, cpx v) {
  const int h = 2 * p;
  if (!Z) {
    float *a = t.out + (long)x * t.xs + h;
    if (t.vec && h + 1 < t.lim) {
      *reinterpret_cast<float2 *>(a) = make_float2(v.re, v.im);
    } else {
      if (h < t.lim) a[0] = v.re;
      if (h + 1 < t.lim) a[1] = v.im;
    }
  } else {
    float *a = t.out + (long)h * t.xs + x;
    if (h < t.lim) a[0] = v.re;
    if (h + 1 < t.lim) a[t.xs] = v.im;
  }
}

// Global access of a block's lines: two real lines as one complex line.
template <bool Z>
struct PairIO {
  static constexpr bool kLds = false;   // loads from LDS the pass then overwrites
  __device__ cpx load(const Tile &t, int x, int p) const { return gload<Z>(t, x, p); }
  __device__ void store(const Tile &t, int x, int p, cpx v) const { gstore<Z>(t, x, p, v); }
};

// z lines read from rows staged in LDS, row 2p + h at raw[(2 p + h + 1) n]
// (row -1 and row 2P are the neighbours of the tile)
template <bool Z>
struct RawIO {
  static constexpr bool kLds = true;
  const float *raw;
  __device__ cpx load(const Tile &t, int x, int p) const {
    return cpx{raw[(2 * p + 1) * t.n + x], raw[(2 * p + 2) * t.n + x]};
  }
  __device__ void store(const Tile &t, int x, int p, cpx v) const { gstore<Z>(t, x, p, v); }
};

// One pass of radix R. SRC: 0 global, 1 LDS, 2 registers (the carried
// items); DST: 0 global, 1 LDS, 2 registers. Items are tid + it * T;
// rsync: wait for every thread's LDS reads before the writes (in place).
// io: the global loads (SRC 0) and stores (DST 0).
template <bool Z, int E, int T, int R, int S, int SRC, int DST, class IO = PairIO<Z>>
__device__ __attribute__((always_inline)) inline void pass(const Tile &t, cpx (&v)[E], cpx *lds, const cpx *tw, int Ns, uint32_t mnr,
                            uint32_t mns, bool rsync, const IO &io = IO()) {
  constexpr int IT = E / R;
  const int n = t.n, nR = n / R, items = t.P * nR;
  const int tid = threadIdx.x;
  if (SRC != 2) {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int w = tid + it * T;
      if (w < items) {
        int p, j;
        item<Z>(t, w, nR, mnr, p, j);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int x = j + r * nR;
          if (SRC == 0) {
            v[it * R + r] = io.load(t, x, p);
          } else {
            const float2 q = reinterpret_cast<const float2 *>(lds)[lds_at<Z>(t, x, p)];
            v[it * R + r] = cpx{q.x, q.y};
          }
        }
      }
    }
    if ((SRC == 1 || IO::kLds) && rsync) __syncthreads();
  }
  const int stride = Ns > 1 ? n / (Ns * R) : 0;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = tid + it * T;
    if (w < items) {
      int p, j;
      item<Z>(t, w, nR, mnr, p, j);
      cpx *a = v + it * R;
      int k = 0;
      if (Ns > 1) {
        k = j - Ns * (int)divm((uint32_t)j, (uint32_t)Ns, mns);
        const int m = k * stride;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 q = reinterpret_cast<const float2 *>(tw)[r * m];
          a[r] = crot<S>(a[r], q.x, -q.y);   // tw holds exp(-2 pi i m / n)
        }
      }
      Dft<R, S>::run(a);
      if (DST != 2) {
        const int base = (j - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int x = base + q * Ns;
          if (DST == 0) {
            io.store(t, x, p, a[q]);
          } else {
            reinterpret_cast<float2 *>(lds)[lds_at<Z>(t, x, p)] = make_float2(a[q].re, a[q].im);
          }
        }
      }
    }
  }
  if (DST == 1) __syncthreads();
}

// the derivative factors on the carried items of a radix-R pass: item j
// holds coefficients j + q n/R
template <bool Z, int E, int T, int R>
__device__ __attribute__((always_inline)) inline void deriv(const Tile &t, cpx (&v)[E], float cfac, uint32_t mnr) {
  constexpr int IT = E / R;
  const int n = t.n, nR = n / R, items = t.P * nR;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = threadIdx.x + it * T;
    if (w < items) {
      int p, j;
      item<Z>(t, w, nR, mnr, p, j);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int m = j + q * nR;
        const int km = 2 * m < n ? m : (2 * m == n ? 0 : m - n);
        const float f = cfac * (float)km;
        const cpx a = v[it * R + q];
        v[it * R + q] = cpx{-f * a.im, f * a.re};
      }
    }
  }
}

// Pass s of the forward (S = -1) or inverse (S = +1) transform with radix R
// of nr passes; after the last forward pass the derivative factors.
template <bool Z, int E, int T, int S, int R, class IO = PairIO<Z>>
__device__ __attribute__((always_inline)) inline void step_r(const Tile &t, cpx (&v)[E], cpx *lds, const cpx *tw, int s, int nr, int Ns,
                              uint32_t mnr, uint32_t mns, float cfac, const IO &io = IO()) {
  const bool first = s == 0, last = s == nr - 1;
  if (S < 0) {
    // a first pass reading LDS rows it then overwrites waits for every read
    if (first && last) pass<Z, E, T, R, S, 0, 2, IO>(t, v, lds, tw, Ns, mnr, mns, false, io);
    else if (first) pass<Z, E, T, R, S, 0, 1, IO>(t, v, lds, tw, Ns, mnr, mns, IO::kLds, io);
    else if (last) pass<Z, E, T, R, S, 1, 2>(t, v, lds, tw, Ns, mnr, mns, true);
    else pass<Z, E, T, R, S, 1, 1>(t, v, lds, tw, Ns, mnr, mns, true);
    if (last) deriv<Z, E, T, R>(t, v, cfac, mnr);
  } else {
    if (first && last) pass<Z, E, T, R, S, 2, 0>(t, v, lds, tw, Ns, mnr, mns, false);
    else if (first) pass<Z, E, T, R, S, 2, 1>(t, v, lds, tw, Ns, mnr, mns, false);
    else if (last) pass<Z, E, T, R, S, 1, 0>(t, v, lds, tw, Ns, mnr, mns, false);
    else pass<Z, E, T, R, S, 1, 1>(t, v, lds, tw, Ns, mnr, mns, true);
  }
}

template <bool Z, int E, int T, int S, class IO = PairIO<Z>>
__device__ __attribute__((always_inline)) inline void step(int R, const Tile &t, cpx (&v)[E], cpx *lds, const cpx *tw, int s, int nr, int Ns,
                            uint32_t mnr, uint32_t mns, float cfac, const IO &io = IO()) {
  switch (R) {
    case 16: step_r<Z, E, T, S, 16, IO>(t, v, lds, tw, s, nr, Ns, mnr, mns, cfac, io); break;
    case 8: step_r<Z, E, T, S, 8, IO>(t, v, lds, tw, s, nr, Ns, mnr, mns, cfac, io); break;
    case 4: step_r<Z, E, T, S, 4, IO>(t, v, lds, tw, s, nr, Ns, mnr, mns, cfac, io); break;
    case 2: step_r<Z, E, T, S, 2, IO>(t, v, lds, tw, s, nr, Ns, mnr, mns, cfac, io); break;
    case 3: step_r<Z, E, T, S, 3, IO>(t, v, lds, tw, s, nr, Ns, mnr, mns, cfac, io); break;
    default: step_r<Z, E, T, S, 5, IO>(t, v, lds, tw, s, nr, Ns, mnr, mns, cfac, io); break;
  }
}

// Radix plans: Rad<> reads the plan of the axis at run time; Rad<R0, ...>
// fixes it at compile time, so the passes unroll into straight-line code
// with the pass geometry constant.
template <int... Rs>
struct Rad {
  static constexpr int np = sizeof...(Rs);
  __device__ static constexpr int at(int s) {
    constexpr int r[] = {Rs...};
    return r[s];
  }
  __device__ static constexpr int len() { return (Rs * ...); }
};
template <>
struct Rad<> {
  static constexpr int np = 0;
};

template <bool Z, int E, int T, class PL, bool DY = false>
__global__ void __launch_bounds__(T) k_sder(SderArgs g) {
  extern __shared__ float2 sder_lds[];
  const SderAxis &A = g.ax;
  int n;
  if constexpr (PL::np > 0) n = PL::len();
  else n = A.n;
  cpx *lds = reinterpret_cast<cpx *>(sder_lds);
  // with d/dy the data region first holds the tile's rows and their two
  // neighbours, 2P + 2 rows of n floats
  cpx *tw = lds + (((A.P + (DY ? 1 : 0)) * n + 31) & ~31);
  for (int m = threadIdx.x; m < n; m += T) {
    const float2 q = A.tw[m];
    tw[m] = cpx{q.x, q.y};
  }
  const long tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  Tile t;
  t.P = A.P;
  t.lp = A.lp;
  t.n = n;
  t.vec = false;
  const long plane = (long)g.ny * g.nz;
  if (!Z) {
    // tile = ((f ny) + y) nzt + zt
    const int nzt = (g.nz + 2 * A.P - 1) / (2 * A.P);
    const int zt = (int)(tile % nzt);
    const long rest = tile / nzt;
    const int y = (int)(rest % g.ny), f = (int)(rest / g.ny);
    const long o = (long)y * g.nz + 2L * A.P * zt;
    t.in = g.in + f * g.in_fs + o;
    t.out = g.out + f * g.out_fs + o;
    t.xs = plane;
    t.lim = g.nz - 2 * A.P * zt;
    t.vec = (g.nz & 1) == 0 && (g.in_fs & 1) == 0 && (g.out_fs & 1) == 0;
  } else {
    const long rows = (long)g.nx * g.ny;
    const long nrt = (rows + 2 * A.P - 1) / (2 * A.P);
    const long rt = tile % nrt;
    const int f = (int)(tile / nrt);
    const long o = rt * 2 * A.P * g.nz;
    t.in = g.in + f * g.in_fs + o;
    t.out = g.out + f * g.out_fs + o;
    t.xs = g.nz;
    t.lim = (int)min((long)2 * A.P, rows - rt * 2 * A.P);
    if constexpr (DY) {
      // d/dy: rows r0 - 1 .. r0 + 2P of the field into LDS (zeros past the
      // field), eight loads in flight per thread, and the weights of each
      // tile row for its y (the wall rows use the mirror rows folded into D)
      // beside them; then each tile row from its neighbours
      float *raw = reinterpret_cast<float *>(lds);
      float *wts = reinterpret_cast<float *>(tw + n);
      const long r0 = rt * 2 * A.P;
      const float *src = g.in + f * g.in_fs;
      const long e_at = (r0 - 1) * g.nz;   // raw element e is field element e_at + e
      const long lo = r0 == 0 ? n : 0, hi = (rows - r0 + 1) * (long)n;
      const int total = (2 * A.P + 2) * n;
      for (int e0 = 0; e0 < total; e0 += 8 * T) {
        float r[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int e = e0 + k * T + (int)threadIdx.x;
          r[k] = e < total && e >= lo && e < hi ? src[e_at + e] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int e = e0 + k * T + (int)threadIdx.x;
          if (e < total) raw[e] = r[k];
        }
      }
      const float *D = g.D[(g.pmask >> f) & 1u];
      if ((int)threadIdx.x < t.lim) {   // one thread per tile row (2P <= T, checked on the host)
        const int q = threadIdx.x;
        const int y = (int)((r0 + q) % g.ny);
        float d0 = 0.0f, d1, d2 = 0.0f, kind = 0.0f;   // kind: 0 interior, 1 y = 0, 2 y = ny - 1
        if (y == 0) {
          d1 = D[0];
          d2 = D[1];
          kind = 1.0f;
        } else if (y == g.ny - 1) {
          const float *Dl = D + (long)y * g.kp + (y - 1);
          d0 = Dl[0];
          d1 = Dl[1];
          kind = 2.0f;
        } else {
          const float *Dr = D + (long)y * g.kp + (y - 1);
          d0 = Dr[0];
          d1 = Dr[1];
          d2 = Dr[2];
        }
        wts[4 * q] = d0;
        wts[4 * q + 1] = d1;
        wts[4 * q + 2] = d2;
        wts[4 * q + 3] = kind;
      }
      __syncthreads();
      float *dst = g.dy + f * g.out_fs + r0 * g.nz;
      for (int q = 0; q < t.lim; ++q) {
        const float d0 = wts[4 * q], d1 = wts[4 * q + 1], d2 = wts[4 * q + 2], kind = wts[4 * q + 3];
        const float *um = raw + q * n, *u0 = raw + (q + 1) * n, *up = raw + (q + 2) * n;
        float *o = dst + (long)q * g.nz;
        // a wall row reads no row of the neighbouring column
        if (kind == 1.0f) {
          for (int x = threadIdx.x; x < n; x += T) o[x] = d1 * u0[x] + d2 * up[x];
        } else if (kind == 2.0f) {
          for (int x = threadIdx.x; x < n; x += T) o[x] = d0 * um[x] + d1 * u0[x];
        } else {
          for (int x = threadIdx.x; x < n; x += T) o[x] = d0 * um[x] + d1 * u0[x] + d2 * up[x];
        }
      }
    }
  }
  cpx v[E];
  [[maybe_unused]] const RawIO<Z> rio{reinterpret_cast<const float *>(lds)};
  if constexpr (DY) {
    static_assert(Z, "d/dy rides on the z lines");
    if constexpr (PL::np > 0) {
      constexpr int nr = PL::np;
      int Ns = 1;
#pragma unroll
      for (int s = 0; s < nr; ++s) {
        step<Z, E, T, -1, RawIO<Z>>(PL::at(s), t, v, lds, tw, s, nr, Ns, A.mnr[s], A.mns[s], A.cfac, rio);
        Ns *= PL::at(s);
      }
      Ns = 1;
#pragma unroll
      for (int s = 0; s < nr; ++s) {
        const int si = nr - 1 - s;
        step<Z, E, T, 1, RawIO<Z>>(PL::at(si), t, v, lds, tw, s, nr, Ns, A.mnr[si], A.imns[s], A.cfac, rio);
        Ns *= PL::at(si);
      }
    } else {
      const int nr = A.nrad;
      int Ns = 1;
      for (int s = 0; s < nr; ++s) {
        step<Z, E, T, -1, RawIO<Z>>(A.rad[s], t, v, lds, tw, s, nr, Ns, A.mnr[s], A.mns[s], A.cfac, rio);
        Ns *= A.rad[s];
      }
      Ns = 1;
      for (int s = 0; s < nr; ++s) {
        const int si = nr - 1 - s;
        step<Z, E, T, 1, RawIO<Z>>(A.rad[si], t, v, lds, tw, s, nr, Ns, A.mnr[si], A.imns[s], A.cfac, rio);
        Ns *= A.rad[si];
      }
    }
    return;
  }
  if constexpr (PL::np > 0) {
    constexpr int nr = PL::np;
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < nr; ++s) {
      step<Z, E, T, -1>(PL::at(s), t, v, lds, tw, s, nr, Ns, A.mnr[s], A.mns[s], A.cfac);
      Ns *= PL::at(s);
    }
    Ns = 1;
#pragma unroll
    for (int s = 0; s < nr; ++s) {
      const int si = nr - 1 - s;
      step<Z, E, T, 1>(PL::at(si), t, v, lds, tw, s, nr, Ns, A.mnr[si], A.imns[s], A.cfac);
      Ns *= PL::at(si);
    }
  } else {
    const int nr = A.nrad;
    int Ns = 1;
    for (int s = 0; s < nr; ++s) {
      step<Z, E, T, -1>(A.rad[s], t, v, lds, tw, s, nr, Ns, A.mnr[s], A.mns[s], A.cfac);
      Ns *= A.rad[s];
    }
    Ns = 1;
    for (int s = 0; s < nr; ++s) {
      const int si = nr - 1 - s;
      step<Z, E, T, 1>(A.rad[si], t, v, lds, tw, s, nr, Ns, A.mnr[si], A.imns[s], A.cfac);
      Ns *= A.rad[si];
    }
  }
}

// ---- real transforms (the differential filter's x and z transforms)
//
// Two real lines a, b travel as z = a + i b. Forward: Z = DFT(z) with
// exp(-2 pi i k x / n), then A_k = (Z_k + conj Z_{n-k}) / 2 and B_k = (Z_k -
// conj Z_{n-k}) / (2 i) are the transforms of a and b, and the folded real
// coefficients of a line are C_k = Re A_k at position k (k = 0 .. n/2) and
// S_k = -Im A_k at position n/2 + k (k = 1 .. (n - 1)/2): the sums of the
// line times cos and sin (2 pi k x / n). Inverse: A_k = C_k - i S_k for k <=
// n/2, A_{n-k} = conj A_k, the same for B, z = DFT^-1(A + i B) / n.

// forward input: the field's two real lines, or (the x transform of the
// stress) the field formed from u: u_a' or u_a' u_b', with u1' = u1 - m(y)
template <bool Z>
struct FwdIO {
  static constexpr bool kLds = false;
  const float *ua, *ub;   // products: the factors' lines at the tile's origin; else null
  float sa, sb;           // shifts subtracted from the factors
  bool two;               // a product of two factors
  __device__ cpx load(const Tile &t, int x, int p) const {
    if (!ua) return gload<Z>(t, x, p);
    cpx v{0.0f, 0.0f};
    const int h = 2 * p;
    const long o = (long)x * t.xs + h;
    if (h < t.lim) {
      const float a = ua[o] - sa;
      v.re = two ? a * (ub[o] - sb) : a;
    }
    if (h + 1 < t.lim) {
      const float a = ua[o + 1] - sa;
      v.im = two ? a * (ub[o + 1] - sb) : a;
    }
    return v;
  }
  __device__ void store(const Tile &, int, int, cpx) const {}
};

// inverse input: Z_k = A_k + i B_k from the folded coefficients of both
// lines; output: the two real lines scaled by 1/n
template <bool Z>
struct InvIO {
  static constexpr bool kLds = false;
  int h, hs;
  float scale;
  bool zero;   // the lines are wall rows of an odd field: exactly zero
  __device__ cpx load(const Tile &t, int k, int p) const {
    const bool up = k > h;
    const int kk = up ? t.n - k : k;
    const cpx c = gload<Z>(t, kk, p);
    const cpx sn = kk >= 1 && kk <= hs ? gload<Z>(t, h + kk, p) : cpx{0.0f, 0.0f};
    const cpx A{c.re, up ? sn.re : -sn.re}, B{c.im, up ? sn.im : -sn.im};
    return cpx{A.re - B.im, A.im + B.re};
  }
  __device__ void store(const Tile &t, int x, int p, cpx v) const {
    gstore<Z>(t, x, p, zero ? cpx{0.0f, 0.0f} : cpx{v.re * scale, v.im * scale});
  }
};

// A_k, B_k from the natural-order Z in LDS, as folded coefficients
template <bool Z, int T>
__device__ inline void fwd_epilogue(const Tile &t, const cpx *lds, int h, int hs) {
  const int n = t.n, items = t.P * (h + 1);
  for (int w = threadIdx.x; w < items; w += T) {
    int p, k;
    if (!Z) {
      p = w & (t.P - 1);
      k = w >> t.lp;
    } else {
      p = w / (h + 1);
      k = w - p * (h + 1);
    }
    const float2 zk = reinterpret_cast<const float2 *>(lds)[lds_at<Z>(t, k, p)];
    const float2 zm = reinterpret_cast<const float2 *>(lds)[lds_at<Z>(t, k == 0 ? 0 : n - k, p)];
    const cpx A{0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)};
    const cpx B{0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x)};
    gstore<Z>(t, k, p, cpx{A.re, B.re});
    if (k >= 1 && k <= hs) gstore<Z>(t, h + k, p, cpx{-A.im, -B.im});
  }
}

// pass s of a forward (S = -1: global in, LDS out, natural order after the
// last pass) or inverse (S = +1: global in and out) transform
template <bool Z, int E, int T, int S, int R, class IO>
__device__ __attribute__((always_inline)) inline void tstep_r(const Tile &t, cpx (&v)[E], cpx *lds, const cpx *tw,
                                                              int s, int nr, int Ns, uint32_t mnr, uint32_t mns,
                                                              const IO &io) {
  const bool first = s == 0, last = s == nr - 1;
  if (S < 0) {
    if (first) pass<Z, E, T, R, S, 0, 1, IO>(t, v, lds, tw, Ns, mnr, mns, false, io);
    else pass<Z, E, T, R, S, 1, 1, IO>(t, v, lds, tw, Ns, mnr, mns, true, io);
  } else {
    if (first && last) pass<Z, E, T, R, S, 0, 0, IO>(t, v, lds, tw, Ns, mnr, mns, false, io);
    else if (first) pass<Z, E, T, R, S, 0, 1, IO>(t, v, lds, tw, Ns, mnr, mns, false, io);
    else if (last) pass<Z, E, T, R, S, 1, 0, IO>(t, v, lds, tw, Ns, mnr, mns, false, io);
    else pass<Z, E, T, R, S, 1, 1, IO>(t, v, lds, tw, Ns, mnr, mns, true, io);
  }
}

template <bool Z, int E, int T, int S, class IO>
__device__ __attribute__((always_inline)) inline void tstep(int R, const Tile &t, cpx (&v)[E], cpx *lds,
                                                            const cpx *tw, int s, int nr, int Ns, uint32_t mnr,
                                                            uint32_t mns, const IO &io) {
  switch (R) {
    case 16: tstep_r<Z, E, T, S, 16>(t, v, lds, tw, s, nr, Ns, mnr, mns, io); break;
    case 8: tstep_r<Z, E, T, S, 8>(t, v, lds, tw, s, nr, Ns, mnr, mns, io); break;
    case 4: tstep_r<Z, E, T, S, 4>(t, v, lds, tw, s, nr, Ns, mnr, mns, io); break;
    case 2: tstep_r<Z, E, T, S, 2>(t, v, lds, tw, s, nr, Ns, mnr, mns, io); break;
    case 3: tstep_r<Z, E, T, S, 3>(t, v, lds, tw, s, nr, Ns, mnr, mns, io); break;
    default: tstep_r<Z, E, T, S, 5>(t, v, lds, tw, s, nr, Ns, mnr, mns, io); break;
  }
}

template <bool Z, int E, int T, int S, class PL, class IO>
__device__ __attribute__((always_inline)) inline void transform(const SderAxis &A, const Tile &t, cpx (&v)[E],
                                                                cpx *lds, const cpx *tw, const IO &io) {
  if constexpr (PL::np > 0) {
    constexpr int nr = PL::np;
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < nr; ++s) {
      tstep<Z, E, T, S>(PL::at(s), t, v, lds, tw, s, nr, Ns, A.mnr[s], A.mns[s], io);
      Ns *= PL::at(s);
    }
  } else {
    const int nr = A.nrad;
    int Ns = 1;
    for (int s = 0; s < nr; ++s) {
      tstep<Z, E, T, S>(A.rad[s], t, v, lds, tw, s, nr, Ns, A.mnr[s], A.mns[s], io);
      Ns *= A.rad[s];
    }
  }
}

// nf fields [nf][nx][ny][nz]: x lines (tile = ((y nzt + zt) nf + f), the
// fields of one tile on neighbouring blocks, which share u when the fields
// are formed from it) or z lines (tile = rt nf + f)
template <bool INV, bool Z, int E, int T, class PL>
__global__ void __launch_bounds__(T) k_rfft(RfftArgs g) {
  extern __shared__ float2 rfft_lds[];
  const SderAxis &A = g.ax;
  int n;
  if constexpr (PL::np > 0) n = PL::len();
  else n = A.n;
  cpx *lds = reinterpret_cast<cpx *>(rfft_lds);
  cpx *tw = lds + ((A.P * n + 31) & ~31);
  for (int m = threadIdx.x; m < n; m += T) {
    const float2 q = A.tw[m];
    tw[m] = cpx{q.x, q.y};
  }
  const long tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  Tile t;
  t.P = A.P;
  t.lp = A.lp;
  t.n = n;
  t.vec = false;
  const long plane = (long)g.ny * g.nz;
  const int f = (int)(tile % g.nf);
  const long rest = tile / g.nf;
  FwdIO<Z> fio{nullptr, nullptr, 0.0f, 0.0f, false};
  bool zero = false;
  long o;
  if (!Z) {
    const int nzt = (g.nz + 2 * A.P - 1) / (2 * A.P);
    const int zt = (int)(rest % nzt), y = (int)(rest / nzt);
    // the paired lines' rounding would leave traces of the neighbouring
    // lines on the wall rows of odd fields, which are zero by parity
    zero = INV && ((g.zmask >> f) & 1u) && (y == 0 || y == g.ny - 1);
    o = (long)y * g.nz + 2L * A.P * zt;
    t.xs = plane;
    t.lim = g.nz - 2 * A.P * zt;
    t.vec = (g.nz & 1) == 0 && (g.in_fs & 1) == 0 && (g.out_fs & 1) == 0;
    if (!INV && g.prod) {
      // stress field f: u1', u2, u3, u1'u1', u1'u2, u1'u3, u2u2, u2u3, u3u3
      const int ca = f < 3 ? f : (f < 6 ? 0 : (f < 8 ? 1 : 2));
      const int cb = f < 3 ? f : (f < 6 ? f - 3 : (f == 6 ? 1 : 2));
      const float m = g.prof[y];
      fio = FwdIO<Z>{g.in + ca * g.in_fs + o, g.in + cb * g.in_fs + o, ca == 0 ? m : 0.0f, cb == 0 ? m : 0.0f,
                     f >= 3};
    }
  } else {
    const long rows = (long)g.nx * g.ny;
    o = rest * 2 * A.P * g.nz;
    t.xs = g.nz;
    t.lim = (int)min((long)2 * A.P, rows - rest * 2 * A.P);
  }
  t.in = g.in + f * g.in_fs + o;
  t.out = g.out + f * g.out_fs + o;
  const int h = n / 2, hs = (n - 1) / 2;
  cpx v[E];
  if (!INV) {
    transform<Z, E, T, -1, PL>(A, t, v, lds, tw, fio);
    fwd_epilogue<Z, T>(t, lds, h, hs);
  } else {
    transform<Z, E, T, 1, PL>(A, t, v, lds, tw, InvIO<Z>{h, hs, 1.0f / (float)n, zero});
  }
}

// exp(-2 pi i m / n) in FP64, rounded to FP32
__global__ void __launch_bounds__(256) k_sder_tw(int n, float2 *tw) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= n) return;
  double s, c;
  sincospi(2.0 * m / n, &s, &c);
  tw[m] = make_float2((float)c, (float)-s);
}

typedef void (*SderKernel)(SderArgs);

// The plans of 192, 512, 768 and 1024 nodes have compile-time instances;
// every other runs through the run-time plan, in blocks of 256.
int sder_fixed(const int *rad, int nr) {
  static const int plans[4][3] = {{16, 16, 4}, {16, 16, 3}, {16, 16, 2}, {16, 4, 3}};
  for (int k = 0; k < 4; ++k)
    if (nr == 3 && rad[0] == plans[k][0] && rad[1] == plans[k][1] && rad[2] == plans[k][2]) return k + 1;
  return 0;
}

template <bool Z, int E, int T>
SderKernel sder_kernel(const SderAxis &a) {
  switch (sder_fixed(a.rad, a.nrad)) {
    case 1: return k_sder<Z, E, T, Rad<16, 16, 4>>;
    case 2: return k_sder<Z, E, T, Rad<16, 16, 3>>;
    case 3: return k_sder<Z, E, T, Rad<16, 16, 2>>;
    case 4: return k_sder<Z, E, T, Rad<16, 4, 3>>;
    default: return nullptr;
  }
}

// z lines with the fused d/dy
template <int E>
SderKernel sder_kernel_dy(const SderAxis &a) {
  switch (sder_fixed(a.rad, a.nrad)) {
    case 1: return k_sder<true, E, 256, Rad<16, 16, 4>, true>;
    case 2: return k_sder<true, E, 256, Rad<16, 16, 3>, true>;
    case 3: return k_sder<true, E, 256, Rad<16, 16, 2>, true>;
    case 4: return k_sder<true, E, 256, Rad<16, 4, 3>, true>;
    default: return k_sder<true, E, 256, Rad<>, true>;
  }
}

SderKernel sder_pick(const SderAxis &a, bool zaxis) {
  if (!sder_fixed(a.rad, a.nrad)) {
    if (zaxis) return a.E == 16 ? k_sder<true, 16, 256, Rad<>> : k_sder<true, 32, 256, Rad<>>;
    return a.E == 16 ? k_sder<false, 16, 256, Rad<>> : k_sder<false, 32, 256, Rad<>>;
  }
  if (zaxis) return a.E == 16 ? sder_kernel<true, 16, 256>(a) : sder_kernel<true, 32, 256>(a);
  if (a.T == 1024) return sder_kernel<false, 16, 1024>(a);
  if (a.T == 512) return a.E == 16 ? sder_kernel<false, 16, 512>(a) : sder_kernel<false, 32, 512>(a);
  return a.E == 16 ? sder_kernel<false, 16, 256>(a) : sder_kernel<false, 32, 256>(a);
}

}  // namespace

typedef void (*RfftKernel)(RfftArgs);

template <bool Z, int E, int T, bool INV>
RfftKernel rfft_kernel(const SderAxis &a) {
  switch (sder_fixed(a.rad, a.nrad)) {
    case 1: return k_rfft<INV, Z, E, T, Rad<16, 16, 4>>;
    case 2: return k_rfft<INV, Z, E, T, Rad<16, 16, 3>>;
    case 3: return k_rfft<INV, Z, E, T, Rad<16, 16, 2>>;
    case 4: return k_rfft<INV, Z, E, T, Rad<16, 4, 3>>;
    default: return nullptr;
  }
}

template <bool INV>
RfftKernel rfft_pick_t(const SderAxis &a, bool zaxis) {
  if (!sder_fixed(a.rad, a.nrad)) {
    if (zaxis) return a.E == 16 ? k_rfft<INV, true, 16, 256, Rad<>> : k_rfft<INV, true, 32, 256, Rad<>>;
    return a.E == 16 ? k_rfft<INV, false, 16, 256, Rad<>> : k_rfft<INV, false, 32, 256, Rad<>>;
  }
  if (zaxis) return a.E == 16 ? rfft_kernel<true, 16, 256, INV>(a) : rfft_kernel<true, 32, 256, INV>(a);
  if (a.T == 512) return a.E == 16 ? rfft_kernel<false, 16, 512, INV>(a) : rfft_kernel<false, 32, 512, INV>(a);
  return a.E == 16 ? rfft_kernel<false, 16, 256, INV>(a) : rfft_kernel<false, 32, 256, INV>(a);
}

RfftKernel rfft_pick(const SderAxis &a, bool zaxis, bool inverse) {
  return inverse ? rfft_pick_t<true>(a, zaxis) : rfft_pick_t<false>(a, zaxis);
}

size_t sder_lds_bytes(const SderAxis &a) { return (size_t)(((a.P * a.n + 31) & ~31) + a.n) * 8; }

// the largest power-of-two P <= 64 whose items fit every pass's E
// registers in blocks of T threads
static int sder_lines(int n, const int *rad, int nr, int E, int T) {
  int best = 0;
  for (int P = 1; P <= 64; P *= 2) {
    if ((long)P * n > (long)T * E) break;
    bool ok = true;
    for (int s = 0; s < nr; ++s) {
      const long items = (long)P * (n / rad[s]);
      if ((items + T - 1) / T > E / rad[s]) ok = false;
    }
    if (ok) best = P;
  }
  return best;
}

bool sder_plan(int n, double length, bool zaxis, SderAxis *a) {
  a->n = n;
  a->nrad = 0;
  a->cfac = (float)(2.0 * M_PI / (length * n));
  int m = n, nr = 0;
  for (int r : {16, 8, 4, 2, 3, 5})
    while (m % r == 0 && nr < kSderMaxPass) {
      a->rad[nr++] = r;
      m /= r;
    }
  if (m != 1 || n < 2) return false;
  // z lines are contiguous rows: 16 values per thread in blocks of 256
  // where that still holds two complex lines, else 32. x lines read one
  // 8P-byte piece per x row: blocks of 512 threads with 16 values each
  // give P = 8 (64-byte pieces) at 1024 nodes with two blocks per CU.
  int P = 0;
  const int shapes[2][2] = {{16, zaxis || !sder_fixed(a->rad, nr) ? 256 : 512}, {32, 256}};
  for (const auto &sh : shapes) {
    a->E = sh[0];
    a->T = sh[1];
    P = sder_lines(n, a->rad, nr, a->E, a->T);
    if (P >= 2) break;
  }
  if (!P) return false;
  a->P = P;
  a->lp = 0;
  while ((1 << a->lp) < P) ++a->lp;
  auto mag = [](long d) { return d <= 1 ? 0u : (uint32_t)(((1ull << 32) + (unsigned long long)d - 1) / d); };
  long ns = 1, ins = 1;
  for (int s = 0; s < nr; ++s) {
    a->mnr[s] = mag(n / a->rad[s]);
    a->mns[s] = mag(ns);
    ns *= a->rad[s];
    a->imns[s] = mag(ins);
    ins *= a->rad[nr - 1 - s];
  }
  a->nrad = nr;
  return true;
}

hipError_t sder_setup(const SderAxis &a, hipStream_t s) {
  if (!a.nrad) return hipSuccess;
  k_sder_tw<<<(unsigned)((a.n + 255) / 256), 256, 0, s>>>(a.n, a.tw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t bytes = sder_lds_bytes(a);
  for (bool z : {false, true}) {
    if (bytes <= 65536 || e != hipSuccess) break;
    e = hipFuncSetAttribute((const void *)sder_pick(a, z), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  }
  return e;
}

hipError_t launch_sder(const GradView &v, bool zaxis, const float *ubar, float *out, long out_fstride,
                       hipStream_t s) {
  SderArgs g;
  g.ax = zaxis ? v.sz : v.sx;
  if (!g.ax.nrad) return hipErrorInvalidValue;
  g.in = ubar;
  g.out = out;
  g.in_fs = (long)v.nx * v.ny * v.nz;
  g.out_fs = out_fstride;
  g.nx = v.nx;
  g.ny = v.ny;
  g.nz = v.nz;
  g.zaxis = zaxis;
  g.dy = nullptr;
  g.D[0] = g.D[1] = nullptr;
  g.kp = 0;
  g.pmask = 0;
  const int P2 = 2 * g.ax.P;
  const long tiles = zaxis ? 3L * (((long)v.nx * v.ny + P2 - 1) / P2) : 3L * v.ny * ((v.nz + P2 - 1) / P2);
  if (tiles > 0x7fffffffL) return hipErrorInvalidValue;
  sder_pick(g.ax, zaxis)<<<(unsigned)tiles, g.ax.T, sder_lds_bytes(g.ax), s>>>(g);
  return hipGetLastError();
}

// LDS of the z kernel with the fused d/dy: 2P + 2 staged rows in the data
// region, the twiddles, and four floats of weights per tile row (no more
// than 64 KB: the fused kernel is not given a larger limit)
static size_t sder_dy_lds_bytes(const SderAxis &a) {
  return (size_t)((((a.P + 1) * a.n + 31) & ~31) + a.n) * 8 + (size_t)8 * a.P * 4;
}

bool sder_zy_ok(const GradView &v) {
  return v.sz.nrad && v.sz.T == 256 && 2 * v.sz.P <= v.sz.T && v.ny >= 3 && sder_dy_lds_bytes(v.sz) <= 65536;
}

hipError_t launch_sder_zy(const GradView &v, const float *ubar, float *out, float *dy, long out_fstride,
                          unsigned pmask, hipStream_t s) {
  const SderAxis &a = v.sz;
  if (!sder_zy_ok(v)) return hipErrorInvalidValue;
  SderArgs g;
  g.ax = a;
  g.in = ubar;
  g.out = out;
  g.in_fs = (long)v.nx * v.ny * v.nz;
  g.out_fs = out_fstride;
  g.nx = v.nx;
  g.ny = v.ny;
  g.nz = v.nz;
  g.zaxis = 1;
  g.dy = dy;
  g.D[0] = v.dy32[0];
  g.D[1] = v.dy32[1];
  g.kp = v.kpy;
  g.pmask = pmask;
  const int P2 = 2 * a.P;
  const long tiles = 3L * (((long)v.nx * v.ny + P2 - 1) / P2);
  if (tiles > 0x7fffffffL) return hipErrorInvalidValue;
  const SderKernel k = a.E == 16 ? sder_kernel_dy<16>(a) : sder_kernel_dy<32>(a);
  k<<<(unsigned)tiles, 256, sder_dy_lds_bytes(a), s>>>(g);
  return hipGetLastError();
}

hipError_t rfft_setup(const SderAxis &a, hipStream_t s) {
  if (!a.nrad) return hipSuccess;
  k_sder_tw<<<(unsigned)((a.n + 255) / 256), 256, 0, s>>>(a.n, a.tw);
  hipError_t e = hipGetLastError();
  const size_t bytes = sder_lds_bytes(a);
  for (int k = 0; k < 4 && e == hipSuccess && bytes > 65536; ++k)
    e = hipFuncSetAttribute((const void *)rfft_pick(a, k & 1, k >> 1), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bytes);
  return e;
}

hipError_t launch_rfft(const SderAxis &a, bool zaxis, bool inverse, const float *in, float *out, const float *prof,
                       long in_fs, long out_fs, int nx, int ny, int nz, int nf, bool prod, unsigned zmask,
                       hipStream_t s) {
  if (!a.nrad || nf < 1 || (prod && (zaxis || inverse || nf != 9))) return hipErrorInvalidValue;
  RfftArgs g;
  g.zmask = zmask;
  g.ax = a;
  g.in = in;
  g.out = out;
  g.prof = prof;
  g.in_fs = in_fs;
  g.out_fs = out_fs;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.nf = nf;
  g.prod = prod ? 1 : 0;
  const int P2 = 2 * a.P;
  const long tiles = zaxis ? (long)nf * (((long)nx * ny + P2 - 1) / P2) : (long)nf * ny * ((nz + P2 - 1) / P2);
  if (tiles > 0x7fffffffL) return hipErrorInvalidValue;
  rfft_pick(a, zaxis, inverse)<<<(unsigned)tiles, a.T, sder_lds_bytes(a), s>>>(g);
  return hipGetLastError();
}

}  // namespace eles
