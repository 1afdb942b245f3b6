// The paper's differential filter (Sec. 3, eq. (12)): ubar solves
// (1 - a^2 lap) ubar = u, with spectral second derivatives in the periodic
// x and z directions and the three-point second difference on the
// non-uniform wall-normal nodes of the flow reflected across both walls as
// in eq. (7).
//
// The operator is diagonal in the real Fourier basis of x and z (cosines
// and sines of the grid wavenumbers share the eigenvalue -k^2), so a field
// is transformed along x and along z (dense real transform matrices on the
// FP32 matrix cores), every (x coefficient, z coefficient) column is then a
// tridiagonal system in y, solved by elimination with factors built once
// per grid, and the result is transformed back.
//
// Stress: u1 is shifted by its plane-mean profile m(y); the twelve fields
// u1', u2, u3, their six products and m u1', m u2, m u3 are filtered, and
//   ubar_1 = F(u1') + M,  M = F(m),
//   tau_11 = F(u1'u1') - F(u1')^2 + 2 (F(m u1') - M F(u1')) + F(m^2) - M^2,
//   tau_1j = F(u1'u_j) - F(u1') F(u_j) + F(m u_j) - M F(u_j)   (j = 2, 3),
//   tau_ij = F(u_i u_j) - F(u_i) F(u_j) otherwise,
// the expansion of u1 = u1' + m, exact for any profile.
#include "eles_internal.h"

namespace eles {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kQT = 4;   // 16-row output tiles per wave of the transforms
// interleaved accumulators of a transform sum: K-step s adds into set
// s % kNA, so each set sums a quarter of the terms and the rounding error
// grows with about half the sequential one
constexpr int kNA = 4;

// |wavenumber| index of real-basis coefficient q of an n-point axis:
// q = 0 .. n/2 are cosines of index q, the rest sines of index q - n/2
__device__ __host__ inline int widx(int q, int n) {
  const int h = n / 2;
  return q <= h ? q : q - h;
}

// ---------------------------------------------------------------- setup

// Forward transform T [qp][kp] (coefficient q from node k) and inverse
// transform I [qp][kp] (node q from coefficient k), zero-padded:
//   cosine s: T = w_s cos(2 pi s k / n), w_0 = w_{n/2} = 1/n, else 2/n;
//   sine s:   T = (2/n) sin(2 pi s k / n);   I is the basis itself.
__global__ void k_dtrans(int n, int qp, int kp, float *T, float *I) {
  const int q = blockIdx.x, k = threadIdx.x + blockIdx.y * blockDim.x;
  if (q >= qp || k >= kp) return;
  float t = 0.0f, v = 0.0f;
  if (q < n && k < n) {
    const int h = n / 2;
    // forward: row q (coefficient), column k (node)
    {
      const bool cosine = q <= h;
      const int s = cosine ? q : q - h;
      const long arg = (2L * s * k) % (2L * n);   // angle / pi, times n
      double sn, cs;
      sincospi((double)arg / n, &sn, &cs);
      const double w = (s == 0 || (cosine && 2 * s == n)) ? 1.0 / n : 2.0 / n;
      t = (float)(cosine ? w * cs : w * sn);
    }
    // inverse: row q (node), column k (coefficient)
    {
      const bool cosine = k <= h;
      const int s = cosine ? k : k - h;
      const long arg = (2L * s * q) % (2L * n);
      double sn, cs;
      sincospi((double)arg / n, &sn, &cs);
      v = (float)(cosine ? cs : sn);
    }
  }
  T[(size_t)q * kp + k] = t;
  I[(size_t)q * kp + k] = v;
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
// sub-diagonal -a^2 lo_j (FP64 arithmetic, FP32 storage).
__global__ void k_dfactor(DView v) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long ncol = (long)(v.hx + 1) * (v.hz + 1);
  if (t >= 2 * ncol) return;
  const int p = (int)(t / ncol);
  const long col = t - p * ncol;
  const int sx = (int)(col / (v.hz + 1)), sz = (int)(col % (v.hz + 1));
  const int ny = v.ny;
  const double a2 = v.a * v.a;
  const double kx = 2.0 * M_PI * sx / v.lx, kz = 2.0 * M_PI * sz / v.lz;
  const double c = 1.0 + a2 * (kx * kx + kz * kz);
  const double *d = v.d64 + (size_t)p * 3 * ny;
  const int j0 = p ? 1 : 0, j1 = p ? ny - 2 : ny - 1;
  float *cp = v.cp + ((size_t)p * ncol + col) * ny;
  float *inv = v.inv + ((size_t)p * ncol + col) * ny;
  double cprev = 0.0;
  for (int j = j0; j <= j1; ++j) {
    const double L = -a2 * d[j], Dg = c - a2 * d[ny + j], U = -a2 * d[2 * ny + j];
    const double den = j == j0 ? Dg : Dg - L * cprev;
    const double cj = U / den;
    cp[j] = (float)cj;
    inv[j] = (float)(1.0 / den);
    cprev = cj;
  }
  if (col == 0)
    for (int j = 0; j < ny; ++j) v.lo32[(size_t)p * ny + j] = (float)(-a2 * d[j]);
}

// ---------------------------------------------------------------- per call

// plane mean of u1 in FP64 -> prof[0] = m (FP32)
__global__ void __launch_bounds__(256) k_dmean(DView v, const float *__restrict__ u1) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  const long cnt = (long)v.nx * v.nz;
  for (long t = threadIdx.x; t < cnt; t += 256) {
    const long x = t / v.nz, z = t - x * v.nz;
    s += (double)u1[((size_t)x * v.ny + j) * v.nz + z];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) v.prof[j] = (float)(red[0] / (double)cnt);
}

// M = F(m) and F(m^2) - M^2 (the zero-wavenumber even system, FP64)
__global__ void k_dprof(DView v) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int ny = v.ny;
  const double a2 = v.a * v.a;
  const double *d = v.d64;   // even
  double *w = v.scratch64;   // [3][ny]: c', r'(m), r'(m^2)
  double cprev = 0.0, r1 = 0.0, r2 = 0.0;
  for (int j = 0; j < ny; ++j) {
    const double L = -a2 * d[j], Dg = 1.0 - a2 * d[ny + j], U = -a2 * d[2 * ny + j];
    const double den = j == 0 ? Dg : Dg - L * cprev;
    const double m = (double)v.prof[j];
    r1 = ((j == 0 ? m : m - L * r1)) / den;
    r2 = ((j == 0 ? m * m : m * m - L * r2)) / den;
    cprev = U / den;
    w[j] = cprev;
    w[ny + j] = r1;
    w[2 * ny + j] = r2;
  }
  double x1 = 0.0, x2 = 0.0;
  for (int j = ny - 1; j >= 0; --j) {
    x1 = w[ny + j] - (j == ny - 1 ? 0.0 : w[j] * x1);
    x2 = w[2 * ny + j] - (j == ny - 1 ? 0.0 : w[j] * x2);
    v.prof[ny + j] = (float)x1;
    v.prof[2 * ny + j] = (float)(x2 - x1 * x1);
  }
}

// the twelve fields of the stress from u and m
__global__ void k_dprod(DView v, const float *__restrict__ u, size_t n, float *__restrict__ out) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int y = (int)((t / v.nz) % v.ny);
  const float m = v.prof[y];
  const float v0 = u[t] - m, v1 = u[n + t], v2 = u[2 * n + t];
  const float q[kDFields] = {v0, v1, v2, v0 * v0, v0 * v1, v0 * v2, v1 * v1, v1 * v2, v2 * v2, m * v0, m * v1, m * v2};
#pragma unroll
  for (int f = 0; f < kDFields; ++f) out[f * n + t] = q[f];
}

// out[b][q][c] = sum_k T[q][k] in[b][k][c]  (transform along a middle axis;
// c contiguous, C columns). One wave: 16 columns x up to kQT 16-row tiles.
__global__ void __launch_bounds__(256) k_dmat_mid(const float *__restrict__ T, int Q, int K, int kp,
                                                  const float *__restrict__ in, float *__restrict__ out, int B,
                                                  long C, size_t bstride) {
  const int lane = threadIdx.x & 63, i = lane & 15, j = lane >> 4;
  const long w = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const long nct = (C + 15) / 16;
  const int nqg = (Q + 16 * kQT - 1) / (16 * kQT);
  const long total = (long)B * nqg * nct;
  if (w >= total) return;
  const int b = (int)(w / ((long)nqg * nct));
  const long r = w - (long)b * nqg * nct;
  const int qg = (int)(r / nct);
  const long c0 = (r - (long)qg * nct) * 16;
  const int q0 = qg * 16 * kQT;
  const int ntile = min(kQT, (Q - q0 + 15) / 16);
  const float *src = in + (size_t)b * bstride;
  const long c = c0 + i;
  f4 acc[kNA][kQT];
#pragma unroll
  for (int g = 0; g < kNA; ++g)
#pragma unroll
    for (int t = 0; t < kQT; ++t) acc[g][t] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 4 * kNA) {
#pragma unroll
    for (int g = 0; g < kNA; ++g) {
      const int k = k0 + 4 * g + j;
      if (k0 + 4 * g >= K) break;
      const float bv = (k < K && c < C) ? src[(size_t)k * C + c] : 0.0f;
#pragma unroll
      for (int t = 0; t < kQT; ++t)
        if (t < ntile) acc[g][t] = mma(T[(size_t)(q0 + 16 * t + i) * kp + k], bv, acc[g][t]);
    }
  }
#pragma unroll
  for (int t = 0; t < kQT; ++t) acc[0][t] = (acc[0][t] + acc[1][t]) + (acc[2][t] + acc[3][t]);
  float *dst = out + (size_t)b * bstride;
#pragma unroll
  for (int t = 0; t < kQT; ++t) {
    if (t >= ntile) break;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int q = q0 + 16 * t + 4 * j + e;
      if (q < Q && c < C) dst[(size_t)q * C + c] = acc[0][t][e];
    }
  }
}

// out[r][q] = sum_k in[r][k] T[q][k]  (transform along the contiguous last
// axis of R rows). One wave: 16 rows x up to kQT 16-column tiles.
__global__ void __launch_bounds__(256) k_dmat_last(const float *__restrict__ T, int Q, int K, int kp,
                                                   const float *__restrict__ in, float *__restrict__ out, long R) {
  const int lane = threadIdx.x & 63, i = lane & 15, j = lane >> 4;
  const long w = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nqg = (Q + 16 * kQT - 1) / (16 * kQT);
  const long nrt = (R + 15) / 16;
  if (w >= nrt * nqg) return;
  const long r0 = (w / nqg) * 16;
  const int qg = (int)(w % nqg);
  const int q0 = qg * 16 * kQT;
  const int ntile = min(kQT, (Q - q0 + 15) / 16);
  const long r = r0 + i;
  f4 acc[kNA][kQT];
#pragma unroll
  for (int g = 0; g < kNA; ++g)
#pragma unroll
    for (int t = 0; t < kQT; ++t) acc[g][t] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 4 * kNA) {
#pragma unroll
    for (int g = 0; g < kNA; ++g) {
      const int k = k0 + 4 * g + j;
      if (k0 + 4 * g >= K) break;
      const float av = (k < K && r < R) ? in[(size_t)r * K + k] : 0.0f;
#pragma unroll
      for (int t = 0; t < kQT; ++t)
        if (t < ntile) acc[g][t] = mma(av, T[(size_t)(q0 + 16 * t + i) * kp + k], acc[g][t]);
    }
  }
#pragma unroll
  for (int t = 0; t < kQT; ++t) acc[0][t] = (acc[0][t] + acc[1][t]) + (acc[2][t] + acc[3][t]);
#pragma unroll
  for (int t = 0; t < kQT; ++t) {
    if (t >= ntile) break;
    const int q = q0 + 16 * t + i;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const long rr = r0 + 4 * j + e;
      if (q < Q && rr < R) out[(size_t)rr * Q + q] = acc[0][t][e];
    }
  }
}

// Tridiagonal solves in y for every (field, x coefficient, z coefficient)
// column, in place: data [f][qx][y][qz]; parity of field f from pmask.
__global__ void __launch_bounds__(256) k_dsolve(DView v, float *__restrict__ d, int nf, unsigned pmask) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long ncolf = (long)v.nx * v.nz;
  if (t >= nf * ncolf) return;
  const int f = (int)(t / ncolf);
  const long col = t - f * ncolf;
  const int qx = (int)(col / v.nz), qz = (int)(col - (long)qx * v.nz);
  const int p = (pmask >> f) & 1;   // 1: odd
  const int ny = v.ny, nz = v.nz;
  const long ncol = (long)(v.hx + 1) * (v.hz + 1);
  const long fc = (long)widx(qx, v.nx) * (v.hz + 1) + widx(qz, v.nz);
  const float *cp = v.cp + ((size_t)p * ncol + fc) * ny;
  const float *inv = v.inv + ((size_t)p * ncol + fc) * ny;
  const float *lo = v.lo32 + (size_t)p * ny;
  float *x = d + ((size_t)f * v.nx + qx) * (size_t)ny * nz + qz;
  const int j0 = p ? 1 : 0, j1 = p ? ny - 2 : ny - 1;
  float r = x[(size_t)j0 * nz] * inv[j0];
  x[(size_t)j0 * nz] = r;
  for (int j = j0 + 1; j <= j1; ++j) {
    r = (x[(size_t)j * nz] - lo[j] * r) * inv[j];
    x[(size_t)j * nz] = r;
  }
  for (int j = j1 - 1; j >= j0; --j) {
    r = x[(size_t)j * nz] - cp[j] * r;
    x[(size_t)j * nz] = r;
  }
  if (p) {
    x[0] = 0.0f;
    x[(size_t)(ny - 1) * nz] = 0.0f;
  }
}

// ubar and tau from the twelve filtered fields g
__global__ void k_depi(DView v, const float *__restrict__ g, size_t n, float *__restrict__ ubar,
                       float *__restrict__ tau) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int y = (int)((t / v.nz) % v.ny);
  const float M = v.prof[v.ny + y], S = v.prof[2 * v.ny + y];
  float G[kDFields];
#pragma unroll
  for (int f = 0; f < kDFields; ++f) G[f] = g[f * n + t];
  ubar[t] = G[0] + M;
  ubar[n + t] = G[1];
  ubar[2 * n + t] = G[2];
  tau[t] = (G[3] - G[0] * G[0]) + 2.0f * (G[9] - M * G[0]) + S;
  tau[n + t] = (G[4] - G[0] * G[1]) + (G[10] - M * G[1]);
  tau[2 * n + t] = (G[5] - G[0] * G[2]) + (G[11] - M * G[2]);
  tau[3 * n + t] = G[6] - G[1] * G[1];
  tau[4 * n + t] = G[7] - G[1] * G[2];
  tau[5 * n + t] = G[8] - G[2] * G[2];
}

unsigned grid_of(long work, int per) { return (unsigned)((work + per - 1) / per); }

}  // namespace

hipError_t launch_dsetup(const DView &v, hipStream_t s) {
  k_dtrans<<<dim3(v.qpx, (v.kpx + 255) / 256), 256, 0, s>>>(v.nx, v.qpx, v.kpx, v.tx, v.itx);
  k_dtrans<<<dim3(v.qpz, (v.kpz + 255) / 256), 256, 0, s>>>(v.nz, v.qpz, v.kpz, v.tz, v.itz);
  k_dsecond<<<grid_of(v.ny, 256), 256, 0, s>>>(v);
  const long ncol = 2L * (v.hx + 1) * (v.hz + 1);
  k_dfactor<<<grid_of(ncol, 64), 64, 0, s>>>(v);
  return hipGetLastError();
}

// fields [nf][nx][ny][nz] in `in` -> filtered in `out`; w0, w1: workspaces
// of nf fields; in may equal w0 (it is only read by the first transform)
hipError_t launch_dfilter(const DView &v, const float *in, int nf, unsigned pmask, float *w0, float *w1, float *out,
                          hipStream_t s) {
  const size_t n = (size_t)v.nx * v.ny * v.nz;
  const long C = (long)v.ny * v.nz;
  const long nqgx = (v.nx + 16 * kQT - 1) / (16 * kQT), nqgz = (v.nz + 16 * kQT - 1) / (16 * kQT);
  const long wx = (long)nf * nqgx * ((C + 15) / 16);
  const long R = (long)nf * v.nx * v.ny;
  const long wz = ((R + 15) / 16) * nqgz;
  // x forward: in -> w1, z forward: w1 -> w0 (may be in: in is no longer needed)
  k_dmat_mid<<<grid_of(wx, 4), 256, 0, s>>>(v.tx, v.nx, v.nx, v.kpx, in, w1, nf, C, n);
  k_dmat_last<<<grid_of(wz, 4), 256, 0, s>>>(v.tz, v.nz, v.nz, v.kpz, w1, w0, R);
  k_dsolve<<<grid_of((long)nf * v.nx * v.nz, 256), 256, 0, s>>>(v, w0, nf, pmask);
  k_dmat_last<<<grid_of(wz, 4), 256, 0, s>>>(v.itz, v.nz, v.nz, v.kpz, w0, w1, R);
  k_dmat_mid<<<grid_of(wx, 4), 256, 0, s>>>(v.itx, v.nx, v.nx, v.kpx, w1, out, nf, C, n);
  return hipGetLastError();
}

hipError_t launch_dsgs(const DView &v, const float *u, float *w0, float *w1, float *ubar, float *tau,
                       hipStream_t s) {
  const size_t n = (size_t)v.nx * v.ny * v.nz;
  k_dmean<<<v.ny, 256, 0, s>>>(v, u);
  k_dprof<<<1, 64, 0, s>>>(v);
  k_dprod<<<grid_of((long)n, 256), 256, 0, s>>>(v, u, n, w0);
  // parities of the twelve fields: u1', u2, u3, products, m u1', m u2, m u3
  const unsigned odd = (1u << 1) | (1u << 4) | (1u << 7) | (1u << 10);
  hipError_t e = launch_dfilter(v, w0, kDFields, odd, w0, w1, w0, s);
  if (e != hipSuccess) return e;
  k_depi<<<grid_of((long)n, 256), 256, 0, s>>>(v, w0, n, ubar, tau);
  return hipGetLastError();
}

}  // namespace eles
