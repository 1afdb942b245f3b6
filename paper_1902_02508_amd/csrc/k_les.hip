// The stress on an LES grid (Sec. 2, the discrete filtered equations):
// T_ij = I(F(u_i u_j)) - I(F(u_i)) I(F(u_j)), with I the discretization
// operator, second-order linear interpolation from the DNS grid to the LES
// grid (Sec. 4), and the commutation error of I with the second-order
// wall-normal derivative.
//
// With F(u_i u_j) = tau_ij + ubar_i ubar_j on the DNS grid and the
// interpolation weights w_c of the eight DNS corners of an LES node summing
// to one,
//   T_ij = I(tau_ij) + sum_c w_c (ubar_i^c - I ubar_i)(ubar_j^c - I ubar_j),
// the weighted covariance of the corner velocities: no difference of large
// products is formed.
#include "eles_internal.h"

namespace eles {
namespace {

// corner weights and flat DNS offsets of LES node (xl, yl, zl)
struct Corners {
  float w[8];
  size_t off[8];
};
__device__ inline Corners corners(const LesView &v, int xl, int yl, int zl) {
  Corners c;
  const int x0 = v.ix[xl], y0 = v.iy[yl], z0 = v.iz[zl];
  const int x1 = x0 + 1 == v.nx ? 0 : x0 + 1, y1 = y0 + 1, z1 = z0 + 1 == v.nz ? 0 : z0 + 1;
  const float wx = v.wx[xl], wy = v.wy[yl], wz = v.wz[zl];
  const int xs[2] = {x0, x1}, ys[2] = {y0, y1}, zs[2] = {z0, z1};
  const float fx[2] = {1.0f - wx, wx}, fy[2] = {1.0f - wy, wy}, fz[2] = {1.0f - wz, wz};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const int k = 4 * a + 2 * b + d;
        c.w[k] = fx[a] * fy[b] * fz[d];
        c.off[k] = ((size_t)xs[a] * v.ny + ys[b]) * v.nz + zs[d];
      }
  return c;
}

// thread per LES node: tilde(ubar) [3] and T [6]
__global__ void __launch_bounds__(256) k_les_stress(LesView v, const float *__restrict__ ubar,
                                                    const float *__restrict__ tau, float *__restrict__ ul,
                                                    float *__restrict__ T) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nl = (size_t)v.nxl * v.nyl * v.nzl;
  if (t >= nl) return;
  const int zl = (int)(t % v.nzl);
  const int yl = (int)((t / v.nzl) % v.nyl);
  const int xl = (int)(t / ((size_t)v.nzl * v.nyl));
  const size_t n = (size_t)v.nx * v.ny * v.nz;
  const Corners c = corners(v, xl, yl, zl);
  float u[3][8], iu[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    iu[i] = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      u[i][k] = ubar[i * n + c.off[k]];
      iu[i] += c.w[k] * u[i][k];
    }
    ul[i * nl + t] = iu[i];
  }
  const int P[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int i = P[q][0], j = P[q][1];
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += c.w[k] * (tau[q * n + c.off[k]] + (u[i][k] - iu[i]) * (u[j][k] - iu[j]));
    T[q * nl + t] = s;
  }
}

// second-order d/dy of g at DNS node (x, j, z) / of I g at LES node row jl
__device__ inline double ddy_dns(const LesView &v, const float *__restrict__ g, int x, int j, int z) {
  const int b = v.db[j];
  const size_t o = ((size_t)x * v.ny + b) * v.nz + z;
  return v.dc[3 * j] * g[o] + v.dc[3 * j + 1] * g[o + v.nz] + v.dc[3 * j + 2] * g[o + 2 * (size_t)v.nz];
}
__device__ inline double interp(const LesView &v, const float *__restrict__ g, int xl, int yl, int zl) {
  const Corners c = corners(v, xl, yl, zl);
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += (double)c.w[k] * g[c.off[k]];
  return s;
}

// Commutation error partials, block (xc, yl) over kLxc LES x nodes: FP64
// sums of (A - B)^2 and B^2 with A = d_y^LES(I g), B = I(d_y^DNS g),
// part[(q nyl + yl) nxc + xc].
constexpr int kLxc = 16;
__global__ void __launch_bounds__(256) k_les_comm(LesView v, const float *__restrict__ g, double *__restrict__ part) {
  __shared__ double red[4][2];
  const int xc = blockIdx.x, yl = blockIdx.y, nxc = gridDim.x;
  const int x0 = xc * kLxc, x1 = min(v.nxl, x0 + kLxc);
  const int cnt = (x1 - x0) * v.nzl;
  double sa = 0.0, sb = 0.0;
  const int bl = v.lb[yl];
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int xo = e / v.nzl, zl = e - xo * v.nzl;
    const int xl = x0 + xo;
    const double A = v.lc[3 * yl] * interp(v, g, xl, bl, zl) + v.lc[3 * yl + 1] * interp(v, g, xl, bl + 1, zl) +
                     v.lc[3 * yl + 2] * interp(v, g, xl, bl + 2, zl);
    // B: the interpolation of the DNS derivative, corner by corner
    const int xa = v.ix[xl], ya = v.iy[yl], za = v.iz[zl];
    const int xb = xa + 1 == v.nx ? 0 : xa + 1, zb = za + 1 == v.nz ? 0 : za + 1;
    const double wx = v.wx[xl], wy = v.wy[yl], wz = v.wz[zl];
    const double d00 = (1 - wz) * ddy_dns(v, g, xa, ya, za) + wz * ddy_dns(v, g, xa, ya, zb);
    const double d01 = (1 - wz) * ddy_dns(v, g, xa, ya + 1, za) + wz * ddy_dns(v, g, xa, ya + 1, zb);
    const double d10 = (1 - wz) * ddy_dns(v, g, xb, ya, za) + wz * ddy_dns(v, g, xb, ya, zb);
    const double d11 = (1 - wz) * ddy_dns(v, g, xb, ya + 1, za) + wz * ddy_dns(v, g, xb, ya + 1, zb);
    const double B = (1 - wx) * ((1 - wy) * d00 + wy * d01) + wx * ((1 - wy) * d10 + wy * d11);
    sa += (A - B) * (A - B);
    sb += B * B;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sa += __shfl_xor(sa, o);
    sb += __shfl_xor(sb, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = sa;
    red[threadIdx.x >> 6][1] = sb;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int q = threadIdx.x;
    part[((size_t)q * v.nyl + yl) * nxc + xc] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  }
}

// out = sqrt(sum_yl w_yl sum (A-B)^2 / sum_yl w_yl sum B^2), chunks in order
__global__ void __launch_bounds__(256) k_les_comm_final(LesView v, const double *__restrict__ part, int nxc,
                                                        double *__restrict__ out) {
  __shared__ double red[4][2];
  double sa = 0.0, sb = 0.0;
  for (int yl = threadIdx.x; yl < v.nyl; yl += blockDim.x) {
    double a = 0.0, b = 0.0;
    for (int c = 0; c < nxc; ++c) {
      a += part[(size_t)yl * nxc + c];
      b += part[((size_t)v.nyl + yl) * nxc + c];
    }
    sa += v.lw[yl] * a;
    sb += v.lw[yl] * b;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sa += __shfl_xor(sa, o);
    sb += __shfl_xor(sb, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = sa;
    red[threadIdx.x >> 6][1] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double a = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
    const double b = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    out[0] = sqrt(a / b);
  }
}

}  // namespace

hipError_t launch_les_stress(const LesView &v, const float *ubar, const float *tau, float *ul, float *T,
                             hipStream_t s) {
  const size_t nl = (size_t)v.nxl * v.nyl * v.nzl;
  k_les_stress<<<(unsigned)((nl + 255) / 256), 256, 0, s>>>(v, ubar, tau, ul, T);
  return hipGetLastError();
}

long les_comm_parts(const LesView &v) { return 2L * v.nyl * ((v.nxl + kLxc - 1) / kLxc); }

hipError_t launch_les_commutation(const LesView &v, const float *g, double *part, double *out, hipStream_t s) {
  const int nxc = (v.nxl + kLxc - 1) / kLxc;
  k_les_comm<<<dim3(nxc, v.nyl), 256, 0, s>>>(v, g, part);
  k_les_comm_final<<<1, 256, 0, s>>>(v, part, nxc, out);
  return hipGetLastError();
}

}  // namespace eles
