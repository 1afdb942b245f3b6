// Gradient operators of the closure features, built in FP64 on the device,
// and the z-derivative product.
//
// x and z: the Fourier differentiation matrix of a periodic grid of n
// nodes and period L, D_ij = (pi/L) (-1)^(i-j) cot(pi (i-j)/n) for even n
// (the Nyquist mode differentiates to zero) and (pi/L) (-1)^(i-j)
// csc(pi (i-j)/n) for odd n, zero diagonal. It is the derivative of the
// trigonometric interpolant, i.e. the spectral derivative, as a dense
// circulant applied on the matrix cores.
//
// y: the three-point Lagrange derivative on the non-uniform nodes; at a
// wall the node across it is the mirror of the first interior node,
// carrying the field's parity under the extension of eq. (7), so the wall
// row is 0 for even fields and f_1/(y_1 - y_0) (resp. -f_{n-2}/...) for odd.
#include "k_gemm.h"

namespace eles {
namespace {

__device__ inline void put(float *a32, uint16_t *hi, uint16_t *lo, size_t o, double w) {
  const float f = (float)w;
  if (a32) a32[o] = f;
  const uint16_t h = g_bf16(f);
  hi[o] = h;
  lo[o] = g_bf16(f - g_f32(h));
}

// Dense spectral differentiation matrix, padded to [mp][kp], row bands full.
__global__ void __launch_bounds__(256) k_dspec(int n, double length, int mp, int kp, float *a32, uint16_t *hi,
                                               uint16_t *lo, int *band) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)mp * kp) return;
  const int i = (int)(idx / kp), j = (int)(idx % kp);
  double w = 0.0;
  if (i < n && j < n && i != j) {
    const int d = i - j;
    const double ang = M_PI * d / n;
    const double sgn = (d & 1) ? -1.0 : 1.0;
    w = (M_PI / length) * sgn * ((n % 2 == 0) ? cos(ang) / sin(ang) : 1.0 / sin(ang));
  }
  put(a32, hi, lo, idx, w);
  if (j == 0 && band) {
    band[2 * i] = 0;
    band[2 * i + 1] = i < n ? n : 0;
  }
}

__global__ void __launch_bounds__(256) k_dy(const double *y, int ny, int mp, int kp, float *e32, uint16_t *ehi,
                                            uint16_t *elo, float *o32, uint16_t *ohi, uint16_t *olo, int *band) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)mp * kp) return;
  const int i = (int)(idx / kp), j = (int)(idx % kp);
  double we = 0.0, wo = 0.0;
  if (i > 0 && i < ny - 1 && j >= i - 1 && j <= i + 1) {
    const double h1 = y[i] - y[i - 1], h2 = y[i + 1] - y[i];
    if (j == i - 1) we = -h2 / (h1 * (h1 + h2));
    if (j == i) we = (h2 - h1) / (h1 * h2);
    if (j == i + 1) we = h1 / (h2 * (h1 + h2));
    wo = we;
  } else if (i == 0 && j == 1) {
    wo = 1.0 / (y[1] - y[0]);
  } else if (i == ny - 1 && j == ny - 2) {
    wo = -1.0 / (y[ny - 1] - y[ny - 2]);
  }
  put(e32, ehi, elo, idx, we);
  put(o32, ohi, olo, idx, wo);
  if (j == 0) {
    band[2 * i] = i < ny ? (i > 0 ? i - 1 : 0) : 0;
    band[2 * i + 1] = i < ny ? (i + 2 < ny ? i + 2 : ny) : 0;
  }
}

// d/dy of the three filtered velocities, one lane per (field, y segment,
// x, z) walking its rows with a three-value window: the interior rows of
// the operator are the central three-point differences (columns j - 1 ..
// j + 1), the wall rows those of the mirror extension (columns 0, 1 and
// ny - 2, ny - 1), with the FP32 weights of the operator rows built by
// k_dy. Rows are requested in chunks of kDyU, the next chunk before the
// current one is used; kDySeg segments per column keep enough columns in
// flight.
constexpr int kDyU = 8;
constexpr int kDySeg = 4;
__global__ void __launch_bounds__(64) k_ddy(GradView v, const float *__restrict__ u, float *__restrict__ out,
                                            long ofs, unsigned pmask) {
  const int z = blockIdx.x * 64 + threadIdx.x;
  const int x = blockIdx.y, f = blockIdx.z / kDySeg, sg = blockIdx.z % kDySeg;
  const int ny = v.ny, nz = v.nz;
  const int per = (ny + kDySeg - 1) / kDySeg;
  const int jb = sg * per, je = min(ny, jb + per);   // rows [jb, je) of this segment
  if (z >= nz || jb >= je) return;
  const long kp = v.kpy;
  const float *D = ((pmask >> f) & 1) ? v.dy32[1] : v.dy32[0];
  const size_t n = (size_t)v.nx * ny * nz;
  const float *uc = u + f * n + (size_t)x * ny * nz + z;
  float *oc = out + f * ofs + (size_t)x * ny * nz + z;
  // window: rows j - 1 and j (row 0 has no j - 1; its weight reads row 0)
  float um = uc[(size_t)max(jb - 1, 0) * nz], u0 = uc[(size_t)jb * nz];
  float a[kDyU], b[kDyU];
  // w[e] = row j0 + e + 1 (clamped), the j + 1 of row j0 + e
  auto fetch = [&](float (&w)[kDyU], int j0) {
#pragma unroll
    for (int e = 0; e < kDyU; ++e) w[e] = uc[(size_t)min(j0 + e + 1, ny - 1) * nz];
  };
  auto rows = [&](const float (&w)[kDyU], int j0) {
#pragma unroll
    for (int e = 0; e < kDyU; ++e) {
      const int j = j0 + e;
      if (j < je) {
        float o;
        if (j == 0) {
          o = D[0] * u0 + D[1] * w[e];
        } else if (j == ny - 1) {
          const float *Dl = D + (long)j * kp + (j - 1);
          o = Dl[0] * um + Dl[1] * u0;
        } else {
          const float *Dr = D + (long)j * kp + (j - 1);
          o = Dr[0] * um + Dr[1] * u0 + Dr[2] * w[e];
        }
        oc[(size_t)j * nz] = o;
        um = u0;
        u0 = w[e];
      }
    }
  };
  fetch(a, jb);
  for (int j0 = jb; j0 < je; j0 += 2 * kDyU) {
    fetch(b, j0 + kDyU);
    rows(a, j0);
    if (j0 + kDyU >= je) break;
    fetch(a, j0 + 2 * kDyU);
    rows(b, j0 + kDyU);
  }
}

__global__ void __launch_bounds__(256) k_walldist(const double *y, int nx, int ny, int nz, float *out) {
  const long n = (long)nx * ny * nz;
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  const int j = (int)((idx / nz) % ny);
  out[idx] = (float)(1.0 - fabs(y[j]));
}

struct EpiStore {
  float *out;        // field z of the output at out + z * out_bstride
  long out_bstride;
  long M;
  int N, ldo;
  __device__ void operator()(long m0, int n0, gf4 (&acc)[4], float, int z) const {
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int n = n0 + 16 * t + col;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long m = m0 + 4 * grp + r;
        if (m < M && n < N) out[z * out_bstride + m * ldo + n] = acc[t][r];
      }
    }
  }
};

// rows of every field times D^T: the derivative along the contiguous axis
__global__ void __launch_bounds__(256) k_dz(NTArgs g, EpiStore e) {
  const long mtile = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (mtile * 16 >= g.M) return;
  const int k32 = (g.K + 31) & ~31;
  EpiStore epi = e;
  nt_gemm_wave<2, 4>(g, mtile * 16, blockIdx.y * 64, 0, k32, blockIdx.z, epi);
}

}  // namespace

hipError_t launch_build_grad_ops(const GradView &v, const double *y64, hipStream_t s) {
  long n = (long)v.mpx * v.kpx;
  k_dspec<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(v.nx, v.lx, v.mpx, v.kpx, v.dx32, v.dxhi, v.dxlo,
                                                      v.dxband);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  n = (long)v.mpz * v.kpz;
  k_dspec<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(v.nz, v.lz, v.mpz, v.kpz, nullptr, v.dzhi, v.dzlo,
                                                      nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  n = (long)v.mpy * v.kpy;
  k_dy<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(y64, v.ny, v.mpy, v.kpy, v.dy32[0], v.dyhi[0], v.dylo[0],
                                                   v.dy32[1], v.dyhi[1], v.dylo[1], v.dyband);
  return hipGetLastError();
}

hipError_t launch_dz(const GradView &v, const float *ubar, float *out, long out_fstride, hipStream_t s) {
  const long npts = (long)v.nx * v.ny * v.nz;
  const long M = (long)v.nx * v.ny;
  NTArgs g{ubar, v.nz, v.dzhi, v.dzlo, v.kpz, M, v.nz, v.nz, (v.nz + 31) & ~31, npts, 0};
  EpiStore e{out, out_fstride, M, v.nz, v.nz};
  const long mtiles = (M + 15) / 16;
  dim3 grid((unsigned)((mtiles + 3) / 4), (unsigned)((v.nz + 63) / 64), 3);
  k_dz<<<grid, 256, 0, s>>>(g, e);
  return hipGetLastError();
}

hipError_t launch_ddy(const GradView &v, const float *ubar, float *out, long out_fstride, unsigned pmask,
                      hipStream_t s) {
  if (v.ny < 3) return hipErrorInvalidValue;
  k_ddy<<<dim3((unsigned)((v.nz + 63) / 64), (unsigned)v.nx, 3 * kDySeg), 64, 0, s>>>(v, ubar, out, out_fstride,
                                                                                   pmask);
  return hipGetLastError();
}

hipError_t launch_walldist(const double *y64, int nx, int ny, int nz, float *out, hipStream_t s) {
  const long n = (long)nx * ny * nz;
  k_walldist<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(y64, nx, ny, nz, out);
  return hipGetLastError();
}

}  // namespace eles
