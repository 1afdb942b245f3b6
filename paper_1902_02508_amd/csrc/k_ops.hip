// Operator build, FP64 on the device.
//
// x and z: the periodic direction is sampled by the rectangle rule
// (Sec. 2.1, eq. (2)); the stencil keeps the kernel at offsets -m..m, each
// periodic image being a separate offset when m exceeds the period, and is
// normalised to unit sum.
//
// y: eq. (2) on the wall-normal line extended by reflection about both walls
// with the parities of eq. (7) (Sec. 2.2); the extension repeats with period
// 4. Node j contributes directly at y_j + 4n and, if interior, as a mirror
// image at 4n + 2 - y_j with the field's parity as sign. Trapezoid weights
// of the extended line give a wall node a full cell. Rows are normalised by
// the all-positive sum; an odd field's wall values are ignored (it vanishes
// there, eq. (11)).
//
// Mean shift (per call): u1 is replaced by u1 - m(y) before products are
// formed; the exact correction operators C^s = W^s diag(m) - diag(W^+ m) W^s
// and the profiles M = W^+ m, s = W^+ m^2 - M^2 are built here in FP64.
#include "eles_internal.h"

namespace eles {
namespace {

constexpr int kT = 256;

__device__ inline double kernel_val(double r, double delta) {
  // unit-integral Gaussian with variance delta^2/12
  return sqrt(6.0 / (M_PI * delta * delta)) * exp(-6.0 * r * r / (delta * delta));
}

__device__ inline bool kept(double r, double delta, double tau) {
  return exp(-6.0 * r * r / (delta * delta)) >= tau;
}

// Deterministic tree sum over the block (blockDim.x == kT).
__device__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__device__ int block_min(int v, int *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  int r = red[0];
  __syncthreads();
  return r;
}

__device__ int block_max(int v, int *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  int r = red[0];
  __syncthreads();
  return r;
}

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ inline uint16_t bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__device__ inline float bf16_val(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ inline void store_operator(const OpsView &v, int which, int i, int j, double w) {
  size_t o = (size_t)i * v.kpad + j;
  float f = (float)w;
  v.a32[which][o] = f;
  uint16_t hi = bf16_rne(f);
  v.ahi[which][o] = hi;
  v.alo[which][o] = bf16_rne(f - bf16_val(hi));
}

// FP64 taps for offsets -m..m and their FP32 copy in the zero-padded layout
// the stencils read: entry q holds the tap of offset q - (kXzTileX - 1) - m.
__global__ void __launch_bounds__(kT) k_taps(OpsView v) {
  __shared__ double red[kT];
  const bool isx = blockIdx.x == 0;
  const int n = isx ? v.nx : v.nz;
  const int m = isx ? v.mx : v.mz;
  const double h = (isx ? v.lx : v.lz) / n;
  const double delta = isx ? v.dx : v.dz;
  double *w64 = isx ? v.wx64 : v.wz64;
  float *w32 = isx ? v.wx32 : v.wz32;
  for (int q = threadIdx.x; q < tap_pad_len(m); q += kT) w32[q] = 0.0f;
  double part = 0.0;
  for (int t = threadIdx.x; t <= 2 * m; t += kT) {
    double r = (t - m) * h;
    double val = kept(r, delta, v.tau) ? h * kernel_val(r, delta) : 0.0;
    w64[t] = val;
    part += val;
  }
  double z = block_sum(part, red);
  for (int t = threadIdx.x; t <= 2 * m; t += kT) {
    double w = w64[t] / z;
    w64[t] = w;
    w32[t + kXzTileX - 1] = (float)w;
  }
}

__device__ inline double wall_cell(const double *y, int ny, int j) {
  if (j == 0) return y[1] - y[0];
  if (j == ny - 1) return y[ny - 1] - y[ny - 2];
  return 0.5 * (y[j + 1] - y[j - 1]);
}

// Unnormalised direct and mirror sums for every (i, j).
__global__ void __launch_bounds__(kT) k_yraw(OpsView v, int nimg) {
  const int ny = v.ny;
  const long idx = (long)blockIdx.x * kT + threadIdx.x;
  if (idx >= (long)ny * ny) return;
  const int i = (int)(idx / ny), j = (int)(idx % ny);
  const double yi = v.y64[i], yj = v.y64[j];
  const double om = wall_cell(v.y64, ny, j);
  const bool interior = j > 0 && j < ny - 1;
  double dsum = 0.0, msum = 0.0;
  for (int n = -nimg; n <= nimg; ++n) {
    double rd = yi - (yj + 4.0 * n);
    if (kept(rd, v.dy, v.tau)) dsum += om * kernel_val(rd, v.dy);
    double rm = yi - (4.0 * n + 2.0 - yj);
    if (interior && kept(rm, v.dy, v.tau)) msum += om * kernel_val(rm, v.dy);
  }
  v.wp64[idx] = dsum + msum;
  v.wm64[idx] = dsum - msum;
}

// Normalise row i, emit the padded FP32 / BF16 copies and the row's band.
__global__ void __launch_bounds__(kT) k_ynorm(OpsView v) {
  __shared__ double red[kT];
  __shared__ int ired[kT];
  const int i = blockIdx.x, ny = v.ny;
  if (i < ny) {
    double part = 0.0;
    for (int j = threadIdx.x; j < ny; j += kT) part += v.wp64[(size_t)i * ny + j];
    const double z = block_sum(part, red);
    int lo = 1 << 30, hi = -1;
    for (int j = threadIdx.x; j < ny; j += kT) {
      size_t o = (size_t)i * ny + j;
      double wp = v.wp64[o] / z;
      double wm = (j == 0 || j == ny - 1) ? 0.0 : v.wm64[o] / z;
      v.wp64[o] = wp;
      v.wm64[o] = wm;
      store_operator(v, 0, i, j, wp);
      store_operator(v, 1, i, j, wm);
      store_operator(v, 2, i, j, 0.0);
      store_operator(v, 3, i, j, 0.0);
      if (wp != 0.0 || wm != 0.0) {
        lo = min(lo, j);
        hi = max(hi, j);
      }
    }
    for (int j = ny + threadIdx.x; j < v.kpad; j += kT)
      for (int w = 0; w < 4; ++w) store_operator(v, w, i, j, 0.0);
    lo = block_min(lo, ired);
    hi = block_max(hi, ired);
    if (threadIdx.x == 0) {
      v.rowband[2 * i] = hi >= 0 ? lo : 0;
      v.rowband[2 * i + 1] = hi + 1;
    }
  } else {
    for (int j = threadIdx.x; j < v.kpad; j += kT)
      for (int w = 0; w < 4; ++w) store_operator(v, w, i, j, 0.0);
    if (threadIdx.x == 0) {
      v.rowband[2 * i] = 0;
      v.rowband[2 * i + 1] = 0;
    }
  }
  if (threadIdx.x < 3) v.prof32[threadIdx.x * v.mpad + i] = 0.0f;
}

// m(y_j): mean of u1 over z and kMeanSlabs evenly spaced x-slabs, rounded to FP32.
__global__ void __launch_bounds__(kT) k_mean(OpsView v, const float *u1) {
  __shared__ double red[kT];
  const int j = blockIdx.x;
  const int ns = v.nx < kMeanSlabs ? v.nx : kMeanSlabs;
  const int sx = v.nx / ns;
  const long cnt = (long)ns * v.nz;
  double part = 0.0;
  // element t = q nz + z of slab row q, t = threadIdx + kT k: eight
  // elements are requested together (independent loads), then summed in
  // order
  const int cnt_i = ns * v.nz;
  for (int t0 = (int)threadIdx.x; t0 < cnt_i; t0 += 8 * kT) {
    float w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int t = t0 + k * kT;
      const bool ok = t < cnt_i;
      const int tc = ok ? t : 0;   // in-bounds address for the unused lanes
      const int q = tc / v.nz, z = tc - q * v.nz;
      const float val = u1[((size_t)(q * sx) * v.ny + j) * v.nz + z];
      w[k] = ok ? val : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) part += (double)w[k];
  }
  double s = block_sum(part, red);
  if (threadIdx.x == 0) {
    float m = (float)(s / (double)cnt);
    v.prof32[j] = m;
    v.shift64[j] = (double)m;
  }
}

__global__ void __launch_bounds__(kT) k_shift(OpsView v) {
  __shared__ double red[kT];
  const int i = blockIdx.x, ny = v.ny;
  const double *m = v.shift64;
  if (i < ny) {
    double part = 0.0;
    for (int j = threadIdx.x; j < ny; j += kT) part += v.wp64[(size_t)i * ny + j] * m[j];
    const double M = block_sum(part, red);
    part = 0.0;
    for (int j = threadIdx.x; j < ny; j += kT) {
      double d = m[j] - M;
      part += v.wp64[(size_t)i * ny + j] * d * d;
    }
    const double s = block_sum(part, red);
    for (int j = threadIdx.x; j < ny; j += kT) {
      size_t o = (size_t)i * ny + j;
      double d = m[j] - M;
      store_operator(v, 2, i, j, v.wp64[o] * d);
      store_operator(v, 3, i, j, v.wm64[o] * d);
    }
    if (threadIdx.x == 0) {
      v.shift64[ny + i] = M;
      v.shift64[2 * ny + i] = s;
      v.prof32[v.mpad + i] = (float)M;
      v.prof32[2 * v.mpad + i] = (float)s;
    }
  } else if (threadIdx.x == 0) {
    v.prof32[v.mpad + i] = 0.0f;
    v.prof32[2 * v.mpad + i] = 0.0f;
  }
}

}  // namespace

hipError_t launch_build_ops(const OpsView &v, hipStream_t s) {
  k_taps<<<2, kT, 0, s>>>(v);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double cut = v.dy * sqrt(log(1.0 / v.tau) / 6.0);
  const int nimg = (int)ceil((cut + 4.0) / 4.0) + 1;
  const long nn = (long)v.ny * v.ny;
  k_yraw<<<(unsigned)((nn + kT - 1) / kT), kT, 0, s>>>(v, nimg);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_ynorm<<<v.mpad, kT, 0, s>>>(v);
  return hipGetLastError();
}

hipError_t launch_shift_ops(const OpsView &v, const float *u1, hipStream_t s) {
  k_mean<<<v.ny, kT, 0, s>>>(v, u1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_shift<<<v.mpad, kT, 0, s>>>(v);
  return hipGetLastError();
}

}  // namespace eles
