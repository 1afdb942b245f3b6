// Plane means of FP32 fields in FP64, and the non-finite test on them.
//
// This unit is built with IEEE semantics (no finite-math assumptions), so
// a NaN or an infinity anywhere in a plane carries into that plane's FP64
// sum (finite FP32 values cannot overflow an FP64 sum of a plane), and the
// test reads the sums' exponent bits as integers.
#include "eles_internal.h"

namespace eles {
namespace {

// <f_q>(y_j) over x and z for planar fields [nq][nx][ny][nz], FP64 sums:
// each block adds an x-range of one (q, j) plane, a second kernel adds the
// kPlaneSplit partial sums in order.
constexpr int kPlaneSplit = 16;

__global__ void __launch_bounds__(256) k_plane_part(const float *f, int nx, int ny, int nz, double *part) {
  __shared__ double red[256];
  const int j = blockIdx.x, q = blockIdx.y, sp = blockIdx.z;
  const int xb = (int)((long)nx * sp / kPlaneSplit), xe = (int)((long)nx * (sp + 1) / kPlaneSplit);
  const float *base = f + (long)q * nx * ny * nz;
  double s = 0.0;
  // element t = (x - xb) nz + z of the slab, walked with 32-bit (x, z)
  // steps of 256 (no division per element)
  int x = xb + (int)threadIdx.x / nz, z = (int)threadIdx.x % nz;
  const int dx = 256 / nz, dz = 256 % nz;
  while (x < xe) {
    s += (double)base[((long)x * ny + j) * nz + z];
    x += dx;
    z += dz;
    if (z >= nz) {
      z -= nz;
      ++x;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[((long)q * ny + j) * kPlaneSplit + sp] = red[0];
}

__global__ void __launch_bounds__(256) k_plane_final(const double *part, int n, double inv, double *out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int sp = 0; sp < kPlaneSplit; ++sp) s += part[(long)i * kPlaneSplit + sp];
  out[i] = s * inv;
}

// <f_q>(y_j) from the FP64 sums of each (x, y) row, rows[q][x ny + j]:
// one block per (j, q), thread t adding x = t, t + 256, ... in order, then
// a fixed tree over the threads
__global__ void __launch_bounds__(256) k_row_means(const double *rows, int nx, int ny, double inv, double *out) {
  __shared__ double red[256];
  const int j = blockIdx.x, q = blockIdx.y;
  const double *r = rows + (long)q * nx * ny + j;
  double s = 0.0;
  for (int x = threadIdx.x; x < nx; x += 256) s += r[(long)x * ny];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q * ny + j] = red[0] * inv;
}

// flag = 1 if any of v[0..n) has an all-ones exponent (NaN or infinity),
// else 0; one block.
__global__ void __launch_bounds__(256) k_nonfinite(const double *v, int n, int *flag) {
  int bad = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v[i]);
    bad |= ((b >> 52) & 0x7ffull) == 0x7ffull;
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) *flag = bad ? 1 : 0;
}

}  // namespace

hipError_t launch_plane_mean(const float *f, int nq, int nx, int ny, int nz, double *part, double *out,
                             hipStream_t s) {
  k_plane_part<<<dim3(ny, nq, kPlaneSplit), 256, 0, s>>>(f, nx, ny, nz, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_plane_final<<<(nq * ny + 255) / 256, 256, 0, s>>>(part, nq * ny, 1.0 / ((double)nx * nz), out);
  return hipGetLastError();
}

hipError_t launch_row_means(const double *rows, int nq, int nx, int ny, int nz, double *out, hipStream_t s) {
  k_row_means<<<dim3(ny, nq), 256, 0, s>>>(rows, nx, ny, 1.0 / ((double)nx * nz), out);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const double *v, int n, int *flag, hipStream_t s) {
  k_nonfinite<<<1, 256, 0, s>>>(v, n, flag);
  return hipGetLastError();
}

}  // namespace eles
