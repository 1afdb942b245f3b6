// The learned closure: a 10-64-64-64-6 perceptron with GELU hidden layers
// that maps the filtered velocity gradient and the wall distance to the six
// components of the exact stress. Weights and activations are BF16 on the
// matrix cores with FP32 accumulation; master weights, Adam moments and the
// loss are FP32 / FP64.
//
// Training runs layer by layer over a minibatch drawn with SplitMix64
// (counter-based, so a step's batch depends only on the seed and the step
// index): every product is C = A B^T with K-contiguous operands, activations
// are kept in both orientations so the weight gradients reduce over the
// batch as contiguous K, and split-K partials are summed in a fixed order by
// the Adam kernel. Inference runs all four layers of a 16-point tile inside
// one wave, activations staying in registers and a 2 KB LDS transpose.
#include "k_gemm.cuh"

namespace eles {
namespace {

constexpr int H = kMlpHidden;
constexpr int K1 = kMlpInPad;

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline uint64_t draw_index(uint64_t seed, uint64_t n, uint64_t count) {
  return ((splitmix64(seed, n) >> 32) * count) >> 32;
}

// ---------------------------------------------------------------- sampler

__global__ void __launch_bounds__(256) k_sample(uint64_t seed, long step, int batch, uint64_t count,
                                                int64_t *out) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= batch) return;
  out[b] = (int64_t)draw_index(seed, (uint64_t)step * batch + b, count);
}

// Draw the minibatch of `step` and gather standardised features and targets.
__global__ void __launch_bounds__(256) k_gather(ClosureView c, TrainData d, uint64_t seed, long step, int batch,
                                                uint16_t *x0, uint16_t *x0t, float *tb) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= batch) return;
  const uint64_t count = (uint64_t)d.nsnap * (uint64_t)d.npts;
  const uint64_t idx = draw_index(seed, (uint64_t)step * batch + b, count);
  const uint64_t s = idx / (uint64_t)d.npts, p = idx % (uint64_t)d.npts;
  const float *fs = d.feat + s * (uint64_t)kMlpIn * d.npts + p;
  const float *ts = d.tau + s * (uint64_t)kMlpOut * d.npts + p;
  uint32_t packed[K1 / 2];
#pragma unroll
  for (int q = 0; q < K1 / 2; ++q) packed[q] = 0u;
#pragma unroll
  for (int f = 0; f < kMlpIn; ++f) {
    const float v = fs[(uint64_t)f * d.npts] * c.fsc[f] + c.fsh[f];
    const uint16_t h = g_bf16(v);
    packed[f / 2] |= (uint32_t)h << (16 * (f % 2));
    x0t[(long)f * batch + b] = h;
  }
  uint4 *row = reinterpret_cast<uint4 *>(x0 + (long)b * K1);
#pragma unroll
  for (int q = 0; q < K1 / 8; ++q)
    row[q] = make_uint4(packed[4 * q], packed[4 * q + 1], packed[4 * q + 2], packed[4 * q + 3]);
#pragma unroll
  for (int o = 0; o < kMlpOut; ++o) tb[(long)b * 8 + o] = ts[(uint64_t)o * d.npts] * c.tsc[o] + c.tsh[o];
}

// ---------------------------------------------------------------- products

enum { E_HIDDEN = 0, E_OUT = 1, E_DX = 2, E_DW = 3 };

struct EpiArgs {
  const float *bias;      // hidden / out: bias of this layer (FP32 master)
  int nvalid;             // out: number of real outputs
  long batch;
  uint16_t *h, *ht, *g;   // hidden: activation, its transpose, GELU'
  const float *tb;        // out: standardised targets [batch][8]
  uint16_t *dy, *dyt;     // out: loss gradient and its transpose
  double *lossp;          // out: per-wave partial sums of squared errors
  float dscale;           // out: 2 / (batch * outputs)
  const uint16_t *gin;    // dx: GELU' of the layer input
  uint16_t *dz, *dzt;     // dx: gradient at the pre-activation (either may be null)
  float *pw, *pb;         // dw: weight / bias partials [chunk][M][N], [chunk][M]
  int ldg;                // row length of h, g, dz (features)
};

template <int KIND, int NT>
struct Epi {
  const EpiArgs &e;
  int chunk;
  int M, N;
  __device__ void operator()(long m0, int n0, gf4 (&acc)[NT], float rowsum, int) const {
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, grp = lane >> 4;
    if (KIND == E_HIDDEN) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int n = n0 + 16 * t + col;
        const float bia = e.bias[n];
        uint16_t hv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long m = m0 + 4 * grp + r;
          const float z = acc[t][r] + bia;
          hv[r] = g_bf16(gelu(z));
          e.h[m * e.ldg + n] = hv[r];
          e.g[m * e.ldg + n] = g_bf16(gelu_grad(z));
        }
        uint2 pk = make_uint2(hv[0] | ((uint32_t)hv[1] << 16), hv[2] | ((uint32_t)hv[3] << 16));
        *reinterpret_cast<uint2 *>(e.ht + (long)n * e.batch + m0 + 4 * grp) = pk;
      }
    } else if (KIND == E_OUT) {
      double sq = 0.0;
      const int n = n0 + col;
      const bool valid = n < e.nvalid;
      const float bia = valid ? e.bias[n] : 0.0f;
      uint16_t dv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long m = m0 + 4 * grp + r;
        float d = 0.0f;
        if (valid) {
          d = acc[0][r] + bia - e.tb[m * 8 + n];
          sq += (double)d * d;
        }
        dv[r] = g_bf16(e.dscale * d);
        e.dy[m * kMlpInPad + n] = dv[r];
      }
      uint2 pk = make_uint2(dv[0] | ((uint32_t)dv[1] << 16), dv[2] | ((uint32_t)dv[3] << 16));
      *reinterpret_cast<uint2 *>(e.dyt + (long)n * e.batch + m0 + 4 * grp) = pk;
      for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
      if (lane == 0) e.lossp[m0 / 16] = sq;
    } else if (KIND == E_DX) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int n = n0 + 16 * t + col;
        uint16_t dv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long m = m0 + 4 * grp + r;
          dv[r] = g_bf16(acc[t][r] * g_f32(e.gin[m * e.ldg + n]));
          if (e.dz) e.dz[m * e.ldg + n] = dv[r];
        }
        uint2 pk = make_uint2(dv[0] | ((uint32_t)dv[1] << 16), dv[2] | ((uint32_t)dv[3] << 16));
        *reinterpret_cast<uint2 *>(e.dzt + (long)n * e.batch + m0 + 4 * grp) = pk;
      }
    } else {  // E_DW
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int n = n0 + 16 * t + col;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = (int)m0 + 4 * grp + r;
          if (m < M && n < N) e.pw[((long)chunk * M + m) * N + n] = acc[t][r];
        }
      }
      float s = rowsum;
      s += __shfl_xor(s, 16);
      s += __shfl_xor(s, 32);
      const int m = (int)m0 + col;
      if (n0 == 0 && grp == 0 && m < M) e.pb[(long)chunk * M + m] = s;
    }
  }
};

template <int KIND, int NT>
__global__ void __launch_bounds__(256) k_train_gemm(NTArgs g, EpiArgs e, int mtiles, int nchunks) {
  const long item = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int mt = (int)(item % mtiles);
  const long ch = item / mtiles;
  if (ch >= nchunks) return;
  const int k32 = (g.K + 31) & ~31;
  const int kb = (int)ch * g.kchunk;
  const int ke = min(k32, kb + g.kchunk);
  Epi<KIND, NT> epi{e, (int)ch, (int)g.M, g.N};
  nt_gemm_wave<0, NT>(g, (long)mt * 16, blockIdx.y * 16 * NT, kb, ke, 0, epi);
}

// ------------------------------------------------------------------- Adam

struct ParamLoc {
  int layer, bias, n, k;
};

__device__ inline ParamLoc locate(int p) {
  const int fin[4] = {kMlpIn, H, H, H};
  const int fout[4] = {H, H, H, kMlpOut};
  ParamLoc L{0, 0, 0, 0};
  int o = 0;
  for (int l = 0; l < 4; ++l) {
    const int nw = fin[l] * fout[l];
    if (p < o + nw) {
      L.layer = l;
      L.n = (p - o) / fin[l];
      L.k = (p - o) % fin[l];
      return L;
    }
    o += nw;
    if (p < o + fout[l]) {
      L.layer = l;
      L.bias = 1;
      L.n = p - o;
      return L;
    }
    o += fout[l];
  }
  return L;
}

// Padded BF16 shadows: rows of W_l and of W_l^T as the products read them.
__device__ inline void write_shadow(const ClosureView &c, const ParamLoc &L, float w) {
  const uint16_t h = g_bf16(w);
  switch (L.layer) {
    case 0: c.w1[L.n * K1 + L.k] = h; break;
    case 1: c.w2[L.n * H + L.k] = h; c.w2t[L.k * H + L.n] = h; break;
    case 2: c.w3[L.n * H + L.k] = h; c.w3t[L.k * H + L.n] = h; break;
    default: c.w4[L.n * H + L.k] = h; c.w4t[L.k * K1 + L.n] = h; break;
  }
}

// Sum the split-K partials of every gradient in a fixed order, then apply
// one Adam step; thread 0 also totals the loss of the step.
__global__ void __launch_bounds__(256) k_adam(ClosureView c, AdamArgs a) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p == 0 && a.loss_out) {
    double s = 0.0;
    for (int w = 0; w < a.nloss; ++w) s += a.lossp[w];
    a.loss_out[0] = (float)(s / ((double)a.batch * kMlpOut));
  }
  if (p >= kMlpNParam) return;
  const ParamLoc L = locate(p);
  const int fin[4] = {kMlpIn, H, H, H};
  const int fout[4] = {H, H, H, kMlpOut};
  const int M = a.mrows[L.layer], N = a.ncols[L.layer];
  (void)fout;
  double gsum = 0.0;
  if (L.bias) {
    const float *pb = a.pb[L.layer];
    for (int ch = 0; ch < a.nchunks; ++ch) gsum += pb[(long)ch * M + L.n];
  } else {
    const float *pw = a.pw[L.layer];
    for (int ch = 0; ch < a.nchunks; ++ch) gsum += pw[((long)ch * M + L.n) * N + L.k];
  }
  (void)fin;
  const float g = (float)gsum;
  const float m = a.b1 * c.m[p] + (1.0f - a.b1) * g;
  const float v = a.b2 * c.v[p] + (1.0f - a.b2) * g * g;
  c.m[p] = m;
  c.v[p] = v;
  const float th = c.theta[p] - a.lr * (m * a.bc1) / (sqrtf(v * a.bc2) + a.eps);
  c.theta[p] = th;
  if (!L.bias) write_shadow(c, L, th);
}

__global__ void __launch_bounds__(256) k_shadows(ClosureView c) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kMlpNParam) return;
  const ParamLoc L = locate(p);
  if (!L.bias) write_shadow(c, L, c.theta[p]);
}

// -------------------------------------------------------------- inference

constexpr int kInferBlocks = 2048;

// All four layers of 16-point tiles; the weights sit in LDS, activations of
// a tile go through a per-wave 16 x 64 BF16 transpose.
__global__ void __launch_bounds__(256) k_infer(ClosureView c, const float *__restrict__ feat, long npts,
                                               float *__restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint16_t sw1[H * K1], sw2[H * H], sw3[H * H], sw4[16 * H];
  __shared__ float sb[3 * H + 16];
  __shared__ __attribute__((aligned(16))) uint16_t sh[4][16 * H];
  for (int i = threadIdx.x; i < H * K1; i += 256) sw1[i] = c.w1[i];
  for (int i = threadIdx.x; i < H * H; i += 256) {
    sw2[i] = c.w2[i];
    sw3[i] = c.w3[i];
  }
  for (int i = threadIdx.x; i < 16 * H; i += 256) sw4[i] = c.w4[i];
  for (int i = threadIdx.x; i < 3 * H + 16; i += 256) {
    float b = 0.0f;
    if (i < H) b = c.theta[kMlpOffB1 + i];
    else if (i < 2 * H) b = c.theta[kMlpOffB2 + i - H];
    else if (i < 3 * H) b = c.theta[kMlpOffB3 + i - 2 * H];
    else if (i - 3 * H < kMlpOut) b = c.theta[kMlpOffB4 + i - 3 * H];
    sb[i] = b;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  uint16_t *hs = sh[wave];
  const long ntile = (npts + 15) / 16;
  for (long tile = (long)blockIdx.x * 4 + wave; tile < ntile; tile += (long)gridDim.x * 4) {
    const long p = tile * 16 + col;
    const bool pok = p < npts;
    // standardised features of point p, features 8 grp .. 8 grp + 7
    gus8 xb = gus8{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int f = 8 * grp + e;
      if (f < kMlpIn && pok) xb[e] = g_bf16(feat[(long)f * npts + p] * c.fsc[f] + c.fsh[f]);
    }
    gus8 bk[2];
    // layer 1: K = 32 (one step)
    {
      gf4 acc[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const gus8 aw = *reinterpret_cast<const gus8 *>(sw1 + (16 * t + col) * K1 + 8 * grp);
        acc[t] = g_mma(aw, xb, gf4{0.f, 0.f, 0.f, 0.f});
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        uint16_t hv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) hv[r] = g_bf16(gelu(acc[t][r] + sb[16 * t + 4 * grp + r]));
        *reinterpret_cast<uint2 *>(hs + col * H + 16 * t + 4 * grp) =
            make_uint2(hv[0] | ((uint32_t)hv[1] << 16), hv[2] | ((uint32_t)hv[3] << 16));
      }
    }
    // layers 2 and 3: K = 64 (two steps)
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const uint16_t *sw = l == 0 ? sw2 : sw3;
      const float *bb = sb + (l + 1) * H;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int s = 0; s < 2; ++s) bk[s] = *reinterpret_cast<const gus8 *>(hs + col * H + 32 * s + 8 * grp);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      gf4 acc[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc[t] = gf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const gus8 aw = *reinterpret_cast<const gus8 *>(sw + (16 * t + col) * H + 32 * s + 8 * grp);
          acc[t] = g_mma(aw, bk[s], acc[t]);
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        uint16_t hv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) hv[r] = g_bf16(gelu(acc[t][r] + bb[16 * t + 4 * grp + r]));
        *reinterpret_cast<uint2 *>(hs + col * H + 16 * t + 4 * grp) =
            make_uint2(hv[0] | ((uint32_t)hv[1] << 16), hv[2] | ((uint32_t)hv[3] << 16));
      }
    }
    // output layer
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int s = 0; s < 2; ++s) bk[s] = *reinterpret_cast<const gus8 *>(hs + col * H + 32 * s + 8 * grp);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    gf4 acc = gf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const gus8 aw = *reinterpret_cast<const gus8 *>(sw4 + col * H + 32 * s + 8 * grp);
      acc = g_mma(aw, bk[s], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * grp + r;
      if (o < kMlpOut && pok) out[(long)o * npts + p] = (acc[r] + sb[3 * H + o]) * c.isc[o] + c.ish[o];
    }
  }
}

// --------------------------------------------------------- moments, sums

// pass 0: per-chunk sums; pass 1: per-chunk sums of squared deviations from mean
__global__ void __launch_bounds__(256) k_mom_part(const float *data, int nchan, int nsnap, long npts, long chunk,
                                                  const double *mean, double *part, int nchunks) {
  __shared__ double red[256];
  const int c = blockIdx.y, q = blockIdx.x;
  const long total = (long)nsnap * npts;
  const long b = (long)q * chunk, e = min(total, b + chunk);
  const double mu = mean ? mean[c] : 0.0;
  double s = 0.0;
  for (long i = b + threadIdx.x; i < e; i += 256) {
    const long sn = i / npts, p = i % npts;
    const double v = (double)data[(sn * nchan + c) * npts + p] - mu;
    s += mean ? v * v : v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long)c * nchunks + q] = red[0];
}

__global__ void k_mom_final(const double *part, int nchunks, int nchan, double count, double *out, int pass) {
  const int c = threadIdx.x;
  if (c >= nchan) return;
  double s = 0.0;
  for (int q = 0; q < nchunks; ++q) s += part[(long)c * nchunks + q];
  if (pass == 0)
    out[c] = s / count;
  else
    out[nchan + c] = sqrt(s / count);
}

// <f_q>(y_j) over x and z for planar fields [nq][nx][ny][nz], FP64 sums.
__global__ void __launch_bounds__(256) k_plane_mean(const float *f, int nx, int ny, int nz, double *out) {
  __shared__ double red[256];
  const int j = blockIdx.x, q = blockIdx.y;
  const long cnt = (long)nx * nz;
  const float *base = f + (long)q * nx * ny * nz;
  double s = 0.0;
  for (long t = threadIdx.x; t < cnt; t += 256) {
    const long x = t / nz, z = t % nz;
    s += (double)base[(x * ny + j) * nz + z];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(long)q * ny + j] = red[0] / (double)cnt;
}

}  // namespace

// ------------------------------------------------------------- launchers

hipError_t launch_sample(uint64_t seed, long step, int batch, uint64_t count, int64_t *out, hipStream_t s) {
  k_sample<<<(batch + 255) / 256, 256, 0, s>>>(seed, step, batch, count, out);
  return hipGetLastError();
}

hipError_t launch_shadows(const ClosureView &c, hipStream_t s) {
  k_shadows<<<(kMlpNParam + 255) / 256, 256, 0, s>>>(c);
  return hipGetLastError();
}

hipError_t launch_infer(const ClosureView &c, const float *feat, long npts, float *out, hipStream_t s) {
  const long tiles = (npts + 15) / 16;
  long blocks = (tiles + 3) / 4;
  if (blocks > kInferBlocks) blocks = kInferBlocks;
  k_infer<<<(unsigned)blocks, 256, 0, s>>>(c, feat, npts, out);
  return hipGetLastError();
}

hipError_t launch_moments(const float *data, int nchan, int nsnap, long npts, double *part, int nchunks,
                          double *out, hipStream_t s) {
  const long total = (long)nsnap * npts;
  const long chunk = (total + nchunks - 1) / nchunks;
  k_mom_part<<<dim3(nchunks, nchan), 256, 0, s>>>(data, nchan, nsnap, npts, chunk, nullptr, part, nchunks);
  k_mom_final<<<1, 64, 0, s>>>(part, nchunks, nchan, (double)total, out, 0);
  k_mom_part<<<dim3(nchunks, nchan), 256, 0, s>>>(data, nchan, nsnap, npts, chunk, out, part, nchunks);
  k_mom_final<<<1, 64, 0, s>>>(part, nchunks, nchan, (double)total, out, 1);
  return hipGetLastError();
}

hipError_t launch_plane_mean(const float *f, int nq, int nx, int ny, int nz, double *out, hipStream_t s) {
  k_plane_mean<<<dim3(ny, nq), 256, 0, s>>>(f, nx, ny, nz, out);
  return hipGetLastError();
}

// One optimisation step over the minibatch of `step`.
hipError_t launch_train_step(const ClosureView &c, const TrainData &d, const TrainWs &w, uint64_t seed, long step,
                             int batch, AdamArgs adam, hipStream_t s) {
  hipError_t e;
  const int B = batch;
  k_gather<<<(B + 255) / 256, 256, 0, s>>>(c, d, seed, step, B, w.x0, w.x0t, w.tb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int mt = B / 16;
  const unsigned gb = (unsigned)((mt + 3) / 4);
  const uint16_t *hin[4] = {w.x0, w.h[0], w.h[1], w.h[2]};
  const uint16_t *wl[4] = {c.w1, c.w2, c.w3, c.w4};
  const int kin[4] = {K1, H, H, H};
  const int boff[4] = {kMlpOffB1, kMlpOffB2, kMlpOffB3, kMlpOffB4};
  // forward, hidden layers
  for (int l = 0; l < 3; ++l) {
    NTArgs g{hin[l], kin[l], wl[l], nullptr, kin[l], (long)B, H, kin[l], kin[l], 0, 0};
    EpiArgs ea{};
    ea.bias = c.theta + boff[l];
    ea.batch = B;
    ea.h = w.h[l];
    ea.ht = w.ht[l];
    ea.g = w.g[l];
    ea.ldg = H;
    k_train_gemm<E_HIDDEN, 4><<<gb, 256, 0, s>>>(g, ea, mt, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // output layer, loss and its gradient
  {
    NTArgs g{w.h[2], H, c.w4, nullptr, H, (long)B, 16, H, H, 0, 0};
    EpiArgs ea{};
    ea.bias = c.theta + kMlpOffB4;
    ea.nvalid = kMlpOut;
    ea.batch = B;
    ea.tb = w.tb;
    ea.dy = w.dy;
    ea.dyt = w.dyt;
    ea.lossp = w.lossp;
    ea.dscale = 2.0f / ((float)B * kMlpOut);
    k_train_gemm<E_OUT, 1><<<gb, 256, 0, s>>>(g, ea, mt, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // backward: weight gradients (split over the batch) and input gradients
  const int kc = kMlpChunk;
  const int nch = (B + kc - 1) / kc;
  const uint16_t *dzt_l[4] = {w.dzt[0], w.dzt[1], w.dzt[2], w.dyt};
  const uint16_t *hint[4] = {w.x0t, w.ht[0], w.ht[1], w.ht[2]};
  const int mrows[4] = {H, H, H, 16};
  const int ncols[4] = {kMlpIn, H, H, H};
  for (int l = 3; l >= 0; --l) {
    if (l < 3) {
      // dZ_l = (dZ_{l+1} W_{l+1}) * GELU'(Z_l)
      const uint16_t *a_in = l == 2 ? w.dy : w.dz[l + 1];
      const int kdim = l == 2 ? K1 : H;
      const uint16_t *wt = l == 2 ? c.w4t : (l == 1 ? c.w3t : c.w2t);
      NTArgs g{a_in, kdim, wt, nullptr, kdim, (long)B, H, kdim, kdim, 0, 0};
      EpiArgs ea{};
      ea.batch = B;
      ea.gin = w.g[l];
      ea.dz = l > 0 ? w.dz[l] : nullptr;
      ea.dzt = w.dzt[l];
      ea.ldg = H;
      k_train_gemm<E_DX, 4><<<gb, 256, 0, s>>>(g, ea, mt, 1);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // dW_l = dZ_l^T H_{l-1}, db_l = sum over the batch of dZ_l
    NTArgs g{dzt_l[l], B, hint[l], nullptr, B, (long)mrows[l], ncols[l], B, kc, 0, 0};
    EpiArgs ea{};
    ea.pw = w.pw[l];
    ea.pb = w.pb[l];
    const int mtl = (mrows[l] + 15) / 16;
    const unsigned gw = (unsigned)((mtl * nch + 3) / 4);
    if (ncols[l] > 16)
      k_train_gemm<E_DW, 4><<<gw, 256, 0, s>>>(g, ea, mtl, nch);
    else
      k_train_gemm<E_DW, 1><<<gw, 256, 0, s>>>(g, ea, mtl, nch);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  adam.nchunks = nch;
  adam.lossp = w.lossp;
  adam.nloss = mt;
  adam.batch = B;
  for (int l = 0; l < 4; ++l) {
    adam.pw[l] = w.pw[l];
    adam.pb[l] = w.pb[l];
    adam.mrows[l] = mrows[l];
    adam.ncols[l] = ncols[l];
  }
  k_adam<<<(kMlpNParam + 255) / 256, 256, 0, s>>>(c, adam);
  return hipGetLastError();
}

}  // namespace eles
