// The learned closure: a 10-64-64-64-6 perceptron with GELU hidden layers
// that maps the filtered velocity gradient and the wall distance to the six
// components of the exact stress. Training runs BF16 weights and
// activations on the matrix cores with FP32 accumulation; master weights,
// Adam moments and the loss are FP32 / FP64. Inference runs FP16 weights
// and activations (the GELU in packed FP16).
//
// Training runs layer by layer over a minibatch drawn with SplitMix64
// (counter-based, so a step's batch depends only on the seed and the step
// index): every product is C = A B^T with K-contiguous operands, activations
// are kept in both orientations so the weight gradients reduce over the
// batch as contiguous K, and split-K partials are summed in a fixed order by
// the Adam kernel. Inference runs all four layers of a 16-point tile inside
// one wave, weights held in registers, activations through a 2 KB LDS
// transpose, and adds up each (x, y) row of its outputs for the plane
// means.
#include "k_gemm.h"

namespace eles {
namespace {

constexpr int H = kMlpHidden;
constexpr int K1 = kMlpInPad;
// word 3 of a raw buffer descriptor on gfx9-family parts (32-bit data
// format, no swizzle)
constexpr int kBufWord3 = 0x00020000;

// GELU(x) = x Phi(x) evaluated without transcendentals: max(x, 0) - h(s),
// s = min(|x|, 4), h(s) = sum_k c_k s^k (k = 1..7) fitted to s Phi(-s) with
// c_1 = 1/2; within 2.4e-4 of x Phi(x), below the BF16 resolution of the
// activations, and free of the branches of an erf evaluation.
__device__ inline float gelu_h(float s) {
  float h = -0.0006385124288499355f;
  h = fmaf(h, s, 0.009885221719741821f);
  h = fmaf(h, s, -0.05751597508788109f);
  h = fmaf(h, s, 0.14029717445373535f);
  h = fmaf(h, s, -0.04402020201086998f);
  h = fmaf(h, s, -0.3894234895706177f);
  h = fmaf(h, s, 0.5f);
  return h * s;
}
__device__ inline float gelu(float z) { return fmaxf(z, 0.0f) - gelu_h(fminf(fabsf(z), 4.0f)); }
__device__ inline float gelu_grad(float z) {
  const float s = fabsf(z);
  float d = 7.0f * -0.0006385124288499355f;
  d = fmaf(d, s, 6.0f * 0.009885221719741821f);
  d = fmaf(d, s, 5.0f * -0.05751597508788109f);
  d = fmaf(d, s, 4.0f * 0.14029717445373535f);
  d = fmaf(d, s, 3.0f * -0.04402020201086998f);
  d = fmaf(d, s, 2.0f * -0.3894234895706177f);
  d = fmaf(d, s, 0.5f);
  d = s < 4.0f ? d : 0.0f;
  return z >= 0.0f ? 1.0f - d : d;
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
// G_ij = sum_k c_k g_ik g_jk for the six pairs (11, 12, 13, 22, 23, 33) of
// the raw gradient features g_ik = feat(3 i + k); zeros without the term.
template <class Feat>
__device__ inline void gradient_model(const ClosureView &c, Feat feat, float *gm) {
  if (!c.use_gm) {
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) gm[o] = 0.0f;
    return;
  }
  float g[9];
#pragma unroll
  for (int f = 0; f < 9; ++f) g[f] = feat(f);
  constexpr int pi[kMlpOut] = {0, 0, 0, 1, 1, 2}, pj[kMlpOut] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int o = 0; o < kMlpOut; ++o) {
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) acc = fmaf(c.gmc[k] * g[3 * pi[o] + k], g[3 * pj[o] + k], acc);
    gm[o] = acc;
  }
}

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
  float gm[kMlpOut];
  gradient_model(c, [&](int f) { return fs[(uint64_t)f * d.npts]; }, gm);
#pragma unroll
  for (int o = 0; o < kMlpOut; ++o) tb[(long)b * 8 + o] = (ts[(uint64_t)o * d.npts] - gm[o]) * c.tsc[o] + c.tsh[o];
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
// one Adam step. Eight lanes share a parameter: lane j adds chunks j, j+8,
// ... in order and the eight sums are combined by a fixed butterfly. The
// last block totals the loss of the step.
constexpr int kAdamLanes = 8;
constexpr int kAdamPerBlock = 256 / kAdamLanes;

__global__ void __launch_bounds__(256) k_adam(ClosureView c, AdamArgs a) {
  __shared__ double red[256];
  if (blockIdx.x == gridDim.x - 1) {
    double s = 0.0;
    for (int w = threadIdx.x; w < a.nloss; w += 256) s += a.lossp[w];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0 && a.loss_out) a.loss_out[0] = (float)(red[0] / ((double)a.batch * kMlpOut));
    return;
  }
  const int sub = threadIdx.x % kAdamLanes;
  const int p = blockIdx.x * kAdamPerBlock + threadIdx.x / kAdamLanes;
  const bool live = p < kMlpNParam;
  const ParamLoc L = locate(live ? p : 0);
  const int M = a.mrows[L.layer], N = a.ncols[L.layer];
  double gsum = 0.0;
  if (L.bias) {
    const float *pb = a.pb[L.layer] + L.n;
#pragma unroll 4
    for (int ch = sub; ch < a.nchunks; ch += kAdamLanes) gsum += pb[(long)ch * M];
  } else {
    const float *pw = a.pw[L.layer] + (long)L.n * N + L.k;
#pragma unroll 4
    for (int ch = sub; ch < a.nchunks; ch += kAdamLanes) gsum += pw[(long)ch * M * N];
  }
  gsum += __shfl_xor(gsum, 1);
  gsum += __shfl_xor(gsum, 2);
  gsum += __shfl_xor(gsum, 4);
  if (!live || sub != 0) return;
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

constexpr int kInferWavesPerCu = 16;


__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- inference arithmetic: FP16 weights and activations on the matrix
// cores (v_mfma_f32_16x16x32_f16, FP32 accumulation) and the GELU in packed
// FP16, two values per instruction. The GELU is the same max(x, 0) - h(s),
// s = min(|x|, 4), with h a degree-7 polynomial in u = s/2 - 1 fitted to
// s Phi(-s) with FP16 coefficients (within 2.4e-4 of x Phi(x) in exact
// arithmetic): Horner in u keeps the intermediates below one in magnitude,
// where the powers of s would cancel from tens and lose the FP16 digits.
typedef _Float16 gh2 __attribute__((ext_vector_type(2)));
typedef _Float16 gh8 __attribute__((ext_vector_type(8)));

__device__ inline gh2 gelu16_h(gh2 u) {
  gh2 h = (gh2)(_Float16)-0.0816650390625f;
  h = h * u + (_Float16)0.05841064453125f;
  h = h * u + (_Float16)0.239013671875f;
  h = h * u + (_Float16)-0.32568359375f;
  h = h * u + (_Float16)0.0142974853515625f;
  h = h * u + (_Float16)0.2218017578125f;
  h = h * u + (_Float16)-0.171630859375f;
  h = h * u + (_Float16)0.04534912109375f;
  return h;
}

// GELU of two FP32 pre-activations, returned as two FP16 (low, high)
__device__ inline uint32_t gelu16x2(float a, float b) {
  const gh2 x = __builtin_convertvector(gf2{a, b}, gh2);
  const gh2 s = __builtin_elementwise_min(__builtin_elementwise_abs(x), (gh2){(_Float16)4.0f, (_Float16)4.0f});
  const gh2 h = gelu16_h(s * (_Float16)0.5f - (_Float16)1.0f);
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(x, (gh2){(_Float16)0.0f, (_Float16)0.0f}) - h);
}

__device__ inline uint32_t h16x2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(gf2{a, b}, gh2));
}

__device__ inline gf4 h_mma(gus8 a, gus8 b, gf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(gh8, a), __builtin_bit_cast(gh8, b), c, 0, 0, 0);
}

// eight FP32 weights (zero past n) as an FP16 A fragment
__device__ inline gus8 w16(const float *w, int n) {
  uint32_t q[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) q[e] = h16x2(2 * e < n ? w[2 * e] : 0.0f, 2 * e + 1 < n ? w[2 * e + 1] : 0.0f);
  return __builtin_bit_cast(gus8, q);
}

struct InferArgs {
  ClosureView c;
  const float *feat;   // features 0..8 of [10][npts]; the wall distance is computed
  long npts;
  int nx, ny, nz;
  const double *y64;   // the grid's y nodes
  float *out;          // [6][npts]
  double *rows;        // [6][nx ny] sums of each output over a (x, y) row, or null
};

// All four layers of 16-point tiles. Each wave walks whole (x, y) rows of
// the grid (row = wave, wave + nwaves, ...), a row as ceil(nz / 16) tiles
// of 16 consecutive z, fetching the next tile's features while the current
// one is computed. It keeps its A fragments of W1 and W4 in registers (W2
// and W3 in LDS, which leaves 128 registers: four waves per SIMD),
// converted from the FP32 master weights; a tile's
// activations go through a per-wave 16 x 64 FP16 LDS transpose between
// layers; each layer's products start from its bias. The wall-distance
// feature 1 - |y| is the row's (the same FP32 value the feature kernel
// stores). With rows given, every lane adds its outputs of the row in FP64
// in tile order and the sixteen points of a tile are then added across
// lanes in a fixed butterfly: the (x, y) row sums, deterministic, which
// the plane means reduce over x.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_infer(InferArgs a) {
  const ClosureView &c = a.c;
  // LDS rows of W2, W3 and of the activation transposes are HP = H + 8 halves
  // (36 words): the sixteen lanes of a lane group, one row each, then fall
  // on disjoint banks (a 32-word stride puts them all on the same ones)
  constexpr int HP = H + 8;
  __shared__ __attribute__((aligned(16))) float sb[3 * H + 16];
  __shared__ __attribute__((aligned(16))) uint16_t sw3[H * HP];
  __shared__ __attribute__((aligned(16))) uint16_t sw2[H * HP];
  __shared__ __attribute__((aligned(16))) uint16_t sh[4][16 * HP];
  for (int i = threadIdx.x; i < 3 * H + 16; i += 256) {
    float b = 0.0f;
    if (i < H) b = c.theta[kMlpOffB1 + i];
    else if (i < 2 * H) b = c.theta[kMlpOffB2 + i - H];
    else if (i < 3 * H) b = c.theta[kMlpOffB3 + i - 2 * H];
    else if (i - 3 * H < kMlpOut) b = c.theta[kMlpOffB4 + i - 3 * H];
    sb[i] = b;
  }
  const float *W1 = c.theta, *W2 = c.theta + kMlpOffB1 + H, *W3 = c.theta + kMlpOffB2 + H,
              *W4 = c.theta + kMlpOffB3 + H;
  for (int i = threadIdx.x; i < H * H / 8; i += 256) {
    const int n = i / (H / 8), k = 8 * (i % (H / 8));
    *reinterpret_cast<gus8 *>(sw3 + n * HP + k) = w16(W3 + n * H + k, 8);
    *reinterpret_cast<gus8 *>(sw2 + n * HP + k) = w16(W2 + n * H + k, 8);
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  uint16_t *hs = sh[wave];
  gus8 a1[4], a4[2];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    a1[t] = w16(W1 + (16 * t + col) * kMlpIn + 8 * grp, grp == 0 ? 8 : (grp == 1 ? kMlpIn - 8 : 0));
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) a4[s] = w16(W4 + (col < kMlpOut ? col : 0) * H + 32 * s + 8 * grp, col < kMlpOut ? 8 : 0);
  // lane (point col, group grp) carries features 8 grp .. 8 grp + 7; of
  // group 1, feature 8 is loaded and feature 9 is the wall distance
  const int nf = grp == 0 ? 8 : (grp == 1 ? kMlpIn - 8 : 0);
  const int nload = grp == 0 ? 8 : (grp == 1 ? 1 : 0);
  float fsc[8], fsh[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    fsc[e] = e < nf ? c.fsc[8 * grp + e] : 0.0f;
    fsh[e] = e < nf ? c.fsh[8 * grp + e] : 0.0f;
  }
  // The row cursor is wave-uniform (scalar registers): each tile reads
  // and writes through buffer descriptors of its row's piece of every
  // plane (nz floats), so points past nz read zeros and drop their stores,
  // and a lane outside a load's or store's lane group gets an offset past
  // the range.
  const int nrows = a.nx * a.ny;
  const int ntz = (a.nz + 15) / 16;
  const int nw = (int)gridDim.x * 4;
  const long npts = a.npts;
  const unsigned nbytes = (unsigned)a.nz * 4u, kOut = 0x80000000u;
  auto plane = [&](const float *base, int q, int r) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)(base + (long)q * npts + (long)r * a.nz), 0, (int)nbytes,
                                             kBufWord3);
  };
  int row = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wave);
  int zb = 0;
  float fv[8];
  auto fetch = [&](int r, int b) {
    const unsigned off = (unsigned)(16 * b + col) * 4u;
    const unsigned o0 = grp == 0 && r < nrows ? off : kOut, o1 = grp == 1 && r < nrows ? off : kOut;
    const int rr = __builtin_amdgcn_readfirstlane(r < nrows ? r : 0);
#pragma unroll
    for (int e = 0; e < 8; ++e)
      fv[e] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(plane(a.feat, e, rr), o0, 0, 0));
    const float f8 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(plane(a.feat, 8, rr), o1, 0, 0));
    fv[0] = grp == 1 ? f8 : fv[0];
  };
  fetch(row, zb);
  double rs[4] = {0.0, 0.0, 0.0, 0.0};
  float wall = row < nrows ? (float)(1.0 - fabs(a.y64[row % a.ny])) : 0.0f;
  while (row < nrows) {
    const int z = 16 * zb + col;
    const bool pok = z < a.nz;
    const unsigned zoff = (unsigned)z * 4u;
    if (grp == 1) fv[1] = wall;
    uint32_t xw[4];
    {
      float xs[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) xs[e] = e < nf ? fv[e] * fsc[e] + fsh[e] : 0.0f;
#pragma unroll
      for (int e = 0; e < 4; ++e) xw[e] = h16x2(xs[2 * e], xs[2 * e + 1]);
    }
    const gus8 xb = __builtin_bit_cast(gus8, xw);
    // gradient-model term of this lane's outputs 4 grp + r, from the raw
    // features of the current tile (lanes of group 0 hold features 0..7,
    // of group 1 features 8, 9; the others are exchanged)
    float gmr[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (c.use_gm) {
      const float t8 = __shfl(fv[0], 16 + col, 64);
      float g[9];
#pragma unroll
      for (int e = 3; e < 8; ++e) {
        const float o = __shfl(fv[e], col, 64);
        g[e] = grp == 0 ? fv[e] : o;
      }
      g[0] = fv[0];
      g[1] = fv[1];
      g[2] = fv[2];
      g[8] = grp == 0 ? t8 : fv[0];
      float G[kMlpOut];
      gradient_model(c, [&](int f) { return g[f]; }, G);
#pragma unroll
      for (int r = 0; r < 4; ++r) gmr[r] = grp == 0 ? G[r] : (r < 2 ? G[4 + r] : 0.0f);
    }
    // advance the cursor and request the next tile's features
    const int crow = __builtin_amdgcn_readfirstlane(row);
    if (++zb == ntz) {
      zb = 0;
      row = __builtin_amdgcn_readfirstlane(row + nw);
    }
    fetch(row, zb);
    auto bias = [&](int base, int t) { return *reinterpret_cast<const gf4 *>(sb + base + 16 * t + 4 * grp); };
    gf4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = h_mma(a1[t], xb, bias(0, t));
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      // GELU of layer l, transposed through LDS into the next B operand
#pragma unroll
      for (int t = 0; t < 4; ++t)
        *reinterpret_cast<uint2 *>(hs + col * HP + 16 * t + 4 * grp) =
            make_uint2(gelu16x2(acc[t][0], acc[t][1]), gelu16x2(acc[t][2], acc[t][3]));
      wave_sync();
      gus8 bk[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) bk[s] = *reinterpret_cast<const gus8 *>(hs + col * HP + 32 * s + 8 * grp);
      wave_sync();
      if (l < 2) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          acc[t] = bias((l + 1) * H, t);
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const gus8 aw = l == 0 ? *reinterpret_cast<const gus8 *>(sw2 + (16 * t + col) * HP + 32 * s + 8 * grp)
                                   : *reinterpret_cast<const gus8 *>(sw3 + (16 * t + col) * HP + 32 * s + 8 * grp);
            acc[t] = h_mma(aw, bk[s], acc[t]);
          }
        }
      } else {
        gf4 y = bias(3 * H, 0);   // output biases, zero past the sixth row
#pragma unroll
        for (int s = 0; s < 2; ++s) y = h_mma(a4[s], bk[s], y);
        // lane group 0 holds outputs 0..3, group 1 outputs 4, 5
        const unsigned s0 = grp == 0 ? zoff : kOut, s1 = grp == 1 ? zoff : kOut;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = 4 * grp + r;
          const float v = y[r] * c.isc[o < kMlpOut ? o : 0] + c.ish[o < kMlpOut ? o : 0] + gmr[r];
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), plane(a.out, r, crow), s0, 0, 0);
          if (r < 2)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), plane(a.out, 4 + r, crow), s1, 0, 0);
          rs[r] += (o < kMlpOut && pok) ? (double)v : 0.0;
        }
      }
    }
    if (row != crow) {
      // the row is done: its sums across the sixteen points, then reset
      if (a.rows) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
          for (int m = 1; m < 16; m <<= 1) rs[r] += __shfl_xor(rs[r], m, 64);
        }
        if (col == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int o = 4 * grp + r;
            if (o < kMlpOut) a.rows[(long)o * nrows + crow] = rs[r];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) rs[r] = 0.0;
      if (row < nrows) wall = (float)(1.0 - fabs(a.y64[row % a.ny]));
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

hipError_t launch_infer(const ClosureView &c, const float *feat, int nx, int ny, int nz, const double *y64,
                        float *out, double *rows, hipStream_t s) {
  const long nrows = (long)nx * ny;
  long blocks = (nrows + 3) / 4;
  const long cap = 256L * kInferWavesPerCu / 4;   // every wave keeps its weights for many rows
  if (blocks > cap) blocks = cap;
  InferArgs a{c, feat, nrows * nz, nx, ny, nz, y64, out, rows};
  k_infer<<<(unsigned)blocks, 256, 0, s>>>(a);
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
  k_adam<<<(kMlpNParam + kAdamPerBlock - 1) / kAdamPerBlock + 1, 256, 0, s>>>(c, adam);
  return hipGetLastError();
}

}  // namespace eles
