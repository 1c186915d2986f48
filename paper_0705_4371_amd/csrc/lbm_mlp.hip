// lbm_mlp.hip -- the learned warm start of the f*_M solve: an MLP
// 4 -> 64 -> 64 -> 4 with SiLU, BF16 operands on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; forward, backward
// (per-block gradient partials, fixed-order reduction) and Adam.
//
// Products are formed transposed, out^T = W . act^T, so that the weights are
// the A operand (held in registers for a whole kernel) and a tile of 16
// samples is the B operand.  With lane l, r = l % 16, g = l / 16:
//   A operand: lane holds A[r][8g .. 8g+7]      (16 x 32, row-major K)
//   B operand: lane holds B[8g .. 8g+7][r]      (32 x 16)
//   D result : lane holds D[4g .. 4g+3][r]      (16 x 16)
// Activations move between layers through per-wave LDS tiles.
//
// BF16 rounding points (the CPU oracle's emulation follows them): inputs,
// weights, hidden activations after SiLU, and back-propagated deltas where
// they enter a product; biases, bias gradients and SiLU are FP32 (a bias is
// the initial value of its product's FP32 accumulator).
#include <hip/hip_runtime.h>

#include "lbm_fstar.hpp"

namespace lbm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// SiLU z sigma(z) and its derivative sigma(z)(1 + z(1 - sigma(z))) in FP32;
// the hardware reciprocal (1 ulp) is ample: the activation is rounded to
// BF16 (8 bits) before its next use
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 v;
  #pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.0f;
  return v;
}

__device__ __forceinline__ bf16x8 load8(const float* p) {
  bf16x8 v;
  #pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (__bf16)p[j];
  return v;
}

// weight operands of the three layers for this lane
struct Mats {
  bf16x8 w1[4];     // layer 1, unit tile t: W1[16t + r][k], k < 4 real
  bf16x8 w2[4][2];  // layer 2, unit tile t, k step kk: W2[16t + r][32kk + 8g + j]
  bf16x8 w3[2];     // layer 3, k step kk: W3[r][32kk + 8g + j], r < 4 real
};
struct Weights : Mats {
  float b1[4][4], b2[4][4];  // bias of unit 16t + 4g + j
  float b3[4];               // bias of output j (lanes g == 0)
};

__device__ void load_mats(const float* __restrict__ p, int r, int g, Mats& w) {
  #pragma unroll
  for (int t = 0; t < 4; ++t) {
    bf16x8 v = zero8();
    if (g == 0) {
      #pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = (__bf16)p[MLP_OW1 + (16 * t + r) * 4 + j];
    }
    w.w1[t] = v;
    #pragma unroll
    for (int kk = 0; kk < 2; ++kk) w.w2[t][kk] = load8(p + MLP_OW2 + (16 * t + r) * 64 + 32 * kk + 8 * g);
  }
  #pragma unroll
  for (int kk = 0; kk < 2; ++kk) w.w3[kk] = r < 4 ? load8(p + MLP_OW3 + r * 64 + 32 * kk + 8 * g) : zero8();
}

__device__ void load_weights(const float* __restrict__ p, int r, int g, Weights& w) {
  load_mats(p, r, g, w);
  #pragma unroll
  for (int t = 0; t < 4; ++t) {
    #pragma unroll
    for (int j = 0; j < 4; ++j) {
      w.b1[t][j] = p[MLP_OB1 + 16 * t + 4 * g + j];
      w.b2[t][j] = p[MLP_OB2 + 16 * t + 4 * g + j];
    }
  }
  #pragma unroll
  for (int j = 0; j < 4; ++j) w.b3[j] = g == 0 ? p[MLP_OB3 + j] : 0.0f;
}

// bias access for forward16: the lane's registers (training) or a per-block
// LDS copy (inference, which keeps fewer registers live)
struct RegBias {
  const Weights& w;
  __device__ float b1(int t, int j) const { return w.b1[t][j]; }
  __device__ float b2(int t, int j) const { return w.b2[t][j]; }
  __device__ float b3(int j) const { return w.b3[j]; }
};
struct LdsBias {
  const float* p;  // the 4740 parameters' bias entries copied to LDS: b1 [64], b2 [64], b3 [4]
  int g;
  __device__ float b1(int t, int j) const { return p[16 * t + 4 * g + j]; }
  __device__ float b2(int t, int j) const { return p[64 + 16 * t + 4 * g + j]; }
  __device__ float b3(int j) const { return g == 0 ? p[128 + j] : 0.0f; }
};

// Epoch shuffle: position i of the epoch reads sample perm(i), perm a
// pseudo-random bijection of [0, n): a 4-round Feistel network on 2h bits
// (2h >= log2 n, round function SplitMix64 of (key, round, half)) with
// cycle-walking into [0, n).  Walking the cycle of a bijection returns to a
// value below n (at worst to i itself), so the loop terminates.
__device__ __forceinline__ uint64_t smix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ uint32_t feistel_perm(uint32_t i, const MlpPerm& p) {
  const uint32_t mask = (1u << p.h) - 1u;
  uint32_t x = i;
  do {
    uint32_t L = x >> p.h, R = x & mask;
    #pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t F = (uint32_t)smix64(p.key ^ ((uint64_t)r << 40) ^ R) & mask;
      const uint32_t t = R;
      R = L ^ F;
      L = t;
    }
    x = (L << p.h) | R;
  } while (x >= p.n);
  return x;
}

// LDS row strides (bf16 elements): site-major rows of 64 units, unit-major
// rows of 32 samples; padded against bank conflicts
constexpr int SROW = 72;
constexpr int TROW = 40;

// forward of one tile of 16 samples.  xin: B operand of layer 1 (lanes g == 0
// hold the 4 BF16 features of sample r).  Hs1/Hs2: this wave's site-major
// LDS tiles [16][SROW].  z1/z2 (optional) receive the pre-activations in the
// D layout; y receives the output (lanes g == 0, outputs 0..3 of sample r).
// sync: per-wave tiles need only the wave's own LDS order (SYNC_WAVE), the
// training kernel's single-wave blocks use a block barrier
enum { SYNC_BLOCK = 0, SYNC_WAVE = 1 };
template <int SYNC>
__device__ __forceinline__ void tile_sync() {
  if constexpr (SYNC == SYNC_WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <bool KEEP, int SYNC = SYNC_BLOCK, class Bias = RegBias>
__device__ __forceinline__ void forward16(const Mats& w, const Bias& bias, bf16x8 xin, __bf16* Hs1, __bf16* Hs2,
                                          int r, int g, f32x4* z1, f32x4* z2, f32x4& y) {
  // each product starts from its bias (the accumulator's initial value), so
  // no separate bias addition follows it
  #pragma unroll
  for (int t = 0; t < 4; ++t) {
    const f32x4 c = {bias.b1(t, 0), bias.b1(t, 1), bias.b1(t, 2), bias.b1(t, 3)};
    const f32x4 d = mfma(w.w1[t], xin, c);
    bf16x4 h;
    #pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = d[j];
      if (KEEP) z1[t][j] = z;
      h[j] = (__bf16)silu(z);
    }
    *(bf16x4*)(Hs1 + r * SROW + 16 * t + 4 * g) = h;
  }
  tile_sync<SYNC>();
  bf16x8 b2[2];
  #pragma unroll
  for (int kk = 0; kk < 2; ++kk) b2[kk] = *(const bf16x8*)(Hs1 + r * SROW + 32 * kk + 8 * g);
  #pragma unroll
  for (int t = 0; t < 4; ++t) {
    const f32x4 c = {bias.b2(t, 0), bias.b2(t, 1), bias.b2(t, 2), bias.b2(t, 3)};
    f32x4 d = mfma(w.w2[t][0], b2[0], c);
    d = mfma(w.w2[t][1], b2[1], d);
    bf16x4 h;
    #pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = d[j];
      if (KEEP) z2[t][j] = z;
      h[j] = (__bf16)silu(z);
    }
    *(bf16x4*)(Hs2 + r * SROW + 16 * t + 4 * g) = h;
  }
  tile_sync<SYNC>();
  bf16x8 b3[2];
  #pragma unroll
  for (int kk = 0; kk < 2; ++kk) b3[kk] = *(const bf16x8*)(Hs2 + r * SROW + 32 * kk + 8 * g);
  const f32x4 c = {bias.b3(0), bias.b3(1), bias.b3(2), bias.b3(3)};
  f32x4 d = mfma(w.w3[0], b3[0], c);
  d = mfma(w.w3[1], b3[1], d);
  y = d;
}

// ---------------------------------------------------------------------------
// inference
// ---------------------------------------------------------------------------
// Each wave takes tiles of 16 samples on its own (its LDS tiles are private,
// so only the wave's own LDS order matters); the biases sit in LDS, shared by
// the block, which keeps fewer registers live per lane.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ X,
                                                     int64_t n, float* __restrict__ out) {
  __shared__ __bf16 lds[4][2][16 * SROW];
  __shared__ float sbias[132];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
  if (threadIdx.x < 132)
    sbias[threadIdx.x] = threadIdx.x < 64    ? params[MLP_OB1 + threadIdx.x]
                         : threadIdx.x < 128 ? params[MLP_OB2 + threadIdx.x - 64]
                                             : params[MLP_OB3 + threadIdx.x - 128];
  Mats w;
  load_mats(params, r, g, w);
  __syncthreads();
  const LdsBias bias{sbias, g};
  const int64_t ntiles = (n + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t tile = blockIdx.x * 4ll + wv; tile < ntiles; tile += stride) {
    const int64_t s = tile * 16 + r;
    const bool live = s < n;
    bf16x8 xin = zero8();
    if (g == 0 && live) {
      #pragma unroll
      for (int k = 0; k < 4; ++k) xin[k] = (__bf16)X[s * 4 + k];
    }
    f32x4 y;
    forward16<false, SYNC_WAVE>(w, bias, xin, lds[wv][0], lds[wv][1], r, g, nullptr, nullptr, y);
    if (g == 0 && live) *(f32x4*)(out + s * 4) = y;
    tile_sync<SYNC_WAVE>();  // the wave's LDS tiles are rewritten by its next tile
  }
}

// The network's normalised input features of moments (rho, j1, j2, 2E):
// (u1, u2, 2E/rho, |u|^2) with u = j / rho, each mapped by (v - shift) * scale
// and rounded to FP32.  FP64, one reciprocal of rho per site; the training
// pairs and the solver's network start share this function.
__device__ __forceinline__ float4 mlp_features(const double* __restrict__ M, int64_t n, int64_t s,
                                               const MlpNorm& nm) {
  const double ir = 1.0 / M[s];
  const double u1 = M[n + s] * ir, u2 = M[2 * n + s] * ir, e = M[3 * n + s] * ir;
  const double uu = u1 * u1 + u2 * u2;
  float4 x;
  x.x = (float)((u1 - nm.in_shift[0]) * nm.in_scale[0]);
  x.y = (float)((u2 - nm.in_shift[1]) * nm.in_scale[1]);
  x.z = (float)((e - nm.in_shift[2]) * nm.in_scale[2]);
  x.w = (float)((uu - nm.in_shift[3]) * nm.in_scale[3]);
  return x;
}

// The solver's network start: warm[4][n] = (mu0 - ln rho, mu1, mu2, mu3) =
// y / out_scale + out_shift for the network output y of M's features.  A wave
// takes 64 sites per pass: every lane builds the features of one site (into
// the wave's LDS as BF16 rows), the four 16-site tiles go through the matrix
// cores, and every lane writes the four outputs of its site (coalesced per
// output row).
__global__ __launch_bounds__(256) void k_mlp_warm(const float* __restrict__ params, const double* __restrict__ M,
                                                  MlpNorm nm, int64_t n, float* __restrict__ warm) {
  __shared__ __bf16 lds[4][2][16 * SROW];
  __shared__ float sbias[132];
  __shared__ __bf16 sx[4][64 * 4];  // per wave: BF16 features of its 64 sites
  __shared__ float sy[4][64][5];     // per wave: outputs of its 64 sites (padded rows)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
  if (threadIdx.x < 132)
    sbias[threadIdx.x] = threadIdx.x < 64    ? params[MLP_OB1 + threadIdx.x]
                         : threadIdx.x < 128 ? params[MLP_OB2 + threadIdx.x - 64]
                                             : params[MLP_OB3 + threadIdx.x - 128];
  Mats w;
  load_mats(params, r, g, w);
  __syncthreads();
  const LdsBias bias{sbias, g};
  float oinv[4];
  #pragma unroll
  for (int k = 0; k < 4; ++k) oinv[k] = 1.0f / nm.out_scale[k];
  __bf16* xs = sx[wv];
  const int64_t ngroups = (n + 63) / 64;
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t grp = blockIdx.x * 4ll + wv; grp < ngroups; grp += stride) {
    const int64_t s = grp * 64 + lane;
    const bool live = s < n;
    float4 x = {0.f, 0.f, 0.f, 0.f};
    if (live) x = mlp_features(M, n, s, nm);
    bf16x4 xb;
    xb[0] = (__bf16)x.x;
    xb[1] = (__bf16)x.y;
    xb[2] = (__bf16)x.z;
    xb[3] = (__bf16)x.w;
    *(bf16x4*)(xs + lane * 4) = xb;
    tile_sync<SYNC_WAVE>();
    #pragma unroll
    for (int h = 0; h < 4; ++h) {
      bf16x8 xin = zero8();
      if (g == 0) {
        const bf16x4 v = *(const bf16x4*)(xs + (16 * h + r) * 4);
        #pragma unroll
        for (int k = 0; k < 4; ++k) xin[k] = v[k];
      }
      f32x4 y;
      forward16<false, SYNC_WAVE>(w, bias, xin, lds[wv][0], lds[wv][1], r, g, nullptr, nullptr, y);
      if (g == 0) {
        #pragma unroll
        for (int k = 0; k < 4; ++k) sy[wv][16 * h + r][k] = y[k];
      }
      tile_sync<SYNC_WAVE>();  // the wave's LDS tiles are rewritten by its next tile
    }
    if (live) {
      #pragma unroll
      for (int k = 0; k < 4; ++k) warm[k * n + s] = sy[wv][lane][k] * oinv[k] + nm.out_shift[k];
    }
    tile_sync<SYNC_WAVE>();  // sy and the feature rows are rewritten by the next pass
  }
}

// training pairs from moments M and multipliers mu ([4][n] each): the
// network's normalised inputs X [n][4] (the features of the solver's network start,
// the same arithmetic) and, when mu is given, its normalised targets T
// [n][4] = ((mu0 - ln rho, mu1, mu2, mu3) - out_shift) * out_scale
__global__ __launch_bounds__(256) void k_mlp_pairs(const double* __restrict__ M, const double* __restrict__ mu,
                                                   MlpNorm nm, int64_t n, float* __restrict__ X,
                                                   float* __restrict__ T) {
  for (int64_t s = blockIdx.x * 256ll + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256) {
    *(float4*)(X + 4 * s) = mlp_features(M, n, s, nm);
    if (T) {
      const double tg[4] = {mu[s] - ::log(M[s]), mu[n + s], mu[2 * n + s], mu[3 * n + s]};
      float4 t;
      t.x = (float)((tg[0] - nm.out_shift[0]) * nm.out_scale[0]);
      t.y = (float)((tg[1] - nm.out_shift[1]) * nm.out_scale[1]);
      t.z = (float)((tg[2] - nm.out_shift[2]) * nm.out_scale[2]);
      t.w = (float)((tg[3] - nm.out_shift[3]) * nm.out_scale[3]);
      *(float4*)(T + 4 * s) = t;
    }
  }
}

hipError_t launch_mlp_pairs(const MlpNorm& nm, const double* M, const double* mu, int64_t n, float* X, float* T,
                            hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb > 0) hipLaunchKernelGGL(k_mlp_pairs, dim3((unsigned)nb), dim3(256), 0, s, M, mu, nm, n, X, mu ? T : nullptr);
  return hipGetLastError();
}

static unsigned fwd_grid(int64_t n) {
  const int64_t tiles = (n + 15) / 16;
  int64_t nb = (tiles + 3) / 4;
  return (unsigned)(nb < 2048 ? (nb > 0 ? nb : 1) : 2048);
}

hipError_t launch_mlp_forward(const float* params, const float* X, int64_t n, float* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(fwd_grid(n)), dim3(256), 0, s, params, X, n, Y);
  return hipGetLastError();
}

hipError_t launch_mlp_warm(const float* params, const MlpNorm& nm, const double* M, int64_t n, float* warm,
                           hipStream_t s) {
  const int64_t groups = (n + 63) / 64;
  int64_t nb = (groups + 3) / 4;
  nb = nb < 2048 ? (nb > 0 ? nb : 1) : 2048;
  hipLaunchKernelGGL(k_mlp_warm, dim3((unsigned)nb), dim3(256), 0, s, params, M, nm, n, warm);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gradient of the MSE loss L = (1/(4 n)) sum_s sum_o (y_so - t_so)^2
// ---------------------------------------------------------------------------
// Blocks of 2 waves; a wave takes chunks of 32 samples (two tiles of 16),
// the K dimension of the weight-gradient products.  Per-wave LDS:
struct GradLds {
  __bf16 hs1[2][16 * SROW];  // site-major H1 of the two tiles (forward operand)
  __bf16 hs2[2][16 * SROW];  // site-major H2; reused for site-major dZ2
  __bf16 h1t[64 * TROW];     // unit-major H1 [unit][sample]
  __bf16 h2t[64 * TROW];     // unit-major H2
  __bf16 dz2t[64 * TROW];    // unit-major dZ2
  __bf16 dz1t[64 * TROW];    // unit-major dZ1
  __bf16 xt[16 * TROW];      // feature-major X [k][sample], k < 4 real
  __bf16 gyt[16 * TROW];     // output-major dY [o][sample], o < 4 real
  __bf16 gys[32 * 8];        // sample-major dY [sample][o], o < 4 real
};

constexpr int GRAD_WAVES = 1;

__global__ __launch_bounds__(64 * GRAD_WAVES) void k_mlp_grad(const float* __restrict__ params,
                                                              const float* __restrict__ X,
                                                              const float* __restrict__ T, int64_t n,
                                                              MlpPerm perm, float* __restrict__ partials) {
  // the per-wave tiles and the final reduction buffer share the LDS
  constexpr size_t TILE_BYTES = sizeof(GradLds) * GRAD_WAVES;
  constexpr size_t RED_BYTES = sizeof(float) * GRAD_WAVES * (MLP_NPARAM + 1);
  __shared__ __attribute__((aligned(16))) char lds_raw[TILE_BYTES > RED_BYTES ? TILE_BYTES : RED_BYTES];
  GradLds* L = (GradLds*)lds_raw;
  float(*red)[MLP_NPARAM + 1] = (float(*)[MLP_NPARAM + 1])lds_raw;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
  GradLds& S = L[wv];
  Weights w;
  load_weights(params, r, g, w);
  // transposed weight operands for the backward products
  bf16x8 w3t[4];     // A of dH2 = W3^T dY: W3^T[16t + r][o = 8g + j] (o < 4 real)
  bf16x8 w2t[4][2];  // A of dH1 = W2^T dZ2: W2^T[16t + r][32kk + 8g + j] = W2[32kk+8g+j][16t+r]
  #pragma unroll
  for (int t = 0; t < 4; ++t) {
    bf16x8 v = zero8();
    if (g == 0) {
      #pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = (__bf16)params[MLP_OW3 + j * 64 + 16 * t + r];
    }
    w3t[t] = v;
    #pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      bf16x8 u;
      #pragma unroll
      for (int j = 0; j < 8; ++j) u[j] = (__bf16)params[MLP_OW2 + (32 * kk + 8 * g + j) * 64 + 16 * t + r];
      w2t[t][kk] = u;
    }
  }
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 gw1[4], gw2[4][4], gw3[4];  // weight-gradient tiles (D layout)
  float gb1[4][4], gb2[4][4], gb3[4], lsum = 0.f;
  #pragma unroll
  for (int t = 0; t < 4; ++t) {
    gw1[t] = zero;
    gw3[t] = zero;
    #pragma unroll
    for (int u = 0; u < 4; ++u) gw2[t][u] = zero;
    #pragma unroll
    for (int j = 0; j < 4; ++j) { gb1[t][j] = 0.f; gb2[t][j] = 0.f; }
    gb3[t] = 0.f;
  }
  const float gscale = 2.0f / (4.0f * (float)n);

  const int64_t nchunks = (n + 31) / 32;
  for (int64_t base = (int64_t)blockIdx.x * GRAD_WAVES; base < nchunks; base += (int64_t)gridDim.x * GRAD_WAVES) {
    const int64_t chunk = base + wv;
    f32x4 z1[2][4], z2[2][4], y[2];
    float tgt[2][4];
    bool live[2];
    // ---- forward of the two tiles
    #pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t s = chunk * 32 + h * 16 + r;
      live[h] = chunk < nchunks && s < n;
      bf16x8 xin = zero8();
      const int sl = h * 16 + r;  // sample within the chunk
      if (g == 0) {
        float f[4] = {0.f, 0.f, 0.f, 0.f};
        if (live[h]) {
          const int64_t src = perm.on ? (int64_t)feistel_perm((uint32_t)(perm.offset + s), perm) : s;
          #pragma unroll
          for (int k = 0; k < 4; ++k) { f[k] = X[src * 4 + k]; tgt[h][k] = T[src * 4 + k]; }
        }
        #pragma unroll
        for (int k = 0; k < 4; ++k) {
          xin[k] = (__bf16)f[k];
          S.xt[k * TROW + sl] = xin[k];
        }
      }
      forward16<true>(w, RegBias{w}, xin, S.hs1[h], S.hs2[h], r, g, z1[h], z2[h], y[h]);
    }
    // unit-major copies of H1 and H2 for the weight-gradient products
    #pragma unroll
    for (int h = 0; h < 2; ++h)
      #pragma unroll
      for (int t = 0; t < 4; ++t)
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = 16 * t + 4 * g + j;
          S.h1t[u * TROW + h * 16 + r] = S.hs1[h][r * SROW + u];
          S.h2t[u * TROW + h * 16 + r] = S.hs2[h][r * SROW + u];
        }
    // ---- output delta dY = 2 (y - t) / (4 n), FP32; BF16 copies for products
    #pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int sl = h * 16 + r;
      if (g == 0) {
        #pragma unroll
        for (int o = 0; o < 4; ++o) {
          float gy = 0.f;
          if (live[h]) {
            const float d = y[h][o] - tgt[h][o];
            lsum += d * d;
            gy = gscale * d;
          }
          gb3[o] += gy;
          const __bf16 gbf = (__bf16)gy;
          S.gyt[o * TROW + sl] = gbf;
          S.gys[sl * 8 + o] = gbf;
        }
        #pragma unroll
        for (int o = 4; o < 8; ++o) S.gys[sl * 8 + o] = (__bf16)0.0f;
      }
    }
    // zero rows 4..15 of the output-major dY and feature-major X (A/B padding)
    for (int e = lane; e < 12 * 32; e += 64) {
      S.gyt[(4 + e / 32) * TROW + (e & 31)] = (__bf16)0.0f;
      S.xt[(4 + e / 32) * TROW + (e & 31)] = (__bf16)0.0f;
    }
    __syncthreads();
    // ---- dW3 += dY^T-chunk . H2 : A = dY [o][32 samples], B = H2 [32 samples][16 units]
    {
      const bf16x8 a = *(const bf16x8*)(S.gyt + r * TROW + 8 * g);
      #pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bf16x8 b = *(const bf16x8*)(S.h2t + (16 * t + r) * TROW + 8 * g);
        gw3[t] = mfma(a, b, gw3[t]);
      }
    }
    // ---- dZ2 = (W3^T dY) * silu'(z2), per tile of 16 samples
    #pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf16x8 b = zero8();
      if (g == 0) b = *(const bf16x8*)(S.gys + (h * 16 + r) * 8);
      #pragma unroll
      for (int t = 0; t < 4; ++t) {
        const f32x4 dh = mfma(w3t[t], b, zero);
        bf16x4 q;
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float dz = live[h] ? dh[j] * dsilu(z2[h][t][j]) : 0.f;
          gb2[t][j] += dz;
          q[j] = (__bf16)dz;
          S.dz2t[(16 * t + 4 * g + j) * TROW + h * 16 + r] = q[j];
        }
        *(bf16x4*)(S.hs2[h] + r * SROW + 16 * t + 4 * g) = q;  // site-major dZ2
      }
    }
    __syncthreads();
    // ---- dW2 += dZ2 . H1 : A = dZ2 [16 units j][32 samples], B = H1 [32 samples][16 units k]
    #pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      const bf16x8 a = *(const bf16x8*)(S.dz2t + (16 * tj + r) * TROW + 8 * g);
      #pragma unroll
      for (int tk = 0; tk < 4; ++tk) {
        const bf16x8 b = *(const bf16x8*)(S.h1t + (16 * tk + r) * TROW + 8 * g);
        gw2[tj][tk] = mfma(a, b, gw2[tj][tk]);
      }
    }
    // ---- dZ1 = (W2^T dZ2) * silu'(z1)
    #pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf16x8 b[2];
      #pragma unroll
      for (int kk = 0; kk < 2; ++kk) b[kk] = *(const bf16x8*)(S.hs2[h] + r * SROW + 32 * kk + 8 * g);
      #pragma unroll
      for (int t = 0; t < 4; ++t) {
        f32x4 dh = mfma(w2t[t][0], b[0], zero);
        dh = mfma(w2t[t][1], b[1], dh);
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float dz = live[h] ? dh[j] * dsilu(z1[h][t][j]) : 0.f;
          gb1[t][j] += dz;
          S.dz1t[(16 * t + 4 * g + j) * TROW + h * 16 + r] = (__bf16)dz;
        }
      }
    }
    __syncthreads();
    // ---- dW1 += dZ1 . X : A = dZ1 [16 units][32 samples], B = X [32 samples][16 (4 real)]
    {
      const bf16x8 b = *(const bf16x8*)(S.xt + r * TROW + 8 * g);
      #pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bf16x8 a = *(const bf16x8*)(S.dz1t + (16 * t + r) * TROW + 8 * g);
        gw1[t] = mfma(a, b, gw1[t]);
      }
    }
    __syncthreads();  // LDS is rewritten by the next chunk
  }

  // ---- per-wave results -> block partial (fixed order over waves)
  __syncthreads();  // the tiles are dead; the LDS becomes the reduction buffer
  for (int p = threadIdx.x; p < GRAD_WAVES * (MLP_NPARAM + 1); p += blockDim.x) (&red[0][0])[p] = 0.f;
  __syncthreads();
  float* R = red[wv];
  // weight tiles: D layout, lane holds rows 4g + j, column r
  #pragma unroll
  for (int t = 0; t < 4; ++t)
    #pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 16 * t + 4 * g + j;  // hidden unit of layer 1
      if (r < 4) R[MLP_OW1 + row * 4 + r] = gw1[t][j];
      #pragma unroll
      for (int tk = 0; tk < 4; ++tk) R[MLP_OW2 + row * 64 + 16 * tk + r] = gw2[t][tk][j];
    }
  if (g == 0)
    #pragma unroll
    for (int t = 0; t < 4; ++t)
      #pragma unroll
      for (int j = 0; j < 4; ++j) R[MLP_OW3 + j * 64 + 16 * t + r] = gw3[t][j];
  __syncthreads();
  // biases: lanes with the same g share units; sum over r in a fixed order
  #pragma unroll
  for (int t = 0; t < 4; ++t)
    #pragma unroll
    for (int j = 0; j < 4; ++j) {
      float a1 = gb1[t][j], a2 = gb2[t][j];
      #pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
        a1 += __shfl_xor(a1, off, 16);
        a2 += __shfl_xor(a2, off, 16);
      }
      if (r == 0) {
        R[MLP_OB1 + 16 * t + 4 * g + j] = a1;
        R[MLP_OB2 + 16 * t + 4 * g + j] = a2;
      }
    }
  #pragma unroll
  for (int o = 0; o < 4; ++o) {
    float a3 = gb3[o];
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) a3 += __shfl_xor(a3, off);
    if (lane == 0) R[MLP_OB3 + o] = a3;
  }
  float ls = lsum;
  #pragma unroll
  for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off);
  if (lane == 0) R[MLP_NPARAM] = ls;
  __syncthreads();
  for (int p = threadIdx.x; p < MLP_NPARAM + 1; p += blockDim.x) {
    float v = 0.f;
    #pragma unroll
    for (int q = 0; q < GRAD_WAVES; ++q) v += red[q][p];
    partials[(int64_t)blockIdx.x * (MLP_NPARAM + 1) + p] = v;
  }
}

int mlp_grad_blocks(int64_t n) {
  const int64_t chunks = (n + 31) / 32;
  int64_t nb = (chunks + GRAD_WAVES - 1) / GRAD_WAVES;
  return (int)(nb < MLP_GRAD_MAX_BLOCKS ? (nb > 0 ? nb : 1) : MLP_GRAD_MAX_BLOCKS);
}

hipError_t launch_mlp_grad(const float* params, const float* X, const float* T, int64_t n, const MlpPerm& perm,
                           float* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(mlp_grad_blocks(n)), dim3(64 * GRAD_WAVES), 0, s, params, X, T, n, perm,
                     partials);
  return hipGetLastError();
}

// fixed-order sum of the block partials: grad[p] and loss = sum / (4 n).
// Adam (Kingma and Ba) with bias correction c1 = 1 - b1^t, c2 = 1 - b2^t
struct AdamArgs {
  int on;
  float* p;
  float* m;
  float* v;
  float c1, c2, lr, b1, b2, eps;
};

__device__ __forceinline__ void adam_update(const AdamArgs& a, int i, float gi) {
  const float mi = a.b1 * a.m[i] + (1.f - a.b1) * gi;
  const float vi = a.b2 * a.v[i] + (1.f - a.b2) * gi * gi;
  a.m[i] = mi;
  a.v[i] = vi;
  a.p[i] -= a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
}

static AdamArgs adam_args(float* params, float* m, float* v, int64_t t, float lr, float b1, float b2, float eps) {
  AdamArgs a;
  a.on = 1;
  a.p = params;
  a.m = m;
  a.v = v;
  a.c1 = (float)(1.0 - pow((double)b1, (double)t));
  a.c2 = (float)(1.0 - pow((double)b2, (double)t));
  a.lr = lr;
  a.b1 = b1;
  a.b2 = b2;
  a.eps = eps;
  return a;
}

// A block owns 64 parameters; its 16 thread groups sum the partials of
// blocks b = q (mod 16) in increasing b, then the 16 group sums are added in
// group order (a fixed order: the result does not depend on scheduling).
// With ad.on the block applies the Adam step to its 64 parameters at once.
__global__ __launch_bounds__(1024) void k_mlp_reduce(const float* __restrict__ partials, int nblocks, int64_t n,
                                                     float* __restrict__ grad, float* __restrict__ loss,
                                                     AdamArgs ad) {
  __shared__ float red[16][64];
  const int q = threadIdx.x >> 6, j = threadIdx.x & 63;
  const int p = blockIdx.x * 64 + j;
  float s = 0.f;
  if (p <= MLP_NPARAM)
    for (int b = q; b < nblocks; b += 16) s += partials[(int64_t)b * (MLP_NPARAM + 1) + p];
  red[q][j] = s;
  __syncthreads();
  if (q == 0 && p <= MLP_NPARAM) {
    float t = red[0][j];
    for (int v = 1; v < 16; ++v) t += red[v][j];
    if (p < MLP_NPARAM) {
      grad[p] = t;
      if (ad.on) adam_update(ad, p, t);
    } else if (loss) {
      *loss = t / (4.0f * (float)n);
    }
  }
}

hipError_t launch_mlp_reduce(const float* partials, int nblocks, int64_t n, float* grad, float* loss,
                             hipStream_t s) {
  AdamArgs off{};
  hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 1 + 63) / 64), dim3(1024), 0, s, partials, nblocks, n, grad,
                     loss, off);
  return hipGetLastError();
}

hipError_t launch_mlp_reduce_adam(const float* partials, int nblocks, int64_t n, float* grad, float* loss,
                                  float* params, float* m, float* v, int64_t t, float lr, float b1, float b2,
                                  float eps, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 1 + 63) / 64), dim3(1024), 0, s, partials, nblocks, n, grad,
                     loss, adam_args(params, m, v, t, lr, b1, b2, eps));
  return hipGetLastError();
}

// Adam step t >= 1 on all parameters (the separate entry point)
__global__ __launch_bounds__(256) void k_adam(const float* __restrict__ g, AdamArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  adam_update(a, i, g[i]);
}

hipError_t launch_adam(float* params, float* m, float* v, const float* grad, int64_t t, float lr, float b1,
                       float b2, float eps, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, grad,
                     adam_args(params, m, v, t, lr, b1, b2, eps));
  return hipGetLastError();
}

}  // namespace lbm
