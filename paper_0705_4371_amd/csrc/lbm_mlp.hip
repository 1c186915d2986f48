// lbm_mlp.hip -- training of the learned warm start of the f*_M solve (the
// MLP 4 -> 64 -> 64 -> 4 with SiLU of lbm_mlp_dev.hpp): forward and
// backward on BF16 operands of the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation, per-block gradient
// partials reduced in fixed order, and Adam.
#include <hip/hip_runtime.h>

#include "lbm_mlp_dev.hpp"

namespace lbm {

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
