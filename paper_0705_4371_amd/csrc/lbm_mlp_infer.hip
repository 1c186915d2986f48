// lbm_mlp_infer.hip -- inference of the warm-start MLP: the forward pass of
// normalised features and the f*_M solver's network start (features of the
// moments, forward, unnormalised start), and the training pairs.  Compiled
// with the matrix-core results in ordinary vector registers (no
// accumulation-register reads before the activations).
#include <hip/hip_runtime.h>

#include "lbm_mlp_dev.hpp"

namespace lbm {

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
  // four 64-site groups per workgroup pass; a grid of up to 4096 workgroups
  // (four rounds of the workgroups the device holds at once) measured
  // faster than one round or two
  const int64_t groups = (n + 63) / 64;
  int64_t nb = (groups + 3) / 4;
  nb = nb < 4096 ? (nb > 0 ? nb : 1) : 4096;
  hipLaunchKernelGGL(k_mlp_warm, dim3((unsigned)nb), dim3(256), 0, s, params, M, nm, n, warm);
  return hipGetLastError();
}

}  // namespace lbm
