// lbm_mlp_dev.hpp -- device building blocks of the warm-start MLP
// 4 -> 64 -> 64 -> 4 (SiLU) on the gfx950 matrix cores, shared by the
// inference kernels (lbm_mlp_infer.hip) and the training kernels
// (lbm_mlp.hip).
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
#pragma once

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

__device__ inline void load_mats(const float* __restrict__ p, int r, int g, Mats& w) {
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

__device__ inline void load_weights(const float* __restrict__ p, int r, int g, Weights& w) {
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

}  // namespace lbm
