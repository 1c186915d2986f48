// lbm_fstar.hpp -- launch interface of the f*_M solver and the MLP kernels
// (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum : int { START_REST = 0, START_CLOSED = 1, START_WARM = 2, START_PREV = 3, START_PLAIN = 4 };

struct FstarStats {
  unsigned long long hist[16];   // Newton updates per site (FP32 + FP64 phases)
  unsigned long long sum32, sum64, infeasible, fallback, failed;
  unsigned long long maxres_bits; // bits of the largest final residual (non-negative double)
};

// The device keeps FSTAR_STAT_SLOTS copies of the statistics; a workgroup
// adds into copy blockIdx mod FSTAR_STAT_SLOTS, so that the per-workgroup
// atomics of a solve are spread over that many addresses instead of
// serialising on one (measured: with one copy, each extra workgroup of the
// time step's solve cost about 44 ns).  Readers sum the copies.
constexpr int FSTAR_STAT_SLOTS = 16;

__device__ __forceinline__ FstarStats& stat_slot(FstarStats* s) {
  return s[blockIdx.x & (FSTAR_STAT_SLOTS - 1)];
}

// sum (max for the residual) of the copies, on the host
inline FstarStats fstar_stats_total(const FstarStats* slots) {
  FstarStats t = slots[0];
  for (int k = 1; k < FSTAR_STAT_SLOTS; ++k) {
    const FstarStats& s = slots[k];
    for (int i = 0; i < 16; ++i) t.hist[i] += s.hist[i];
    t.sum32 += s.sum32;
    t.sum64 += s.sum64;
    t.infeasible += s.infeasible;
    t.fallback += s.fallback;
    t.failed += s.failed;
    if (s.maxres_bits > t.maxres_bits) t.maxres_bits = s.maxres_bits;
  }
  return t;
}

struct FstarArgs {
  const double* M;      // [4][n]
  int64_t n;
  double* mu;           // [4][n] (START_PREV: read as the start, then overwritten)
  int prod;             // 0: mu holds the multipliers (ln A, ln X, ln Y, ln Z);
                        // 1: the product-form state (A, X, Y, Z) itself
  const float* warm;    // [4][n]: (mu0 - ln rho, mu1, mu2, mu3) start, START_WARM only
  uint8_t* iters;       // [n] or null
  uint8_t* status;      // [n] or null: 0 ok, 1 fallback ok, 2 infeasible, 3 failed
  uint32_t* ctr;        // [4]: ctr[0] = number of failures of the first pass
  uint32_t* fail_list;  // [n]
  FstarStats* stats;    // [FSTAR_STAT_SLOTS]
  double tol;           // FP64 residual target
  float tol32;          // FP32 phase target
  int max32, max64;     // iteration budgets of the two phases
  int polish;           // 1: one more FP64 Newton update after convergence
                        // (to round-off; FP64 time-step contexts)
};

hipError_t launch_fstar(const FstarArgs& a, int start, hipStream_t s);
// the statistics clear and the damped fallback over the listed failures
// (the time step's lattice variant launches its own solve between them)
hipError_t launch_fstar_clear(const FstarArgs& a, hipStream_t s);
hipError_t launch_fstar_fallback(const FstarArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// MLP 4 -> 64 -> 64 -> 4 (SiLU), BF16 MFMA with FP32 accumulation
// ---------------------------------------------------------------------------
constexpr int MLP_NPARAM = 4740;
constexpr int MLP_OW1 = 0, MLP_OB1 = 256, MLP_OW2 = 320, MLP_OB2 = 4416, MLP_OW3 = 4480, MLP_OB3 = 4736;

struct MlpNorm {
  float in_shift[4], in_scale[4];    // x_k = (feature_k - shift) * scale
  float out_shift[4], out_scale[4];  // target_k = y_k / scale + shift
};

// forward of n samples X[n][4] (normalised features) -> Y[n][4]
hipError_t launch_mlp_forward(const float* params, const float* X, int64_t n, float* Y, hipStream_t s);
// warm start for the f*_M solver: features of M, forward, de-normalised
// (mu0 - ln rho, mu1, mu2, mu3) into warm[4][n]
hipError_t launch_mlp_warm(const float* params, const MlpNorm& nm, const double* M, int64_t n, float* warm,
                           hipStream_t s);
// training pairs (normalised inputs X, and targets T when mu is given)
hipError_t launch_mlp_pairs(const MlpNorm& nm, const double* M, const double* mu, int64_t n, float* X, float* T,
                            hipStream_t s);
// sample order of a training epoch: position offset + s reads sample
// perm(offset + s) of the n_total samples (on == 0: identity)
struct MlpPerm {
  int on;
  int h;            // half width in bits of the Feistel domain (2h >= log2 n_total)
  uint32_t n;       // n_total
  uint32_t offset;  // first position of this batch
  uint64_t key;     // epoch key
};
constexpr int MLP_GRAD_MAX_BLOCKS = 1024;
// per-block gradient partials of the MSE loss over n samples; returns the
// number of blocks used (partials is [nblocks][MLP_NPARAM + 1], the last
// column the block's loss sum)
int mlp_grad_blocks(int64_t n);
hipError_t launch_mlp_grad(const float* params, const float* X, const float* T, int64_t n, const MlpPerm& perm,
                           float* partials, hipStream_t s);
// reduce partials (fixed order), Adam update of params (FP32 master), m, v
hipError_t launch_mlp_reduce(const float* partials, int nblocks, int64_t n, float* grad, float* loss,
                             hipStream_t s);
hipError_t launch_adam(float* params, float* m, float* v, const float* grad, int64_t t, float lr, float b1,
                       float b2, float eps, hipStream_t s);
// the reduction followed at once by the Adam step (one launch per training step)
hipError_t launch_mlp_reduce_adam(const float* partials, int nblocks, int64_t n, float* grad, float* loss,
                                  float* params, float* m, float* v, int64_t t, float lr, float b1, float b2,
                                  float eps, hipStream_t s);

}  // namespace lbm
