// lbm_fstar.hip -- entropic quasiequilibrium f*_M with the energy row
// (Sec. 2: f*_M = argmax{S(f) : m(f) = M}, M = (rho, rho u1, rho u2, 2E);
// Sec. 3.3: ln f*_i is linear in the moment rows with Lagrange multipliers).
//
// Per site, Newton's method on the convex dual phi(mu) = sum_i exp(mu.m_i) -
// mu.M in the multiplicative variables (A, X, Y, Z) = exp(mu).  On D2Q9,
// |v|^2 = vx^2 + vy^2, so f*_i = A g(vx) g(vy) with g(0) = 1,
// g(+-1) = Z X^{+-1} (Y for the y factor): every sum of the gradient and
// Hessian follows from n = 1 + Z(X + 1/X), p = Z(X - 1/X), q = Z(X + 1/X)
// per direction, with no per-population loop and no transcendental.
//
// Phases: FP32 Newton from the chosen start until the rho-relative residual
// is ~1e-6; FP64 Newton (exp of small steps by its Taylor polynomial) until
// max_j |m_j(f*) - M_j| / rho <= tol (1e-10); sites still above tol are
// compacted and re-solved by FP64 damped Newton (Armijo backtracking) from
// the isothermal rest start.  Infeasible M (2E/rho outside
// (|u1| + |u2|, 2)) get the mass-momentum closed form of Sec. 4.2.
#include <hip/hip_runtime.h>

#include "lbm_fstar.hpp"
#include "lbm_fstar_dev.hpp"
#include "lbm_fstar_site.hpp"

namespace lbm {

template <int START>
__global__ __launch_bounds__(256) void k_fstar(FstarArgs a) {
  __shared__ SolveAcc sh;
  if (threadIdx.x < sizeof(SolveAcc) / 4) ((uint32_t*)&sh)[threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = a.n;
  uint32_t sum32 = 0, sum64 = 0, ninf = 0;
  double maxres = 0.0;
  // the trip count is uniform across the block so that every lane takes part
  // in the wavefront-level histogram
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t base = blockIdx.x * 256ll; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool live = i < n;
    int it32 = 0, it64 = 0;
    if (live) {
      const double rho = a.M[i], ir = 1.0 / rho;
      const double u1 = a.M[n + i] * ir, u2 = a.M[2 * n + i] * ir, e = a.M[3 * n + i] * ir;
      bool failed = false;
      solve_site<START>(a, i, rho, u1, u2, e, it32, it64, ninf, maxres, failed);
      if (failed) {
        const uint32_t slot = atomicAdd(&a.ctr[0], 1u);
        a.fail_list[slot] = (uint32_t)i;
      }
      sum32 += (uint32_t)it32;
      sum64 += (uint32_t)it64;
      if (a.iters) a.iters[i] = (uint8_t)(it32 + it64 < 255 ? it32 + it64 : 255);
    }
    solve_hist(sh, live, it32 + it64);
  }
  solve_flush(a, sh, sum32, sum64, ninf, maxres);
}

// FP64 damped-Newton fallback over the compacted failures
__global__ __launch_bounds__(64) void k_fstar_fallback(FstarArgs a) {
  const uint32_t nf = a.ctr[0];
  const int64_t n = a.n;
  for (uint32_t t = blockIdx.x * 64u + threadIdx.x; t < nf; t += gridDim.x * 64u) {
    const int64_t i = a.fail_list[t];
    const double rho = a.M[i], u1 = a.M[n + i] / rho, u2 = a.M[2 * n + i] / rho, e = a.M[3 * n + i] / rho;
    fallback_site(a, i, rho, u1, u2, e);
  }
}

// zeroes the failure counter and every copy of the statistics (all of their
// fields are 64-bit words)
__global__ void k_fstar_clear(FstarArgs a) {
  const int t = threadIdx.x;
  if (t < 4) a.ctr[t] = 0;
  unsigned long long* w = (unsigned long long*)a.stats;
  constexpr int words = FSTAR_STAT_SLOTS * (int)(sizeof(FstarStats) / 8);
  for (int j = t; j < words; j += 64) w[j] = 0ull;
}

hipError_t launch_fstar_clear(const FstarArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_fstar_clear, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fstar_fallback(const FstarArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_fstar_fallback, dim3(64), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fstar(const FstarArgs& a, int start, hipStream_t s) {
  hipLaunchKernelGGL(k_fstar_clear, dim3(1), dim3(64), 0, s, a);
  int64_t nb64 = (a.n + 255) / 256;
  const unsigned nb = (unsigned)(nb64 < FSTAR_MAX_BLOCKS ? nb64 : FSTAR_MAX_BLOCKS);
  if (nb > 0) {
    if (start == START_CLOSED) hipLaunchKernelGGL((k_fstar<START_CLOSED>), dim3(nb), dim3(256), 0, s, a);
    else if (start == START_WARM) hipLaunchKernelGGL((k_fstar<START_WARM>), dim3(nb), dim3(256), 0, s, a);
    else if (start == START_PREV) hipLaunchKernelGGL((k_fstar<START_PREV>), dim3(nb), dim3(256), 0, s, a);
    else if (start == START_PLAIN) hipLaunchKernelGGL((k_fstar<START_PLAIN>), dim3(nb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_fstar<START_REST>), dim3(nb), dim3(256), 0, s, a);
  }
  hipLaunchKernelGGL(k_fstar_fallback, dim3(64), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace lbm
