// lbm_fstar_site.hpp -- the per-site f*_M Newton solve and its statistics,
// shared by the solver kernel (moments from a buffer) and the time step's
// lattice variant (moments from the pulled populations).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_fstar.hpp"
#include "lbm_fstar_dev.hpp"

namespace lbm {

// the solution as multipliers mu = ln(A, X, Y, Z) or as the state itself
__device__ __forceinline__ void write_mu(const FstarArgs& a, int64_t i, double rho, const FS<double>& s) {
  const int64_t n = a.n;
  if (a.prod) {
    a.mu[i] = s.a * rho;
    a.mu[n + i] = s.X;
    a.mu[2 * n + i] = s.Y;
    a.mu[3 * n + i] = s.Z;
  } else {
    a.mu[i] = ::log(s.a * rho);
    a.mu[n + i] = ::log(s.X);
    a.mu[2 * n + i] = ::log(s.Y);
    a.mu[3 * n + i] = ::log(s.Z);
  }
}

// FP64 damped Newton from the rest start; returns iterations (negative on failure)
__device__ inline int newton64_damped(double u1, double u2, double e, double tol, int max_it, FS<double>& s,
                               double& res) {
  s.a = 4.0 / 9.0;
  s.X = 1.0;
  s.Y = 1.0;
  s.Z = 0.25;
  double g[4], H[10], d[4];
  for (int it = 0; it <= max_it; ++it) {
    fsys<double>(s, u1, u2, e, g, H);
    res = resid(g);
    if (res <= tol) return it;
    if (it == max_it) break;
    fsolve<double>(H, g, d);
    double t = 1.0;
    if (res > 1e-3) {
      // Armijo on phi/rho = a n_x n_y - (ln a, ln X, ln Y, ln Z) . (1, u1, u2, e)
      const double phi0 = H[0] - (::log(s.a) + ::log(s.X) * u1 + ::log(s.Y) * u2 + ::log(s.Z) * e);
      const double slope = g[0] * d[0] + g[1] * d[1] + g[2] * d[2] + g[3] * d[3];
      for (int ls = 0; ls < 60; ++ls) {
        FS<double> q;
        q.a = s.a * ::exp(t * d[0]);
        q.X = s.X * ::exp(t * d[1]);
        q.Y = s.Y * ::exp(t * d[2]);
        q.Z = s.Z * ::exp(t * d[3]);
        double gq[4], Hq[10];
        fsys<double>(q, u1, u2, e, gq, Hq);
        const double phi = Hq[0] - (::log(q.a) + ::log(q.X) * u1 + ::log(q.Y) * u2 + ::log(q.Z) * e);
        if (phi <= phi0 + 1e-4 * t * slope) break;
        t *= 0.5;
      }
    }
    s.a *= ::exp(t * d[0]);
    s.X *= ::exp(t * d[1]);
    s.Y *= ::exp(t * d[2]);
    s.Z *= ::exp(t * d[3]);
  }
  return -1;
}

// The damped FP64 fallback of one site whose first pass missed the
// tolerance: Newton from the rest start, the solution (or its last iterate)
// written, status 1 (converged) or 3 (failed), counted in the statistics.
__device__ inline void fallback_site(const FstarArgs& a, int64_t i, double rho, double u1, double u2, double e) {
  FS<double> s;
  double res = 0.0;
  const int it = newton64_damped(u1, u2, e, a.tol, 200, s, res);
  if (it >= 0 && a.polish) res = polish_once(s, u1, u2, e);
  write_mu(a, i, rho, s);
  if (a.status) a.status[i] = it >= 0 ? 1 : 3;
  FstarStats& S = stat_slot(a.stats);
  atomicAdd(&S.fallback, 1ull);
  if (it < 0) atomicAdd(&S.failed, 1ull);
  else atomicMax(&S.maxres_bits, (unsigned long long)__double_as_longlong(res));
}

// Statistics are accumulated per thread over its sites, reduced per
// wavefront with shuffles and per block in LDS, and added to the global
// counters once per block (the grid is capped so that these atomics stay few).
struct SolveAcc {
  uint32_t hist[16];
  uint32_t sum32, sum64, infeasible, pad;
  unsigned long long maxres_bits;
};

constexpr int FSTAR_MAX_BLOCKS = 2048;

// One site of the solve: rho and u1, u2, e = 2E/rho of its moments; mu
// (or the state) written for a converged or infeasible site; `failed` set
// when the first pass missed the tolerance (the caller lists the site for the
// damped fallback).  it32 / it64: Newton updates of the two phases.  With
// st non-null the written state is also returned there in product form
// (A rho, X, Y, Z; NaN for a site with no quasiequilibrium).
template <int START>
__device__ __forceinline__ void solve_site(const FstarArgs& a, int64_t i, double rho, double u1, double u2, double e,
                                           int& it32, int& it64, uint32_t& ninf, double& maxres, bool& failed,
                                           double* st = nullptr) {
  const int64_t n = a.n;
  double res = 0.0;
  if (!feasible(rho, u1, u2, e)) {
    ninf++;
    if (__builtin_fabs(u1) < 1.0 && __builtin_fabs(u2) < 1.0 && rho > 0.0) {
      const FS<double> c = closed_form<double>(u1, u2);
      write_mu(a, i, rho, c);
      if (st) { st[0] = c.a * rho; st[1] = c.X; st[2] = c.Y; st[3] = c.Z; }
    } else {
      for (int c = 0; c < 4; ++c) a.mu[c * n + i] = __builtin_nan("");
      if (st) for (int c = 0; c < 4; ++c) st[c] = __builtin_nan("");
    }
    if (a.status) a.status[i] = 2;
  } else if constexpr (START == START_PLAIN) {
    // plain FP64 Newton with Armijo damping from the rest start: the
    // fallback of the method run on every site (the reference solve that
    // the other starts are measured against)
    FS<double> t;
    const int it = newton64_damped(u1, u2, e, a.tol, 200, t, res);
    if (it >= 0) {
      it64 = it;
      write_mu(a, i, rho, t);
      if (st) { st[0] = t.a * rho; st[1] = t.X; st[2] = t.Y; st[3] = t.Z; }
      if (a.status) a.status[i] = 0;
      maxres = fmax(maxres, res);
    } else {
      it64 = 200;
      failed = true;
    }
  } else {
    // ---- FP32 phase
    FS<float> s;
    if (START == START_CLOSED) {
      s = closed_form<float>((float)u1, (float)u2);
    } else if (START == START_WARM) {
      s.a = __expf(a.warm[i]);
      s.X = __expf(a.warm[n + i]);
      s.Y = __expf(a.warm[2 * n + i]);
      s.Z = __expf(a.warm[3 * n + i]);
    } else if (START == START_PREV) {
      // the solution already in mu (e.g. the previous time step's)
      if (a.prod) {
        s.a = (float)(a.mu[i] / rho);
        s.X = (float)a.mu[n + i];
        s.Y = (float)a.mu[2 * n + i];
        s.Z = (float)a.mu[3 * n + i];
      } else {
        s.a = __expf((float)a.mu[i]) / (float)rho;
        s.X = __expf((float)a.mu[n + i]);
        s.Y = __expf((float)a.mu[2 * n + i]);
        s.Z = __expf((float)a.mu[3 * n + i]);
      }
    } else {
      s.a = 4.0f / 9.0f;
      s.X = 1.0f;
      s.Y = 1.0f;
      s.Z = 0.25f;
    }
    // Far from the solution (residual > 1e-3) a Newton step that does not
    // lower the residual is halved, from the point it started from, up to
    // three times; near it the phase ends once an update gains less than a
    // factor 4 (FP32 round-off).  Every step is capped at 1 in each
    // multiplier.
    const float fu1 = (float)u1, fu2 = (float)u2, fe = (float)e;
    float g[4], H[10], d[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float prev = 3.0e38f, len = 1.0f;
    FS<float> base = s;
    for (;;) {
      fsys<float>(s, fu1, fu2, fe, g, H);
      const float r = resid(g);
      if (!(r > a.tol32) || it32 >= a.max32) break;
      if (!(r < prev) && prev > 1e-3f) {
        if (len < 0.2f) {  // three halvings failed: keep the better point
          s = base;
          break;
        }
        len *= 0.5f;
        s = base;
      } else {
        if (!(r < 0.25f * prev) && !(prev > 1e-3f)) break;
        prev = r;
        len = 1.0f;
        base = s;
        fsolve<float>(H, g, d);
      }
      const float dm = fmaxf(fmaxf(fabsf(d[0]), fabsf(d[1])), fmaxf(fabsf(d[2]), fabsf(d[3])));
      const float sc = (dm > 1.0f ? 1.0f / dm : 1.0f) * len;
      s.a = base.a * __expf(sc * d[0]);
      s.X = base.X * __expf(sc * d[1]);
      s.Y = base.Y * __expf(sc * d[2]);
      s.Z = base.Z * __expf(sc * d[3]);
      ++it32;
    }
    // ---- FP64 phase.  The first step is a simplified Newton step with
    // the FP32 Hessian H of the current point (its relative error ~1e-7
    // times a residual ~1e-6 leaves ~1e-13); full FP64 Newton steps
    // follow only if the residual is still above tol.
    FS<double> t{(double)s.a, (double)s.X, (double)s.Y, (double)s.Z};
    bool ok = false;
    if (__builtin_isfinite(t.a) && t.a > 0.0 && t.X > 0.0 && t.Y > 0.0 && t.Z > 0.0 &&
        __builtin_isfinite(t.X) && __builtin_isfinite(t.Y) && __builtin_isfinite(t.Z)) {
      double gd[4], Hd[10], dd[4];
      fsys_grad<double>(t, u1, u2, e, gd);
      res = resid(gd);
      if (res <= a.tol) {
        ok = true;
      } else if (res < 1e-4 && it64 < a.max64) {
        float gf[4] = {(float)gd[0], (float)gd[1], (float)gd[2], (float)gd[3]}, df[4];
        fsolve<float>(H, gf, df);
        t.a *= exp_step((double)df[0]);
        t.X *= exp_step((double)df[1]);
        t.Y *= exp_step((double)df[2]);
        t.Z *= exp_step((double)df[3]);
        ++it64;
        fsys_grad<double>(t, u1, u2, e, gd);
        res = resid(gd);
        ok = res <= a.tol;
      }
      for (; !ok;) {
        fsys<double>(t, u1, u2, e, gd, Hd);
        res = resid(gd);
        if (res <= a.tol) { ok = true; break; }
        if (it64 >= a.max64 || !(res < 1e-2)) break;
        fsolve<double>(Hd, gd, dd);
        t.a *= exp_step(dd[0]);
        t.X *= exp_step(dd[1]);
        t.Y *= exp_step(dd[2]);
        t.Z *= exp_step(dd[3]);
        ++it64;
      }
    }
    if (ok) {
      if (a.polish) {
        res = polish_once(t, u1, u2, e);
        ++it64;
      }
      write_mu(a, i, rho, t);
      if (st) { st[0] = t.a * rho; st[1] = t.X; st[2] = t.Y; st[3] = t.Z; }
      if (a.status) a.status[i] = 0;
      maxres = fmax(maxres, res);
    } else {
      failed = true;
    }
  }
}

// histogram of the updates per site: one pass per distinct value in the
// wavefront (every lane of the wavefront must call it)
__device__ __forceinline__ void solve_hist(SolveAcc& sh, bool live, int updates) {
  const int lane = threadIdx.x & 63;
  const int tot = updates < 15 ? updates : 15;
  unsigned long long rem = __ballot(live);
  while (rem) {
    const int src = __ffsll((long long)rem) - 1;
    const int b = __shfl(tot, src);
    const unsigned long long m = __ballot(live && tot == b);
    if (lane == 0) atomicAdd(&sh.hist[b], (uint32_t)__popcll(m));
    rem &= ~m;
  }
}

// wavefront reductions of the per-thread statistics, one LDS atomic per
// wavefront, then one global atomic per counter and workgroup (into the
// workgroup's copy of the statistics)
__device__ __forceinline__ void solve_flush(const FstarArgs& a, SolveAcc& sh, uint32_t sum32, uint32_t sum64,
                                            uint32_t ninf, double maxres) {
  const int lane = threadIdx.x & 63;
  #pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sum32 += __shfl_xor(sum32, off);
    sum64 += __shfl_xor(sum64, off);
    ninf += __shfl_xor(ninf, off);
    maxres = fmax(maxres, __shfl_xor(maxres, off));
  }
  if (lane == 0) {
    atomicAdd(&sh.sum32, sum32);
    atomicAdd(&sh.sum64, sum64);
    atomicAdd(&sh.infeasible, ninf);
    atomicMax(&sh.maxres_bits, (unsigned long long)__double_as_longlong(maxres));
  }
  __syncthreads();
  FstarStats& S = stat_slot(a.stats);
  if (threadIdx.x < 16 && sh.hist[threadIdx.x]) atomicAdd(&S.hist[threadIdx.x], (unsigned long long)sh.hist[threadIdx.x]);
  if (threadIdx.x == 16) {
    atomicAdd(&S.sum32, (unsigned long long)sh.sum32);
    atomicAdd(&S.sum64, (unsigned long long)sh.sum64);
    atomicAdd(&S.infeasible, (unsigned long long)sh.infeasible);
    atomicMax(&S.maxres_bits, sh.maxres_bits);
  }
}

}  // namespace lbm
