// lbm_kernels.hip -- gfx950 kernels around the time step: initial state,
// population access, moments, FP64 conservation sums, clearing, the f*_M
// moments and initial state; and the dispatch of the step launches to the
// translation units that instantiate them (lbm_step_*.hip, lbm_fstep_*.hip).
#include <hip/hip_runtime.h>

#include "lbm_step.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// initial state, population access, moments, sums, clearing
// ---------------------------------------------------------------------------
template <typename T, int Q, int QE>
__global__ __launch_bounds__(256) void k_init(StepArgs a, const double* __restrict__ rho0,
                                              const double* __restrict__ u0) {
  T* __restrict__ S = (T*)a.B;
  const Geom& g = a.g;
  const int64_t N = g.nx * g.ny;
  for (int64_t s = blockIdx.x * 256ll + threadIdx.x; s < N; s += (int64_t)gridDim.x * 256) {
    int64_t x, y;
    divmod((int64_t)s, g.nx, g.inv_nx, y, x);
    double fs[Q];
    if (is_solid(g, x, y)) {
      #pragma unroll
      for (int i = 0; i < Q; ++i) fs[i] = 0.0;
    } else {
      const double rho = rho0[s], ux = u0[s], uy = Q == 9 ? u0[N + s] : 0.0;
      if (QE == QE_POLY) qe_poly<Q, double>(rho, ux, uy, fs);
      else qe_entropic_mm<Q, double>(rho, ux, uy, fs);
    }
    #pragma unroll
    for (int i = 0; i < Q; ++i) S[sidx<Q>(g, x, y, i)] = (T)fs[i];
  }
}

template <typename T, int Q, bool PULL>
__global__ __launch_bounds__(256) void k_get(StepArgs a, T* __restrict__ out) {
  const T* __restrict__ A = (const T*)a.A;
  const Geom& g = a.g;
  const int64_t N = g.nx * g.ny;
  for (int64_t s = blockIdx.x * 256ll + threadIdx.x; s < N; s += (int64_t)gridDim.x * 256) {
    int64_t x, y;
    divmod((int64_t)s, g.nx, g.inv_nx, y, x);
    T f[Q];
    if (is_solid(g, x, y)) {
      #pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = T(0);
    } else {
      load_site_fast<T, Q, PULL>(A, g, x, y, f);
    }
    #pragma unroll
    for (int i = 0; i < Q; ++i) out[(int64_t)i * N + s] = f[i];
  }
}

template <typename T, int Q>
__global__ __launch_bounds__(256) void k_set(StepArgs a, const T* __restrict__ in) {
  T* __restrict__ S = (T*)a.B;
  const Geom& g = a.g;
  const int64_t N = g.nx * g.ny;
  bool bad = false;
  for (int64_t s = blockIdx.x * 256ll + threadIdx.x; s < N; s += (int64_t)gridDim.x * 256) {
    int64_t x, y;
    divmod((int64_t)s, g.nx, g.inv_nx, y, x);
    #pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T v = in[(int64_t)i * N + s];
      bad |= !__builtin_isfinite(v);
      S[sidx<Q>(g, x, y, i)] = v;
    }
  }
  if (bad) atomicOr(&a.ctr[C_SETBAD], 1u);
}

template <typename T, int Q, bool PULL>
__global__ __launch_bounds__(256) void k_moments(StepArgs a, double* __restrict__ rho,
                                                 double* __restrict__ rhou, double* __restrict__ e2) {
  const T* __restrict__ A = (const T*)a.A;
  const Geom& g = a.g;
  const int64_t N = g.nx * g.ny;
  for (int64_t s = blockIdx.x * 256ll + threadIdx.x; s < N; s += (int64_t)gridDim.x * 256) {
    int64_t x, y;
    divmod((int64_t)s, g.nx, g.inv_nx, y, x);
    double fd[Q];
    if (is_solid(g, x, y)) {
      #pragma unroll
      for (int i = 0; i < Q; ++i) fd[i] = 0.0;
    } else {
      T f[Q];
      load_site_fast<T, Q, PULL>(A, g, x, y, f);
      #pragma unroll
      for (int i = 0; i < Q; ++i) fd[i] = (double)f[i];
    }
    const Moments<Q, double> m = moments<Q, double>(fd);
    if (rho) rho[s] = m.rho;
    if (rhou) { rhou[s] = m.jx; rhou[N + s] = m.jy; }
    if (e2) e2[s] = m.e2;
  }
}

// FP64 sums over fluid sites of rho, rho u1, rho u2, 2E of the current
// pre-collision state (the conservation diagnostics): per-thread sums in a
// fixed grid-stride order, per-block partials, then one block in fixed order

template <typename T, int Q, bool PULL>
__global__ __launch_bounds__(256) void k_sums(StepArgs a) {
  const T* __restrict__ A = (const T*)a.A;
  const Geom& g = a.g;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  // sites in layout order (a wavefront covers one 64-site tile)
  for (int64_t p = blockIdx.x * 256ll + threadIdx.x; p < g.plane; p += (int64_t)gridDim.x * 256) {
    int64_t x, y;
    divmod(p, g.pitch, g.inv_pitch, y, x);
    if (x >= g.nx || is_solid(g, x, y)) continue;
    T f[Q];
    load_site_fast<T, Q, PULL>(A, g, x, y, f);
    double fd[Q];
    #pragma unroll
    for (int q = 0; q < Q; ++q) fd[q] = (double)f[q];
    const Moments<Q, double> m = moments<Q, double>(fd);
    s[0] += m.rho;
    s[1] += m.jx;
    s[2] += m.jy;
    s[3] += m.e2;
  }
  __shared__ double red[4][256];
  for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) a.partials[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_finalize(StepArgs a, int nb) {
  __shared__ double red[4][256];
  const int tid = threadIdx.x;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = tid; b < nb; b += 256)
    for (int c = 0; c < 4; ++c) s[c] += a.partials[b * 4 + c];
  for (int c = 0; c < 4; ++c) red[c][tid] = s[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
      for (int c = 0; c < 4; ++c) red[c][tid] += red[c][tid + w];
    __syncthreads();
  }
  if (tid < 4) a.st->sums[tid] = red[tid][0];
}

__global__ __launch_bounds__(256) void k_clear(StepArgs a) {
  const int64_t t0 = blockIdx.x * 256ll + threadIdx.x, stride = (int64_t)gridDim.x * 256;
  for (int64_t j = t0; j < HIST_WORDS; j += stride) a.hist[j] = 0;
  for (int64_t j = t0; j < SUM_BLOCKS * 4; j += stride) a.partials[j] = 0.0;
  if (t0 < C_COUNT) a.ctr[t0] = 0;
  if (t0 == 0) {
    a.st->n_above = a.st->n_sel = a.st->n_invalid = a.st->total_sel = a.st->n_screened = 0;
    a.st->kth = a.st->max = 0.0;
    for (int c = 0; c < 4; ++c) a.st->sums[c] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// f*_M support: moments for the solver, initial state from the multipliers
// ---------------------------------------------------------------------------
template <typename T, bool PULL>
__global__ __launch_bounds__(STEP_TX) void k_moments_M(StepArgs a) {
  if (halted(a)) return;
  const T* __restrict__ A = (const T*)a.A;
  const Geom& g = a.g;
  const int64_t N = g.nx * g.ny;
  // the row segments of k_step (same interior fast path)
  const int64_t b = xcd_remap(blockIdx.x, a.nblocks);
  const int64_t y = b / a.ntx;
  const int64_t x0 = (b - y * a.ntx) * STEP_TX;
  const int64_t x = x0 + threadIdx.x;
  const bool fluid = x < g.nx && !is_solid(g, x, y);
  T f[9];
  load_segment_site<T, 9, PULL>(A, g, x0, x, y, fluid, f);
  if (x >= g.nx) return;
  double r = 1.0, jx = 0.0, jy = 0.0, e2 = 2.0 / 3.0;
  if (fluid) {
    double fd[9];
    #pragma unroll
    for (int i = 0; i < 9; ++i) fd[i] = (double)f[i];
    const Moments<9, double> m = moments<9, double>(fd);
    r = m.rho;
    jx = m.jx;
    jy = m.jy;
    e2 = m.e2;
  }
  const int64_t s = x + y * g.nx;
  a.Mbuf[s] = r;
  a.Mbuf[N + s] = jx;
  a.Mbuf[2 * N + s] = jy;
  a.Mbuf[3 * N + s] = e2;
}

// f*_M time step for the starts that need no network (rest, closed form,
// previous step): the pull of f(x, t) on the step kernel's row segments, its
// FP64 moments, the per-site Newton solve, the FP32 Delta S screen and the
// collision in one kernel (a grid-stride loop with a uniform trip count per
// block).  A site whose first pass failed is listed with its moments and is
// solved and collided by k_fstep_fallback.

__global__ __launch_bounds__(256) void k_init_M_moments(StepArgs a, const double* __restrict__ rho0,
                                                        const double* __restrict__ u0,
                                                        const double* __restrict__ twoE0) {
  const Geom& g = a.g;
  const int64_t N = g.nx * g.ny;
  for (int64_t s = blockIdx.x * 256ll + threadIdx.x; s < N; s += (int64_t)gridDim.x * 256) {
    int64_t x, y;
    divmod((int64_t)s, g.nx, g.inv_nx, y, x);
    const bool sol = is_solid(g, x, y);
    const double r = sol ? 1.0 : rho0[s];
    a.Mbuf[s] = r;
    a.Mbuf[N + s] = sol ? 0.0 : r * u0[s];
    a.Mbuf[2 * N + s] = sol ? 0.0 : r * u0[N + s];
    a.Mbuf[3 * N + s] = sol ? 2.0 / 3.0 : r * twoE0[s];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_init_M_pops(StepArgs a) {
  T* __restrict__ S = (T*)a.B;
  const Geom& g = a.g;
  const int64_t N = g.nx * g.ny;
  for (int64_t s = blockIdx.x * 256ll + threadIdx.x; s < N; s += (int64_t)gridDim.x * 256) {
    int64_t x, y;
    divmod((int64_t)s, g.nx, g.inv_nx, y, x);
    double fs[9];
    if (is_solid(g, x, y)) {
      #pragma unroll
      for (int i = 0; i < 9; ++i) fs[i] = 0.0;
    } else {
      fstar_from_state<double>(a.mu, N, s, fs);
    }
    #pragma unroll
    for (int i = 0; i < 9; ++i) S[sidx<9>(g, x, y, i)] = (T)fs[i];
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_step(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.prec == 1) return a.Q == 9 ? launch_step_f64q9(a, pull, s, ev0, ev1) : launch_step_f64q3(a, pull, s, ev0, ev1);
  return a.Q == 9 ? launch_step_f32q9(a, pull, s, ev0, ev1) : launch_step_f32q3(a, pull, s, ev0, ev1);
}

static unsigned site_grid(const StepArgs& a) {
  const int64_t N = a.g.nx * a.g.ny;
  int64_t nb = (N + 255) / 256;
  return (unsigned)(nb < 8192 ? (nb > 0 ? nb : 1) : 8192);
}

template <typename T, int Q, int QE>
static void init_t(const StepArgs& a, const double* rho0, const double* u0, hipStream_t s) {
  hipLaunchKernelGGL((k_init<T, Q, QE>), dim3(site_grid(a)), dim3(256), 0, s, a, rho0, u0);
}

hipError_t launch_init(const StepArgs& a, const double* rho0, const double* u0, const double* twoE0,
                       hipStream_t s) {
  (void)twoE0;
  if (a.prec == 1) {
    if (a.Q == 9) { if (a.qe == QE_POLY) init_t<double, 9, QE_POLY>(a, rho0, u0, s); else init_t<double, 9, QE_ENTROPIC_MM>(a, rho0, u0, s); }
    else { if (a.qe == QE_POLY) init_t<double, 3, QE_POLY>(a, rho0, u0, s); else init_t<double, 3, QE_ENTROPIC_MM>(a, rho0, u0, s); }
  } else {
    if (a.Q == 9) { if (a.qe == QE_POLY) init_t<float, 9, QE_POLY>(a, rho0, u0, s); else init_t<float, 9, QE_ENTROPIC_MM>(a, rho0, u0, s); }
    else { if (a.qe == QE_POLY) init_t<float, 3, QE_POLY>(a, rho0, u0, s); else init_t<float, 3, QE_ENTROPIC_MM>(a, rho0, u0, s); }
  }
  return hipGetLastError();
}

template <typename T, int Q>
static void get_t(const StepArgs& a, bool pull, void* out, hipStream_t s) {
  if (pull) hipLaunchKernelGGL((k_get<T, Q, true>), dim3(site_grid(a)), dim3(256), 0, s, a, (T*)out);
  else hipLaunchKernelGGL((k_get<T, Q, false>), dim3(site_grid(a)), dim3(256), 0, s, a, (T*)out);
}

hipError_t launch_get(const StepArgs& a, bool pull, void* out, hipStream_t s) {
  if (a.prec == 1) { if (a.Q == 9) get_t<double, 9>(a, pull, out, s); else get_t<double, 3>(a, pull, out, s); }
  else { if (a.Q == 9) get_t<float, 9>(a, pull, out, s); else get_t<float, 3>(a, pull, out, s); }
  return hipGetLastError();
}

hipError_t launch_set(const StepArgs& a, const void* in, hipStream_t s) {
  const unsigned gr = site_grid(a);
  if (a.prec == 1) {
    if (a.Q == 9) hipLaunchKernelGGL((k_set<double, 9>), dim3(gr), dim3(256), 0, s, a, (const double*)in);
    else hipLaunchKernelGGL((k_set<double, 3>), dim3(gr), dim3(256), 0, s, a, (const double*)in);
  } else {
    if (a.Q == 9) hipLaunchKernelGGL((k_set<float, 9>), dim3(gr), dim3(256), 0, s, a, (const float*)in);
    else hipLaunchKernelGGL((k_set<float, 3>), dim3(gr), dim3(256), 0, s, a, (const float*)in);
  }
  return hipGetLastError();
}

template <typename T, int Q>
static void mom_t(const StepArgs& a, bool pull, double* r, double* ru, double* e, hipStream_t s) {
  if (pull) hipLaunchKernelGGL((k_moments<T, Q, true>), dim3(site_grid(a)), dim3(256), 0, s, a, r, ru, e);
  else hipLaunchKernelGGL((k_moments<T, Q, false>), dim3(site_grid(a)), dim3(256), 0, s, a, r, ru, e);
}

hipError_t launch_moments(const StepArgs& a, bool pull, double* rho, double* rhou, double* e2,
                          hipStream_t s) {
  if (a.prec == 1) { if (a.Q == 9) mom_t<double, 9>(a, pull, rho, rhou, e2, s); else mom_t<double, 3>(a, pull, rho, rhou, e2, s); }
  else { if (a.Q == 9) mom_t<float, 9>(a, pull, rho, rhou, e2, s); else mom_t<float, 3>(a, pull, rho, rhou, e2, s); }
  return hipGetLastError();
}

template <typename T, int Q>
static void sums_t(const StepArgs& a, bool pull, hipStream_t s) {
  if (pull) hipLaunchKernelGGL((k_sums<T, Q, true>), dim3(SUM_BLOCKS), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_sums<T, Q, false>), dim3(SUM_BLOCKS), dim3(256), 0, s, a);
}

hipError_t launch_sums(const StepArgs& a, bool pull, hipStream_t s) {
  if (a.prec == 1) { if (a.Q == 9) sums_t<double, 9>(a, pull, s); else sums_t<double, 3>(a, pull, s); }
  else { if (a.Q == 9) sums_t<float, 9>(a, pull, s); else sums_t<float, 3>(a, pull, s); }
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, a, SUM_BLOCKS);
  return hipGetLastError();
}

hipError_t launch_moments_M(const StepArgs& a, bool pull, hipStream_t s) {
  const unsigned gr = (unsigned)a.nblocks;
  if (a.prec == 1) {
    if (pull) hipLaunchKernelGGL((k_moments_M<double, true>), dim3(gr), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_moments_M<double, false>), dim3(gr), dim3(256), 0, s, a);
  } else {
    if (pull) hipLaunchKernelGGL((k_moments_M<float, true>), dim3(gr), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_moments_M<float, false>), dim3(gr), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

int fstep_resident(int prec, int start, bool pull, bool elbm) {
  return prec == 1 ? fstep_resident_f64(start, pull, elbm) : fstep_resident_f32(start, pull, elbm);
}

hipError_t launch_fstep(const StepArgs& a, const FstarArgs& fa, int start, bool pull, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1) {
  hipError_t e = launch_fstar_clear(fa, s);
  if (e != hipSuccess) return e;
  return a.prec == 1 ? launch_fstep_f64(a, fa, start, pull, s, ev0, ev1) : launch_fstep_f32(a, fa, start, pull, s, ev0, ev1);
}

hipError_t launch_init_M_moments(const StepArgs& a, const double* rho0, const double* u0, const double* twoE0,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_init_M_moments, dim3(site_grid(a)), dim3(256), 0, s, a, rho0, u0, twoE0);
  return hipGetLastError();
}

hipError_t launch_init_M_pops(const StepArgs& a, hipStream_t s) {
  if (a.prec == 1) hipLaunchKernelGGL((k_init_M_pops<double>), dim3(site_grid(a)), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_init_M_pops<float>), dim3(site_grid(a)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_clear(const StepArgs& a, hipStream_t s) {
  int64_t n = HIST_WORDS;
  int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_clear, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace lbm
