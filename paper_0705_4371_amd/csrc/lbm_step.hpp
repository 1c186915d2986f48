// lbm_step.hpp -- device code and launch templates of the time-step kernels,
// included by the translation units that instantiate them (one per
// precision and velocity set, so that they compile in parallel).
//
// The gfx950 kernels of the Ehrenfests'-step regularised LBGK
// time step (Sec. 3.2, eq. (ESLB) of Sec. 4.1, boundary rules of Sec. 4.2).
//
// One time step is four kernels on one stream:
//   k_step      fused pull-stream + boundary rules + moments + f* + FP32
//               Delta S screen + LBGK collision + write; screened sites are
//               appended to a list (one atomic per workgroup).  (HBM bound)
//   k_rank      FP64 Delta S of the screened sites; sites with Delta S > delta
//               become candidates (site, Delta S); with more than k screened
//               sites a 2^15-bin histogram of the top key bits is built.
//   k_partition "fewer than k: all of them", otherwise the keys above the
//               histogram bin b* of the k-th largest key are selected and
//               returned to quasiequilibrium (re-pull f(x, t), recompute f*,
//               overwrite the collided values); the keys in b* are listed.
//   k_refine    one workgroup: radix passes over the listed keys find the
//               rest of the k largest; they are reset; statistics.
// (LBM_SELECT_ONE replaces the last three by k_select_one.)  For the
// entropic f*_M quasiequilibrium k_fstep takes the place of k_step: it also
// runs the per-site Newton solve, and k_fstep_fallback solves and collides
// the few sites whose first pass failed (with a network start the solve
// runs before k_step instead).
//
// State layout: tiles of 64 sites of a row, [ny][pitch/64][Q][64] of T
// (float or double), pitch = nx rounded up to 64 (see sidx).  The state
// buffer holds the post-collision populations f'(x, t-1) at their origin
// site ("pull" layout); right after init or set_populations it holds the
// pre-collision f(x, t) itself ("canonical" layout) and the first step reads
// it in place.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_device.hpp"
#include "lbm_fstar_dev.hpp"
#include "lbm_fstar_site.hpp"
#include "lbm_launch.hpp"

namespace lbm {

// logical block index for a hardware block id: hardware dispatch deals
// blocks round-robin over the 8 XCDs, so consecutive logical tiles (which
// share halo cache lines) are given to the same XCD and its L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t per = nb >> 3, rem = nb & 7, xcd = b & 7, idx = b >> 3;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// f_i(x, y, t) from the post-collision state with the boundary rules:
// x outside: periodic wrap | inlet quasiequilibrium | zero-gradient (the
// value the adjacent inner column receives) | outlet (handled by load_site;
// never reached here); y outside: periodic wrap | free-slip (specular: the
// vertically mirrored population leaving from (x - cx, y)) | zero-gradient;
// source in the solid: halfway bounce-back.
template <typename T, int Q>
__device__ __forceinline__ T pull_general(const T* __restrict__ A, const Geom& g, int64_t x, int64_t y,
                                          int i) {
  const int cx = Lat<Q>::cx[i], cy = Lat<Q>::cy[i];
  for (int it = 0; it < 4; ++it) {
    int64_t sx = x - cx, sy = y - cy;
    int j = i;
    if (sx < 0 || sx >= g.nx) {
      const int b = sx < 0 ? g.bc[0] : g.bc[1];
      if (b == BC_PERIODIC) sx = sx < 0 ? sx + g.nx : sx - g.nx;
      else if (b == BC_INLET_EQ) return T(g.feq_in[i]);
      else if (b == BC_OUTLET_EQ || b == BC_OUTLET_EQ_PREV) return T(0);
      else { x = sx < 0 ? x + 1 : x - 1; continue; }
    }
    if (sy < 0 || sy >= g.ny) {
      const int b = sy < 0 ? g.bc[2] : g.bc[3];
      if (b == BC_PERIODIC) sy = sy < 0 ? sy + g.ny : sy - g.ny;
      else if (b == BC_FREESLIP) { j = Lat<Q>::mir[i]; sy = y; }
      else if (b == BC_INLET_EQ) return T(g.feq_in[i]);
      else { y = sy < 0 ? y + 1 : y - 1; continue; }
    }
    if (is_solid(g, sx, sy)) { j = Lat<Q>::opp[i]; sx = x; sy = y; }
    return A[sidx<Q>(g, sx, sy, j)];
  }
  return T(0);
}

// outlet rule of the channel (Sec. 4.2): the populations entering through
// an outlet face are the quasiequilibrium at the density and velocity of the
// penultimate column xp: of its new state f(xp, y, t) (BC_OUTLET_EQ), or of
// its state one step earlier (BC_OUTLET_EQ_PREV), read from the
// post-collision values stored at (xp, y), which carry the same density and
// momentum
template <typename T, int Q>
__device__ __forceinline__ void pull_outlet(const T* __restrict__ A, const Geom& g, int64_t x, int64_t xp,
                                         int64_t y, bool prev, T* f) {
  T p[Q], fe[Q];
  #pragma unroll
  for (int i = 0; i < Q; ++i) p[i] = prev ? A[sidx<Q>(g, xp, y, i)] : pull_general<T, Q>(A, g, xp, y, i);
  const Moments<Q, T> m = moments<Q, T>(p);
  const T ux = m.jx / m.rho, uy = m.jy / m.rho;
  if (g.out_qe == QE_POLY) qe_poly<Q, T>(m.rho, ux, uy, fe);
  else qe_entropic_mm<Q, T>(m.rho, ux, uy, fe);
  #pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int64_t sx = x - Lat<Q>::cx[i];
    f[i] = (sx < 0 || sx >= g.nx) ? fe[i] : pull_general<T, Q>(A, g, x, y, i);
  }
}

// canonical pre-collision populations of one fluid site
template <typename T, int Q, bool PULL>
__device__ __forceinline__ void load_site(const T* __restrict__ A, const Geom& g, int64_t x, int64_t y,
                                          T* f) {
  if (PULL) {
    if (x == 0 && (g.bc[0] == BC_OUTLET_EQ || g.bc[0] == BC_OUTLET_EQ_PREV)) {
      pull_outlet<T, Q>(A, g, x, 1, y, g.bc[0] == BC_OUTLET_EQ_PREV, f);
      return;
    }
    if (x == g.nx - 1 && (g.bc[1] == BC_OUTLET_EQ || g.bc[1] == BC_OUTLET_EQ_PREV)) {
      pull_outlet<T, Q>(A, g, x, g.nx - 2, y, g.bc[1] == BC_OUTLET_EQ_PREV, f);
      return;
    }
  }
  #pragma unroll
  for (int i = 0; i < Q; ++i)
    f[i] = PULL ? pull_general<T, Q>(A, g, x, y, i) : A[sidx<Q>(g, x, y, i)];
}

// f(x, t) of one fluid site for the ranking and the resets: a site whose
// 3 x 3 neighbourhood lies inside the lattice and clear of the solid pulls
// its nine populations directly (independent loads); others take the
// boundary rules
template <typename T, int Q, bool PULL>
__device__ __forceinline__ void load_site_fast(const T* __restrict__ A, const Geom& g, int64_t x, int64_t y,
                                               T* f) {
  if (PULL) {
    const bool xin = x >= 1 && x <= g.nx - 2;
    const bool yin = (Q == 3) || (y >= 1 && y <= g.ny - 2);
    const bool hit = x - 1 < g.sx1 && x + 1 >= g.sx0 && y - 1 < g.sy1 && y + 1 >= g.sy0;
    if (xin && yin && !hit) {
      const int64_t rs = g.pitch * Q;
      const uint32_t oc[3] = {col_bytes<T, Q>(x - 1), col_bytes<T, Q>(x), col_bytes<T, Q>(x + 1)};
      #pragma unroll
      for (int i = 0; i < Q; ++i) {
        const char* row = (const char*)(A + (y - Lat<Q>::cy[i]) * rs);
        f[i] = *(const T*)(row + oc[1 - Lat<Q>::cx[i]] + i * 64 * (int)sizeof(T));
      }
      return;
    }
  }
  load_site<T, Q, PULL>(A, g, x, y, f);
}

// f*_M populations of site s from the solver's product-form state
// (A, X, Y, Z) [4][N]
template <typename T>
__device__ __forceinline__ void fstar_from_state(const double* __restrict__ st, int64_t N, int64_t s, T* fs) {
  fstar_pop<T>((T)st[s], (T)st[N + s], (T)st[2 * N + s], (T)st[3 * N + s], fs);
}

// block-wide exclusive offset of `flag` and one global atomic per block on
// *counter; s_cnt: STEP_TX / 64 words of LDS; returns the slot of a flagged
// lane
__device__ __forceinline__ uint32_t block_append(bool flag, uint32_t* counter, uint32_t* s_cnt,
                                                 uint32_t* s_base) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const unsigned long long mask = __ballot(flag);
  if (lane == 0) s_cnt[w] = (uint32_t)__popcll(mask);
  __syncthreads();
  if (tid == 0) {
    uint32_t tot = 0u;
    #pragma unroll
    for (int v = 0; v < STEP_TX / 64; ++v) tot += s_cnt[v];
    *s_base = tot ? atomicAdd(counter, tot) : 0u;
  }
  __syncthreads();
  uint32_t base = *s_base;
  for (int v = 0; v < w; ++v) base += s_cnt[v];
  const uint32_t slot = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
  __syncthreads();  // s_cnt / s_base are reused by the next call
  return slot;
}

// f(x, t) of lane x of the row segment [x0, x0 + STEP_TX) of row y: segments
// whose whole 3 x (STEP_TX + 2) neighbourhood is inside the lattice and clear
// of the solid pull directly (a uniform branch per block); other fluid sites
// take the boundary rules; non-fluid lanes get the rest weights (unused)
template <typename T, int Q, bool PULL>
__device__ __forceinline__ void load_segment_site(const T* __restrict__ A, const Geom& g, int64_t x0, int64_t x,
                                                  int64_t y, bool fluid, T* f) {
  if (PULL) {
    const bool xin = x0 >= 1 && x0 + STEP_TX <= g.nx - 1;
    const bool yin = (Q == 3) || (y >= 1 && y <= g.ny - 2);
    const bool hit = x0 - 1 < g.sx1 && x0 + STEP_TX >= g.sx0 && y - 1 < g.sy1 && y + 1 >= g.sy0;
    if (xin && yin && !hit) {
      // rows y - 1, y, y + 1 at uniform bases, columns x - 1, x, x + 1 at
      // per-lane 32-bit offsets, population i at a constant 64 i elements
      const int64_t rs = g.pitch * Q;
      const uint32_t oc[3] = {col_bytes<T, Q>(x - 1), col_bytes<T, Q>(x), col_bytes<T, Q>(x + 1)};
      #pragma unroll
      for (int i = 0; i < Q; ++i) {
        const char* row = (const char*)(A + (y - Lat<Q>::cy[i]) * rs);
        f[i] = *(const T*)(row + oc[1 - Lat<Q>::cx[i]] + i * 64 * (int)sizeof(T));
      }
      return;
    }
  }
  if (fluid) {
    load_site<T, Q, PULL>(A, g, x, y, f);
  } else {
    #pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = T(Lat<Q>::w(i));
  }
}

// ---------------------------------------------------------------------------
// k_step
// ---------------------------------------------------------------------------
// monitoring point (Sec. 4.2): density and velocity of f(x, t), one sample
// per step into a ring (only the probe's lane ever calls it)
template <int Q, typename T>
__device__ __forceinline__ void probe_sample(const StepArgs& a, const Moments<Q, T>& m) {
  const unsigned long long n = *a.probe_n;
  const int64_t j = (int64_t)(n % (unsigned long long)a.probe_cap);
  a.probe_buf[j] = (double)m.rho;
  a.probe_buf[a.probe_cap + j] = (double)m.jx / (double)m.rho;
  a.probe_buf[2 * a.probe_cap + j] = (double)m.jy / (double)m.rho;
  *a.probe_n = n + 1;
}

// FP32 screen of Delta S for the entropic quasiequilibria (artanh series,
// with a margin); screened sites are re-ranked in FP64
template <int Q, typename T>
__device__ __forceinline__ bool screen_entropic(const StepArgs& a, const T* f, const T* fs, T rho) {
  float ff[Q], fsf[Q];
  #pragma unroll
  for (int i = 0; i < Q; ++i) { ff[i] = (float)f[i]; fsf[i] = (float)fs[i]; }
  const float ds = dS_screen<Q>(ff, fsf);
  const float thr = a.thr_a - a.thr_b * __builtin_sqrtf(fmaxf((float)rho, 0.0f));
  return !(ds < thr);
}

// LBGK collision f' = f + 2 beta (f* - f) (eq. (lbgkLB)), or ELBM
// f' = f + alpha beta (f* - f) (eq. (elbmLB)), written at the origin site
// with non-temporal stores (nothing reads it again in this step); returns
// the sum of the written values (non-finite iff one of them is, or they
// overflow)
template <typename T, int Q, bool ELBM>
__device__ __forceinline__ T collide_store(const StepArgs& a, int64_t x, int64_t y, const T* f, const T* fs) {
  T* __restrict__ B = (T*)a.B;
  T b2 = T(a.g.beta2);
  if constexpr (ELBM) {
    double fd[Q], fsd[Q];
    #pragma unroll
    for (int i = 0; i < Q; ++i) { fd[i] = (double)f[i]; fsd[i] = (double)fs[i]; }
    b2 = T(0.5 * a.g.beta2 * elbm_alpha<Q>(fd, fsd));
  }
  T sum = T(0);
  char* row = (char*)(B + y * (a.g.pitch * Q)) + col_bytes<T, Q>(x);
  #pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T v = f[i] + b2 * (fs[i] - f[i]);
    sum += v;
    __builtin_nontemporal_store(v, (T*)(row + i * 64 * (int)sizeof(T)));
  }
  return sum;
}

// Non-finite halt.  The first step that meets non-finite values (in the
// populations it reads or writes) records itself in C_NONFINITE / C_BADSTEP;
// every step kernel launched after that returns at once, so the buffer the
// step read -- the last finite state -- is kept for the host to recover.
__device__ __forceinline__ bool halted(const StepArgs& a) { return a.ctr[C_NONFINITE] != 0u; }

template <bool PULL>
__device__ __forceinline__ void raise_nonfinite(const StepArgs& a) {
  const uint32_t tag = 1u + (uint32_t)a.dst + (PULL ? 0u : 2u);
  if (atomicCAS(&a.ctr[C_NONFINITE], 0u, tag) == 0u) a.ctr[C_BADSTEP] = a.ctr[C_STEP0 + 1 - a.dst] + 1u;
}

// step number of buffer dst: one more than that of the buffer read (the
// latter is not written during this step, so every block sees one value)
__device__ __forceinline__ void count_step(const StepArgs& a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ctr[C_STEP0 + a.dst] = a.ctr[C_STEP0 + 1 - a.dst] + 1u;
}

// the screened sites of the workgroup are appended with one atomic, and the
// non-finite halt is raised (every thread of the block calls this)
template <bool PULL>
__device__ __forceinline__ void append_screened(const StepArgs& a, bool scr, uint32_t site, bool bad) {
  if (__syncthreads_or(scr)) {
    __shared__ uint32_t s_cnt[STEP_TX / 64], s_base;
    const uint32_t slot = block_append(scr, &a.ctr[C_SCREEN], s_cnt, &s_base);
    if (scr) a.screen[slot] = site;
  }
  // once the flag is set, waves only read it (no atomic storm on one word)
  if (__ballot(bad) && (threadIdx.x & 63) == 0 && __atomic_load_n(&a.ctr[C_NONFINITE], __ATOMIC_RELAXED) == 0u)
    raise_nonfinite<PULL>(a);
}

template <typename T, int Q, int QE, bool PULL, bool ELBM = false>
__global__ __launch_bounds__(STEP_TX) void k_step(StepArgs a) {
  // another workgroup of this very step may raise the halt while this one
  // runs, so each wave decides for itself and skips its writes (not the
  // workgroup's barriers)
  const bool live = !halted(a);
  count_step(a);
  const T* __restrict__ A = (const T*)a.A;
  const Geom& g = a.g;
  const int64_t b = xcd_remap(blockIdx.x, a.nblocks);
  const int64_t y = b / a.ntx;
  const int64_t x0 = (b - y * a.ntx) * STEP_TX;
  const int64_t x = x0 + threadIdx.x;
  const bool fluid = x < g.nx && !is_solid(g, x, y);

  T f[Q];
  load_segment_site<T, Q, PULL>(A, g, x0, x, y, fluid, f);

  const Moments<Q, T> m = moments<Q, T>(f);
  if (live && fluid && x + y * g.nx == a.probe) probe_sample<Q, T>(a, m);
  T fs[Q], pb[Q];
  const T inv = inv_of(m.rho);
  const T ux = m.jx * inv, uy = m.jy * inv;
  if constexpr (QE == QE_POLY) qe_poly_br<Q, T>(m.rho, ux, uy, fs, pb);
  else if constexpr (QE == QE_ENTROPIC_MM) qe_entropic_mm<Q, T>(m.rho, ux, uy, fs);
  else {
    if (fluid) fstar_from_state<T>(a.mu, g.nx * g.ny, x + y * g.nx, fs);
    else {
      #pragma unroll
      for (int i = 0; i < Q; ++i) fs[i] = f[i];
    }
  }

  // FP32 screen of Delta S (an upper bound for the polynomial QE, an
  // estimate with a margin otherwise); screened sites are re-ranked in FP64
  bool scr = false;
  if (g.ds_on && fluid) {
    if constexpr (QE == QE_POLY) {
      float ff[Q], fsf[Q], pf[Q];
      #pragma unroll
      for (int i = 0; i < Q; ++i) { ff[i] = (float)f[i]; fsf[i] = (float)fs[i]; pf[i] = (float)pb[i]; }
      const float ds = dS_bound_poly<Q>(ff, fsf, pf, (float)inv);
      const float thr = a.thr_a - a.thr_b * __builtin_sqrtf(fmaxf((float)m.rho, 0.0f));
      scr = !(ds < thr);
    } else {
      scr = screen_entropic<Q, T>(a, f, fs, m.rho);
    }
  }

  T osum = T(0);
  if (live && fluid) osum = collide_store<T, Q, ELBM>(a, x, y, f, fs);
  append_screened<PULL>(a, live && scr, (uint32_t)(x + y * g.nx),
                        live && fluid && !(__builtin_isfinite(m.rho) && __builtin_isfinite(osum)));
}

// ---------------------------------------------------------------------------
// Ranking and selection (Sec. 3.2: at most k sites with Delta S > delta,
// the largest first, ties by lower site index)
// ---------------------------------------------------------------------------
// Key of a candidate: the 63 bits of its non-negative FP64 Delta S followed
// by the 32 bits of ~site (a larger key = larger Delta S, then lower site).
// Keys are unique, so "the k largest keys" is one well-defined set.
//   k_rank      FP64 Delta S of the screened sites; candidates are collected
//               per workgroup in LDS and appended with one atomic per flush
//               of that buffer; when more than k sites were
//               screened, a 2^15-bin histogram of the top key bits is built
//               (in LDS per workgroup when many sites are screened).
//   k_partition with more than k candidates, each workgroup finds the bin b*
//               holding the k-th largest key (and r, the keys to take from
//               it) in the histogram; candidates above b* (or all of them,
//               if there are at most k) are selected and returned to
//               quasiequilibrium at once; candidates in b* go to a boundary
//               list.
//   k_refine    one workgroup: 8-bit radix passes over the boundary list find
//               the r largest keys there, which are selected and reset; the
//               statistics are written and the counters cleared.
// (Kernel boundaries order these phases: a device-wide fence inside a
// kernel would write back the L2 of every XCD.)
__device__ __forceinline__ unsigned long long ds_bits(double d) {
  return (unsigned long long)__double_as_longlong(d);
}

__device__ __forceinline__ uint32_t ds_bin(double d) {
  return (uint32_t)(ds_bits(d) >> 48) & (HIST_BINS - 1);
}

// return one selected site to quasiequilibrium: re-pull f(x, t) from the
// state A, the same f* as k_step, written over the collided values in B
template <typename T, int Q, int QE, bool PULL>
__device__ __forceinline__ void reset_site(const StepArgs& a, uint32_t site) {
  const T* __restrict__ A = (const T*)a.A;
  T* __restrict__ B = (T*)a.B;
  const Geom& g = a.g;
  int64_t x, y;
  divmod((int64_t)site, g.nx, g.inv_nx, y, x);
  T fs[Q];
  if constexpr (QE == QE_ENTROPIC_M) {
    fstar_from_state<T>(a.mu, g.nx * g.ny, site, fs);
  } else {
    T f[Q];
    load_site_fast<T, Q, PULL>(A, g, x, y, f);
    const Moments<Q, T> m = moments<Q, T>(f);
    qe_eval<Q, QE, T>(m, fs);
  }
  #pragma unroll
  for (int i = 0; i < Q; ++i) B[sidx<Q>(g, x, y, i)] = fs[i];
}

// FP64 Delta S of one site for the ranking: f(x, t) re-pulled from the
// state, promoted to FP64; f* in FP64 (for f*_M the solver's state polished
// to FP64 round-off)
template <typename T, int Q, int QE, bool PULL>
__device__ __forceinline__ double rank_site(const StepArgs& a, const T* __restrict__ A, const Geom& g,
                                            uint32_t site) {
  int64_t x, y;
  divmod((int64_t)site, g.nx, g.inv_nx, y, x);
  T fT[Q];
  load_site_fast<T, Q, PULL>(A, g, x, y, fT);
  double fd[Q];
  #pragma unroll
  for (int i = 0; i < Q; ++i) fd[i] = (double)fT[i];
  const Moments<Q, double> m = moments<Q, double>(fd);
  double fs[Q];
  if constexpr (QE == QE_ENTROPIC_M) {
    const int64_t N = g.nx * g.ny;
    const double ir = 1.0 / m.rho;
    if (feasible(m.rho, m.jx * ir, m.jy * ir, m.e2 * ir)) {
      const FS<double> s0{a.mu[site] * ir, a.mu[N + site], a.mu[2 * N + site], a.mu[3 * N + site]};
      const FS<double> p = polish64(s0, m.jx * ir, m.jy * ir, m.e2 * ir, 3);
      fstar_pop<double>(m.rho * p.a, p.X, p.Y, p.Z, fs);
    } else {
      fstar_from_state<double>(a.mu, N, site, fs);
    }
  } else {
    qe_eval<Q, QE, double>(m, fs);
  }
  return dS_fp64<Q>(fd, fs);
}

constexpr int RANK_BLOCKS = 512;
constexpr uint32_t LDS_HIST_MIN = 16384;  // screened sites above which the histogram is built in LDS

// 512 lanes per workgroup: the 64 KB LDS histogram then serves 16 waves of
// a CU (two workgroups) instead of 8 -- the ranking is latency bound
constexpr uint32_t RANK_TX = 512;

// adds the workgroup's LDS histogram (two 16-bit counts per word) to the
// global fine and coarse histograms and clears it; a wavefront's 64 words
// lie in one coarse bin, whose count it adds with one atomic
__device__ __forceinline__ void flush_hist(const StepArgs& a, uint32_t* s_hist) {
  const int tid = threadIdx.x, lane = tid & 63;
  for (int j = tid; j < HIST_BINS / 2; j += (int)RANK_TX) {
    const uint32_t v = s_hist[j];
    const uint32_t lo = v & 0xFFFFu, hi = v >> 16;
    if (lo) atomicAdd(&a.hist[2 * j], lo);
    if (hi) atomicAdd(&a.hist[2 * j + 1], hi);
    s_hist[j] = 0u;
    if (__ballot(v != 0u)) {
      uint32_t c = lo + hi;
      #pragma unroll
      for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
      if (lane == 0 && c) atomicAdd(&a.hist[HIST_BINS + (j >> 7)], c);
    }
  }
}

// FP64 Delta S of every screened site t (its position in the list): the
// candidate entry cand[t] = (site, Delta S) is written in place, with
// Delta S = -1 for a site at or below delta, so that no compaction (no
// barrier, no shared counter) is needed; the candidates are counted per
// workgroup with LDS atomics and added to C_CAND once.  With more than k
// screened sites a 2^15-bin histogram of the candidates' top key bits is
// built (in LDS per workgroup when many sites are screened).
template <typename T, int Q, int QE, bool PULL>
__device__ __forceinline__ void rank_body(const StepArgs& a) {
  if (halted(a)) return;  // (not raised by the selection kernels: uniform)
  __shared__ uint32_t s_hist[HIST_BINS / 2];  // two 16-bit counts per word
  __shared__ uint32_t s_nc, s_ninv;
  const T* __restrict__ A = (const T*)a.A;
  const Geom& g = a.g;
  const int tid = threadIdx.x;
  const uint32_t n = a.ctr[C_SCREEN];
  const uint32_t k = (uint32_t)g.kmax;
  // with at most k screened sites every candidate is selected: no histogram
  const bool need_hist = k > 0 && n > k;
  const bool lds = need_hist && n > LDS_HIST_MIN;
  // only the workgroups that hold screened sites take part
  if (blockIdx.x * RANK_TX >= n) return;
  if (lds)
    for (int j = tid; j < HIST_BINS / 2; j += (int)RANK_TX) s_hist[j] = 0u;
  if (tid == 0) { s_nc = 0u; s_ninv = 0u; }
  __syncthreads();
  uint32_t it = 0;
  // the trip count is uniform over the workgroup (the periodic flush of the
  // LDS histogram has barriers); the site of the thread's next entry is
  // loaded one iteration ahead
  const uint32_t stride = gridDim.x * RANK_TX;
  uint32_t next = blockIdx.x * RANK_TX + tid < n ? a.screen[blockIdx.x * RANK_TX + tid] : 0u;
  for (uint32_t t0 = blockIdx.x * RANK_TX; t0 < n; t0 += stride) {
    const uint32_t t = t0 + tid;
    const uint32_t site = next;
    if (t + stride < n) next = a.screen[t + stride];
    if (t < n) {
      const double ds = rank_site<T, Q, QE, PULL>(a, A, g, site);
      const bool is_c = ds > g.delta;
      a.cand[t] = Cand{site, 0u, is_c ? ds : -1.0};
      if (is_c) {
        atomicAdd(&s_nc, 1u);
        if (__builtin_isinf(ds)) atomicAdd(&s_ninv, 1u);
        const uint32_t bin = ds_bin(ds);
        if (lds) {
          atomicAdd(&s_hist[bin >> 1], 1u << (16 * (bin & 1u)));
        } else if (need_hist) {
          atomicAdd(&a.hist[bin], 1u);
          atomicAdd(&a.hist[HIST_BINS + (bin >> 8)], 1u);
        }
      }
    }
    // flushed every 64 iterations: at most 64 x 512 = 32768 keys per
    // 16-bit count
    if (lds && (++it & (32768u / RANK_TX - 1u)) == 0u) {
      __syncthreads();
      flush_hist(a, s_hist);
      __syncthreads();
    }
  }
  __syncthreads();
  if (lds) flush_hist(a, s_hist);
  if (tid == 0) {
    if (s_nc) atomicAdd(&a.ctr[C_CAND], s_nc);
    if (s_ninv) atomicAdd(&a.ctr[C_INVALID], s_ninv);
  }
}

// Two entry points over the same body: at most 128 VGPRs (two workgroups,
// 16 waves, per CU) where that needs no scratch, and the unconstrained
// bound for the f*_M quasiequilibrium, whose Delta S would spill within 128.
template <typename T, int Q, int QE, bool PULL>
__global__ __launch_bounds__(RANK_TX, 4) void k_rank(StepArgs a) {
  rank_body<T, Q, QE, PULL>(a);
}

template <typename T, int Q, int QE, bool PULL>
__global__ __launch_bounds__(RANK_TX) void k_rank_m(StepArgs a) {
  rank_body<T, Q, QE, PULL>(a);
}

// keys buffered in LDS per partition workgroup (selected / boundary)
constexpr uint32_t PART_BUF = 512;

// inclusive prefix sums of s_scan[0 .. 255] in place (all 256 threads)
__device__ __forceinline__ void scan256(uint32_t* s_scan) {
  const int tid = threadIdx.x;
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t v = tid >= off ? s_scan[tid - off] : 0u;
    __syncthreads();
    s_scan[tid] += v;
    __syncthreads();
  }
}

// b*, the histogram bin that holds the k-th largest key, and r, the keys to
// take from it (1 <= r): the coarse bin holding it first, from the top down
// (thread t reads coarse bin HIST_COARSE - 1 - t), then the 256 fine bins of
// that coarse bin (thread t reads the t-th from its top); 256 threads, both
// reads coalesced.  Needs more than k keys in the histogram.
__device__ __forceinline__ void find_bstar(const uint32_t* __restrict__ hist, uint32_t k, uint32_t* s_scan,
                                           uint32_t* s_sel, uint32_t* s_bstar, uint32_t* s_r) {
  const int tid = threadIdx.x;
  const uint32_t cv = tid < HIST_COARSE ? hist[HIST_BINS + HIST_COARSE - 1 - tid] : 0u;
  s_scan[tid] = cv;
  __syncthreads();
  scan256(s_scan);
  {
    const uint32_t incl = s_scan[tid], excl = incl - cv;
    if (tid < HIST_COARSE && excl < k && incl >= k) { s_sel[0] = HIST_COARSE - 1 - tid; s_sel[1] = k - excl; }
  }
  __syncthreads();
  const uint32_t cs = s_sel[0], r1 = s_sel[1];
  const uint32_t fv = hist[cs * 256 + 255 - tid];
  s_scan[tid] = fv;
  __syncthreads();
  scan256(s_scan);
  {
    const uint32_t incl = s_scan[tid], excl = incl - fv;
    if (excl < r1 && incl >= r1) { *s_bstar = cs * 256 + 255 - tid; *s_r = r1 - excl; }
  }
  __syncthreads();
}

template <typename T, int Q, int QE, bool PULL>
__global__ __launch_bounds__(256) void k_partition(StepArgs a) {
  if (halted(a)) return;
  __shared__ uint32_t s_base, s_bstar, s_r, s_sel[2];
  __shared__ uint32_t s_scan[256];
  __shared__ unsigned long long s_mx[4], s_mn[4];
  // the workgroup's selected keys and boundary keys, collected with LDS
  // atomics (no barrier per iteration) and written out with one global
  // atomic each at the end; beyond PART_BUF a key is appended directly
  __shared__ uint32_t s_ntake, s_nbnd;
  __shared__ Cand s_take[PART_BUF], s_bnd[PART_BUF];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t nc = a.ctr[C_CAND];
  const uint32_t n = a.ctr[C_SCREEN];
  const uint32_t k = (uint32_t)a.g.kmax;
  // only the workgroups that hold candidate entries take part (the others
  // leave neutral partials for k_refine)
  if (nc == 0 || blockIdx.x * 256u >= n) {
    if (tid == 0) {
      a.part[blockIdx.x] = 0ull;
      a.part[PART_BLOCKS + blockIdx.x] = ~0ull;
    }
    return;
  }
  if (tid == 0) { s_ntake = 0u; s_nbnd = 0u; }
  // more than k candidates: every workgroup locates b* in the (complete)
  // histogram itself; workgroup 0 records it for k_refine
  const bool all = k == 0 || n <= k || nc <= k;
  uint32_t bstar = 0;
  if (!all) {
    find_bstar(a.hist, k, s_scan, s_sel, &s_bstar, &s_r);
    bstar = s_bstar;
    if (blockIdx.x == 0 && tid == 0) { a.ctr[C_BSTAR] = bstar; a.ctr[C_R] = s_r; }
  }
  __syncthreads();
  unsigned long long mx = 0ull, mn = ~0ull;
  // the entries of the n screened sites; Delta S < 0 marks a non-candidate.
  // The next entry of the thread is loaded before the current one is
  // handled, so that its latency overlaps the work (no barrier in the loop)
  const uint32_t stride = gridDim.x * 256u;
  uint32_t t = blockIdx.x * 256u + tid;
  Cand cn = t < n ? a.cand[t] : Cand{0u, 0u, -1.0};
  for (; t < n; t += stride) {
    const Cand c = cn;
    if (t + stride < n) cn = a.cand[t + stride];
    if (c.ds < 0.0) continue;
    const uint32_t bin = ds_bin(c.ds);
    const bool take = k > 0 && (all || bin > bstar);
    const bool bnd = !all && k > 0 && bin == bstar;
    mx = ds_bits(c.ds) > mx ? ds_bits(c.ds) : mx;
    if (take) {
      mn = ds_bits(c.ds) < mn ? ds_bits(c.ds) : mn;
      reset_site<T, Q, QE, PULL>(a, c.site);
      const uint32_t slot = atomicAdd(&s_ntake, 1u);
      if (slot < PART_BUF) {
        s_take[slot] = c;
      } else {
        const uint32_t g = atomicAdd(&a.ctr[C_NSEL0], 1u);
        a.sel[g] = c.site;
        a.sel_ds[g] = c.ds;
      }
    }
    if (bnd) {
      const uint32_t slot = atomicAdd(&s_nbnd, 1u);
      if (slot < PART_BUF) s_bnd[slot] = c;
      else a.bnd[atomicAdd(&a.ctr[C_NBND], 1u)] = c;
    }
  }
  __syncthreads();
  const uint32_t nt = s_ntake < PART_BUF ? s_ntake : PART_BUF;
  const uint32_t nb = s_nbnd < PART_BUF ? s_nbnd : PART_BUF;
  if (tid == 0) {
    s_base = nt ? atomicAdd(&a.ctr[C_NSEL0], nt) : 0u;
    s_sel[0] = nb ? atomicAdd(&a.ctr[C_NBND], nb) : 0u;
  }
  __syncthreads();
  for (uint32_t j = tid; j < nt; j += 256u) {
    a.sel[s_base + j] = s_take[j].site;
    a.sel_ds[s_base + j] = s_take[j].ds;
  }
  for (uint32_t j = tid; j < nb; j += 256u) a.bnd[s_sel[0] + j] = s_bnd[j];
  // workgroup max of all candidates and min of the selected ones
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long ox = (unsigned long long)__shfl_xor((long long)mx, off);
    const unsigned long long on = (unsigned long long)__shfl_xor((long long)mn, off);
    mx = ox > mx ? ox : mx;
    mn = on < mn ? on : mn;
  }
  if (lane == 0) { s_mx[w] = mx; s_mn[w] = mn; }
  __syncthreads();
  if (tid == 0) {
    for (int v = 1; v < 4; ++v) {
      mx = s_mx[v] > mx ? s_mx[v] : mx;
      mn = s_mn[v] < mn ? s_mn[v] : mn;
    }
    mx = s_mx[0] > mx ? s_mx[0] : mx;
    mn = s_mn[0] < mn ? s_mn[0] : mn;
    // per-workgroup partials (reduced by k_refine), not atomics on one word
    a.part[blockIdx.x] = mx;
    a.part[PART_BLOCKS + blockIdx.x] = mn;
  }
}

// k_refine: the boundary refinement, the statistics and the clearing of the
// counters for the next step, by one workgroup of REF_TX threads (many
// lanes, so that the resets of the keys taken from the boundary bin run in
// few rounds); boundary keys are staged in LDS when at most REFINE_LDS
constexpr uint32_t REFINE_LDS = 8192;
constexpr int REF_TX = 1024;
static_assert(REF_TX == PART_BLOCKS, "k_refine reads one partition partial per thread");

template <typename T, int Q, int QE, bool PULL>
__global__ __launch_bounds__(REF_TX) void k_refine(StepArgs a) {
  if (halted(a)) return;
  __shared__ uint32_t s_hist[256];
  __shared__ uint32_t s_nsel, s_dig, s_rr, s_exact;
  __shared__ unsigned long long s_mx[REF_TX / 64], s_mn[REF_TX / 64];
  __shared__ unsigned long long s_khi[REFINE_LDS];
  __shared__ uint32_t s_klo[REFINE_LDS];
  const int tid = threadIdx.x;
  const uint32_t nc = a.ctr[C_CAND];
  const uint32_t n = a.ctr[C_SCREEN];
  const uint32_t k = (uint32_t)a.g.kmax;
  const bool all = k == 0 || n <= k || nc <= k;
  const uint32_t nsel0 = a.ctr[C_NSEL0];
  const uint32_t m = a.ctr[C_NBND];
  // max of all candidates and min of the selected ones: the partition's
  // per-workgroup partials, then the keys selected here
  unsigned long long mx = a.part[tid], mn = a.part[PART_BLOCKS + tid];
  if (tid == 0) s_nsel = 0;
  __syncthreads();

  if (nc > 0 && !all) {
    // the remaining key of each boundary candidate: Delta S bits 47..0 and
    // ~site, read once from memory into LDS when they fit
    const bool staged = m <= REFINE_LDS;
    if (staged) {
      for (uint32_t t = tid; t < m; t += REF_TX) {
        const Cand c = a.bnd[t];
        s_khi[t] = ds_bits(c.ds) & 0xFFFFFFFFFFFFull;
        s_klo[t] = ~c.site;
      }
      __syncthreads();
    }
    // 8-bit digits of the remaining key below the histogram bits: Delta S
    // bits 47..0, then ~site; rr keys are still to be taken
    unsigned long long Thi = 0, Mhi = 0;
    uint32_t Tlo = 0, Mlo = 0, rr = a.ctr[C_R];
    for (int pass = 0; pass < 10; ++pass) {
      const bool inhi = pass < 6;
      const int sh = inhi ? 40 - 8 * pass : 24 - 8 * (pass - 6);
      if (tid < 256) s_hist[tid] = 0;
      __syncthreads();
      for (uint32_t t = tid; t < m; t += REF_TX) {
        unsigned long long hi;
        uint32_t lo;
        if (staged) {
          hi = s_khi[t];
          lo = s_klo[t];
        } else {
          const Cand c = a.bnd[t];
          hi = ds_bits(c.ds) & 0xFFFFFFFFFFFFull;
          lo = ~c.site;
        }
        if ((hi & Mhi) == Thi && (lo & Mlo) == Tlo) {
          const uint32_t d = inhi ? (uint32_t)(hi >> sh) & 255u : (lo >> sh) & 255u;
          atomicAdd(&s_hist[d], 1u);
        }
      }
      __syncthreads();
      // the digit holding the rr-th largest remaining key, by the first
      // wavefront alone: lane l holds digits 255 - 4l .. 252 - 4l (from the
      // top), the suffix sums run over the lanes by shuffles
      if (tid < 64) {
        uint32_t h[4], c = 0;
        #pragma unroll
        for (int j = 0; j < 4; ++j) { h[j] = s_hist[255 - 4 * tid - j]; c += h[j]; }
        uint32_t incl = c;
        #pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const uint32_t u = __shfl_up(incl, off);
          if (tid >= off) incl += u;
        }
        uint32_t excl = incl - c;
        if (excl < rr && incl >= rr) {
          #pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (excl < rr && excl + h[j] >= rr) {
              s_dig = 255u - 4u * (uint32_t)tid - (uint32_t)j;
              s_rr = rr - excl;
              s_exact = (h[j] == rr - excl);
            }
            excl += h[j];
          }
        }
      }
      __syncthreads();
      const uint32_t d = s_dig;
      rr = s_rr;
      if (inhi) { Thi |= (unsigned long long)d << sh; Mhi |= 255ull << sh; }
      else { Tlo |= d << sh; Mlo |= 255u << sh; }
      const bool done = s_exact != 0;
      __syncthreads();
      if (done) break;
    }
    // keys of the bin that are >= T (T's unfixed low bits are zero)
    for (uint32_t t = tid; t < m; t += REF_TX) {
      const Cand c = a.bnd[t];
      const unsigned long long hi = ds_bits(c.ds) & 0xFFFFFFFFFFFFull;
      const uint32_t lo = ~c.site;
      if (hi > Thi || (hi == Thi && lo >= Tlo)) {
        const uint32_t i = nsel0 + atomicAdd(&s_nsel, 1u);
        if (i < k) {
          a.sel[i] = c.site;
          a.sel_ds[i] = c.ds;
          reset_site<T, Q, QE, PULL>(a, c.site);
        }
        mn = ds_bits(c.ds) < mn ? ds_bits(c.ds) : mn;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long ox = (unsigned long long)__shfl_xor((long long)mx, off);
    const unsigned long long on = (unsigned long long)__shfl_xor((long long)mn, off);
    mx = ox > mx ? ox : mx;
    mn = on < mn ? on : mn;
  }
  if ((tid & 63) == 0) { s_mx[tid >> 6] = mx; s_mn[tid >> 6] = mn; }
  __syncthreads();
  if (tid == 0) {
    for (int v = 0; v < REF_TX / 64; ++v) {
      mx = s_mx[v] > mx ? s_mx[v] : mx;
      mn = s_mn[v] < mn ? s_mn[v] : mn;
    }
    const uint32_t nsel = k == 0 ? 0u : (nc < k ? nc : k);
    a.st->n_above = nc;
    a.st->n_screened = n;
    a.st->n_sel = nsel;
    a.st->n_invalid = a.ctr[C_INVALID];
    a.st->total_sel += nsel;
    a.st->max = nc ? __longlong_as_double((long long)mx) : 0.0;
    a.st->kth = nsel ? __longlong_as_double((long long)mn) : 0.0;
    a.ctr[C_SCREEN] = 0;
    a.ctr[C_CAND] = 0;
    a.ctr[C_INVALID] = 0;
    a.ctr[C_NSEL0] = 0;
    a.ctr[C_NBND] = 0;
    a.ctr[C_BSTAR] = 0;
    a.ctr[C_R] = 0;
  }
  // clear the histogram for the next step (k_rank fills it, from the
  // candidates only, when more than k sites were screened): the candidates'
  // own bins when they are few, else every bin; and the coarse bins
  if (nc > 0 && k > 0 && n > k) {
    if (n <= HIST_BINS) {
      for (uint32_t t = tid; t < n; t += REF_TX) {
        const double d = a.cand[t].ds;
        if (d >= 0.0) a.hist[ds_bin(d)] = 0;
      }
    } else {
      for (int j = tid; j < HIST_BINS; j += REF_TX) a.hist[j] = 0;
    }
    if (tid < HIST_COARSE) a.hist[HIST_BINS + tid] = 0;
  }
}

// ---------------------------------------------------------------------------
// k_select_one: the whole ranking and selection in one workgroup of 512
// threads (LBM_SELECT_ONE), for small healthy lattices, where each kernel
// boundary costs as much as the work: the same candidates, keys and selected
// set as k_rank + k_partition + k_refine, in one launch instead of three.  The histogram
// lives in LDS (2^15 32-bit counts), the counters in LDS.
// ---------------------------------------------------------------------------
constexpr int ONE_TX = 512;
constexpr int ONE_BINS = HIST_BINS / ONE_TX;  // histogram bins owned by a thread in the b* scan

// workgroup-wide exclusive offset of `flag` over the ONE_TX / 64 waves, base
// from an LDS counter *s_total (no global atomic); s_cnt: ONE_TX / 64 words
__device__ __forceinline__ uint32_t append_one(bool flag, uint32_t* s_total, uint32_t* s_cnt) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const unsigned long long mask = __ballot(flag);
  if (lane == 0) s_cnt[w] = (uint32_t)__popcll(mask);
  __syncthreads();
  uint32_t base = *s_total;
  for (int v = 0; v < w; ++v) base += s_cnt[v];
  const uint32_t slot = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
  __syncthreads();
  if (tid == ONE_TX - 1) {
    uint32_t tot = 0;
    for (int v = 0; v < ONE_TX / 64; ++v) tot += s_cnt[v];
    *s_total += tot;
  }
  __syncthreads();
  return slot;
}

template <typename T, int Q, int QE, bool PULL>
__global__ __launch_bounds__(ONE_TX) void k_select_one(StepArgs a) {
  if (halted(a)) return;
  __shared__ uint32_t s_hist[HIST_BINS];
  __shared__ uint32_t s_cnt[ONE_TX / 64];
  __shared__ uint32_t s_nc, s_ninv, s_nsel, s_nbnd, s_bstar, s_r, s_dig, s_rr, s_exact;
  __shared__ uint32_t s_scan[ONE_TX];
  __shared__ unsigned long long s_mx[ONE_TX / 64], s_mn[ONE_TX / 64];
  const T* __restrict__ A = (const T*)a.A;
  const Geom& g = a.g;
  const int tid = threadIdx.x;
  const uint32_t n = a.ctr[C_SCREEN];
  const uint32_t k = (uint32_t)g.kmax;
  const bool need_hist = k > 0 && n > k;
  if (tid == 0) { s_nc = 0; s_ninv = 0; s_nsel = 0; s_nbnd = 0; s_bstar = 0; s_r = 0; }
  if (need_hist)
    for (int j = tid; j < HIST_BINS; j += ONE_TX) s_hist[j] = 0u;
  __syncthreads();
  // 1. FP64 Delta S of the screened sites (as in k_rank)
  for (uint32_t t0 = 0; t0 < n; t0 += ONE_TX) {
    const uint32_t t = t0 + tid;
    bool is_c = false;
    double ds = 0.0;
    uint32_t site = 0;
    if (t < n) {
      site = a.screen[t];
      ds = rank_site<T, Q, QE, PULL>(a, A, g, site);
      is_c = ds > g.delta;
      // in place, as k_rank writes it (Delta S < 0: not a candidate)
      a.cand[t] = Cand{site, 0u, is_c ? ds : -1.0};
    }
    if (is_c) {
      atomicAdd(&s_nc, 1u);
      if (need_hist) atomicAdd(&s_hist[ds_bin(ds)], 1u);
      if (__builtin_isinf(ds)) atomicAdd(&s_ninv, 1u);
    }
  }
  __syncthreads();
  const uint32_t nc = s_nc;
  const bool all = k == 0 || nc <= k;
  // 2. b* from the histogram (thread t owns the ONE_BINS bins from
  //    HIST_BINS-1-ONE_BINS t down)
  if (!all) {
    uint32_t local = 0;
    for (int j = 0; j < ONE_BINS; ++j) local += s_hist[HIST_BINS - 1 - ONE_BINS * tid - j];
    s_scan[tid] = local;
    __syncthreads();
    for (int off = 1; off < ONE_TX; off <<= 1) {
      const uint32_t v = tid >= off ? s_scan[tid - off] : 0u;
      __syncthreads();
      s_scan[tid] += v;
      __syncthreads();
    }
    const uint32_t incl = s_scan[tid], excl = incl - local;
    if (excl < k && incl >= k) {
      uint32_t c = excl;
      for (int j = 0; j < ONE_BINS; ++j) {
        const uint32_t b = HIST_BINS - 1 - ONE_BINS * tid - j;
        const uint32_t h = s_hist[b];
        if (c + h >= k) { s_bstar = b; s_r = k - c; break; }
        c += h;
      }
    }
    __syncthreads();
  }
  const uint32_t bstar = s_bstar;
  // 3. keys above b* (or all) are selected and reset; keys in b* listed
  unsigned long long mx = 0ull, mn = ~0ull;
  for (uint32_t t0 = 0; t0 < (nc ? n : 0u); t0 += ONE_TX) {
    const uint32_t t = t0 + tid;
    Cand c{0u, 0u, -1.0};
    if (t < n) c = a.cand[t];
    const bool ok = t < n && c.ds >= 0.0;
    const uint32_t bin = ds_bin(c.ds);
    const bool take = ok && k > 0 && (all || bin > bstar);
    const bool bnd = ok && !all && bin == bstar;
    if (ok) mx = ds_bits(c.ds) > mx ? ds_bits(c.ds) : mx;
    if (take) mn = ds_bits(c.ds) < mn ? ds_bits(c.ds) : mn;
    const uint32_t s1 = append_one(take, &s_nsel, s_cnt);
    const uint32_t s2 = append_one(bnd, &s_nbnd, s_cnt);
    if (take) {
      a.sel[s1] = c.site;
      a.sel_ds[s1] = c.ds;
      reset_site<T, Q, QE, PULL>(a, c.site);
    }
    if (bnd) a.bnd[s2] = c;
  }
  __syncthreads();
  // 4. the r largest keys of bin b*: 8-bit radix passes (as in k_refine)
  if (!all) {
    const uint32_t m = s_nbnd;
    unsigned long long Thi = 0, Mhi = 0;
    uint32_t Tlo = 0, Mlo = 0, rr = s_r;
    uint32_t* s_h8 = s_scan;  // 256 digit counts
    for (int pass = 0; pass < 10; ++pass) {
      const bool inhi = pass < 6;
      const int sh = inhi ? 40 - 8 * pass : 24 - 8 * (pass - 6);
      if (tid < 256) s_h8[tid] = 0;
      __syncthreads();
      for (uint32_t t = tid; t < m; t += ONE_TX) {
        const Cand c = a.bnd[t];
        const unsigned long long hi = ds_bits(c.ds) & 0xFFFFFFFFFFFFull;
        const uint32_t lo = ~c.site;
        if ((hi & Mhi) == Thi && (lo & Mlo) == Tlo) {
          const uint32_t d = inhi ? (uint32_t)(hi >> sh) & 255u : (lo >> sh) & 255u;
          atomicAdd(&s_h8[d], 1u);
        }
      }
      __syncthreads();
      if (tid == 0) {
        uint32_t c = 0;
        for (int d = 255; d >= 0; --d) {
          const uint32_t h = s_h8[d];
          if (c + h >= rr) { s_dig = (uint32_t)d; s_rr = rr - c; s_exact = (h == rr - c); break; }
          c += h;
        }
      }
      __syncthreads();
      const uint32_t d = s_dig;
      rr = s_rr;
      if (inhi) { Thi |= (unsigned long long)d << sh; Mhi |= 255ull << sh; }
      else { Tlo |= d << sh; Mlo |= 255u << sh; }
      const bool done = s_exact != 0;
      __syncthreads();
      if (done) break;
    }
    for (uint32_t t = tid; t < m; t += ONE_TX) {
      const Cand c = a.bnd[t];
      const unsigned long long hi = ds_bits(c.ds) & 0xFFFFFFFFFFFFull;
      const uint32_t lo = ~c.site;
      if (hi > Thi || (hi == Thi && lo >= Tlo)) {
        const uint32_t i = atomicAdd(&s_nsel, 1u);  // s_nsel starts at nsel0
        if (i < k) {
          a.sel[i] = c.site;
          a.sel_ds[i] = c.ds;
          reset_site<T, Q, QE, PULL>(a, c.site);
        }
        mn = ds_bits(c.ds) < mn ? ds_bits(c.ds) : mn;
      }
    }
  }
  // 5. statistics; counters cleared for the next step
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long ox = (unsigned long long)__shfl_xor((long long)mx, off);
    const unsigned long long on = (unsigned long long)__shfl_xor((long long)mn, off);
    mx = ox > mx ? ox : mx;
    mn = on < mn ? on : mn;
  }
  if ((tid & 63) == 0) { s_mx[tid >> 6] = mx; s_mn[tid >> 6] = mn; }
  __syncthreads();
  if (tid == 0) {
    for (int v = 0; v < ONE_TX / 64; ++v) {
      mx = s_mx[v] > mx ? s_mx[v] : mx;
      mn = s_mn[v] < mn ? s_mn[v] : mn;
    }
    const uint32_t nsel = k == 0 ? 0u : (nc < k ? nc : k);
    a.st->n_above = nc;
    a.st->n_screened = n;
    a.st->n_sel = nsel;
    a.st->n_invalid = s_ninv;
    a.st->total_sel += nsel;
    a.st->max = nc ? __longlong_as_double((long long)mx) : 0.0;
    a.st->kth = nsel ? __longlong_as_double((long long)mn) : 0.0;
    a.ctr[C_SCREEN] = 0;
  }
}

template <typename T, bool PULL, int START, bool ELBM>
__global__ __launch_bounds__(STEP_TX) void k_fstep(StepArgs s, FstarArgs a) {
  // a workgroup-uniform decision (the halt may be raised meanwhile by
  // another workgroup of this step)
  if (__syncthreads_or(halted(s))) return;
  count_step(s);
  __shared__ SolveAcc sh;
  if (threadIdx.x < sizeof(SolveAcc) / 4) ((uint32_t*)&sh)[threadIdx.x] = 0;
  __syncthreads();
  const T* __restrict__ A = (const T*)s.A;
  const Geom& g = s.g;
  const int64_t N = g.nx * g.ny;
  uint32_t sum32 = 0, sum64 = 0, ninf = 0;
  double maxres = 0.0;
  for (int64_t bb = blockIdx.x; bb < s.nblocks; bb += gridDim.x) {
    const int64_t b = xcd_remap(bb, s.nblocks);
    const int64_t y = b / s.ntx;
    const int64_t x0 = (b - y * s.ntx) * STEP_TX;
    const int64_t x = x0 + threadIdx.x;
    const int64_t i = x + y * g.nx;
    const bool fluid = x < g.nx && !is_solid(g, x, y);
    T f[9];
    load_segment_site<T, 9, PULL>(A, g, x0, x, y, fluid, f);
    const Moments<9, T> m = moments<9, T>(f);
    if (fluid && i == s.probe) probe_sample<9, T>(s, m);
    int it32 = 0, it64 = 0;
    bool scr = false;
    T osum = T(0);
    if (fluid) {
      double fd[9];
      #pragma unroll
      for (int q = 0; q < 9; ++q) fd[q] = (double)f[q];
      const Moments<9, double> md = moments<9, double>(fd);
      const double rho = md.rho, ir = 1.0 / rho, u1 = md.jx * ir, u2 = md.jy * ir, e = md.e2 * ir;
      bool failed = false;
      double st[4];
      solve_site<START>(a, i, rho, u1, u2, e, it32, it64, ninf, maxres, failed, st);
      if (failed) {
        s.Mbuf[i] = md.rho;
        s.Mbuf[N + i] = md.jx;
        s.Mbuf[2 * N + i] = md.jy;
        s.Mbuf[3 * N + i] = md.e2;
        const uint32_t slot = atomicAdd(&a.ctr[0], 1u);
        a.fail_list[slot] = (uint32_t)i;
      } else {
        T fs[9];
        fstar_pop<T>((T)st[0], (T)st[1], (T)st[2], (T)st[3], fs);
        if (g.ds_on) scr = screen_entropic<9, T>(s, f, fs, m.rho);
        osum = collide_store<T, 9, ELBM>(s, x, y, f, fs);
      }
      sum32 += (uint32_t)it32;
      sum64 += (uint32_t)it64;
    }
    solve_hist(sh, fluid, it32 + it64);
    append_screened<PULL>(s, scr, (uint32_t)i,
                          fluid && !(__builtin_isfinite(m.rho) && __builtin_isfinite(osum)));
  }
  solve_flush(a, sh, sum32, sum64, ninf, maxres);
}

// the sites listed by k_fstep: FP64 damped Newton from the rest start on
// their moments, then the same screen and collision (f(x, t) pulled again)
template <typename T, bool PULL, bool ELBM>
__global__ __launch_bounds__(64) void k_fstep_fallback(StepArgs s, FstarArgs a) {
  if (halted(s)) return;  // single-wave workgroups: no barrier to keep
  const uint32_t nf = a.ctr[0];
  const int64_t n = a.n;
  const Geom& g = s.g;
  for (uint32_t t = blockIdx.x * 64u + threadIdx.x; t < nf; t += gridDim.x * 64u) {
    const int64_t i = a.fail_list[t];
    const double rho = a.M[i], u1 = a.M[n + i] / rho, u2 = a.M[2 * n + i] / rho, e = a.M[3 * n + i] / rho;
    FS<double> q;
    double res = 0.0;
    const int it = newton64_damped(u1, u2, e, a.tol, 200, q, res);
    if (it >= 0 && a.polish) res = polish_once(q, u1, u2, e);
    write_mu(a, i, rho, q);
    if (a.status) a.status[i] = it >= 0 ? 1 : 3;
    FstarStats& S = stat_slot(a.stats);
    atomicAdd(&S.fallback, 1ull);
    if (it < 0) atomicAdd(&S.failed, 1ull);
    else atomicMax(&S.maxres_bits, (unsigned long long)__double_as_longlong(res));

    int64_t x, y;
    divmod((int64_t)i, g.nx, g.inv_nx, y, x);
    T f[9], fs[9];
    load_site<T, 9, PULL>((const T*)s.A, g, x, y, f);
    fstar_pop<T>((T)(q.a * rho), (T)q.X, (T)q.Y, (T)q.Z, fs);
    const Moments<9, T> m = moments<9, T>(f);
    if (g.ds_on && screen_entropic<9, T>(s, f, fs, m.rho)) s.screen[atomicAdd(&s.ctr[C_SCREEN], 1u)] = (uint32_t)i;
    const T osum = collide_store<T, 9, ELBM>(s, x, y, f, fs);
    if (!(__builtin_isfinite(m.rho) && __builtin_isfinite(osum))) raise_nonfinite<PULL>(s);
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// ranking, selection and reset of the screened sites
template <typename T, int Q, int QE, bool PULL>
static void select_t(const StepArgs& a, hipStream_t s) {
  if (a.g.ds_on && a.one_wg) {
    hipLaunchKernelGGL((k_select_one<T, Q, QE, PULL>), dim3(1), dim3(ONE_TX), 0, s, a);
  } else if (a.g.ds_on) {
    if constexpr (QE == QE_ENTROPIC_M)
      hipLaunchKernelGGL((k_rank_m<T, Q, QE, PULL>), dim3(RANK_BLOCKS), dim3(RANK_TX), 0, s, a);
    else
      hipLaunchKernelGGL((k_rank<T, Q, QE, PULL>), dim3(RANK_BLOCKS), dim3(RANK_TX), 0, s, a);
    hipLaunchKernelGGL((k_partition<T, Q, QE, PULL>), dim3(PART_BLOCKS), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_refine<T, Q, QE, PULL>), dim3(1), dim3(REF_TX), 0, s, a);
  }
}

template <typename T, int Q, int QE, bool PULL>
static hipError_t step_t(const StepArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0) { hipError_t e = hipEventRecord(ev0, s); if (e != hipSuccess) return e; }
  if (QE != QE_POLY && a.coll == 1)
    hipLaunchKernelGGL((k_step<T, Q, QE, PULL, QE != QE_POLY>), dim3((unsigned)a.nblocks), dim3(STEP_TX), 0, s, a);
  else
    hipLaunchKernelGGL((k_step<T, Q, QE, PULL>), dim3((unsigned)a.nblocks), dim3(STEP_TX), 0, s, a);
  if (ev1) { hipError_t e = hipEventRecord(ev1, s); if (e != hipSuccess) return e; }
  select_t<T, Q, QE, PULL>(a, s);
  return hipGetLastError();
}

template <typename T, int Q, int QE>
static hipError_t step_p(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return pull ? step_t<T, Q, QE, true>(a, s, e0, e1) : step_t<T, Q, QE, false>(a, s, e0, e1);
}

template <typename T, int Q>
static hipError_t step_q(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (a.qe == QE_POLY) return step_p<T, Q, QE_POLY>(a, pull, s, e0, e1);
  if (a.qe == QE_ENTROPIC_MM) return step_p<T, Q, QE_ENTROPIC_MM>(a, pull, s, e0, e1);
  if constexpr (Q == 9) return step_p<T, 9, QE_ENTROPIC_M>(a, pull, s, e0, e1);
  return hipErrorInvalidValue;
}

template <typename T, bool PULL, bool ELBM>
static hipError_t fstep_t(const StepArgs& a, const FstarArgs& fa, int start, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1) {
  // a grid-stride loop over the row segments by the workgroups the device
  // holds at once (one round, no partly filled last round; the statistics
  // atomics stay few), else by at most FSTAR_MAX_BLOCKS
  const int64_t cap = a.fgrid[PULL ? 1 : 0] > 0 ? a.fgrid[PULL ? 1 : 0] : FSTAR_MAX_BLOCKS;
  const unsigned gr = (unsigned)(a.nblocks < cap ? a.nblocks : cap);
  if (ev0) { hipError_t e = hipEventRecord(ev0, s); if (e != hipSuccess) return e; }
  if (start == START_CLOSED) hipLaunchKernelGGL((k_fstep<T, PULL, START_CLOSED, ELBM>), dim3(gr), dim3(STEP_TX), 0, s, a, fa);
  else if (start == START_PREV) hipLaunchKernelGGL((k_fstep<T, PULL, START_PREV, ELBM>), dim3(gr), dim3(STEP_TX), 0, s, a, fa);
  else hipLaunchKernelGGL((k_fstep<T, PULL, START_REST, ELBM>), dim3(gr), dim3(STEP_TX), 0, s, a, fa);
  if (ev1) { hipError_t e = hipEventRecord(ev1, s); if (e != hipSuccess) return e; }
  hipLaunchKernelGGL((k_fstep_fallback<T, PULL, ELBM>), dim3(64), dim3(64), 0, s, a, fa);
  select_t<T, 9, QE_ENTROPIC_M, PULL>(a, s);
  return hipGetLastError();
}

// workgroups of k_fstep<T, PULL, START, ELBM> resident at once on the
// current device: its occupancy per compute unit times the compute units
template <typename T, bool PULL, int START, bool ELBM>
static int fstep_resident_t() {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_fstep<T, PULL, START, ELBM>),
                                                   STEP_TX, 0) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu > 0 && cus > 0 ? per_cu * cus : 0;
}

template <typename T, bool PULL, bool ELBM>
static int fstep_resident_s(int start) {
  if (start == START_CLOSED) return fstep_resident_t<T, PULL, START_CLOSED, ELBM>();
  if (start == START_PREV) return fstep_resident_t<T, PULL, START_PREV, ELBM>();
  return fstep_resident_t<T, PULL, START_REST, ELBM>();
}

template <typename T>
static int fstep_resident_p(int start, bool pull, bool elbm) {
  if (pull) return elbm ? fstep_resident_s<T, true, true>(start) : fstep_resident_s<T, true, false>(start);
  return elbm ? fstep_resident_s<T, false, true>(start) : fstep_resident_s<T, false, false>(start);
}

template <typename T, bool PULL>
static hipError_t fstep_p(const StepArgs& a, const FstarArgs& fa, int start, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1) {
  return a.coll == 1 ? fstep_t<T, PULL, true>(a, fa, start, s, ev0, ev1)
                     : fstep_t<T, PULL, false>(a, fa, start, s, ev0, ev1);
}

// per-translation-unit instantiations (lbm_step_*.hip, lbm_fstep_*.hip)
hipError_t launch_step_f32q9(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_step_f32q3(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_step_f64q9(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_step_f64q3(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_fstep_f32(const StepArgs& a, const FstarArgs& fa, int start, bool pull, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1);
int fstep_resident_f32(int start, bool pull, bool elbm);
int fstep_resident_f64(int start, bool pull, bool elbm);
hipError_t launch_fstep_f64(const StepArgs& a, const FstarArgs& fa, int start, bool pull, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1);

}  // namespace lbm
