// lbm_device.hpp -- device-side lattice tables and per-site arithmetic of the
// Ehrenfests'-step regularised LBGK step (gfx950).
//
// Velocity numbering follows the paper: D1Q3 (rest, left, right), Sec. 4.1;
// D2Q9 (rest, E, N, W, S, NE, NW, SW, SE), Sec. 4.2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// 1/x in FP64 for finite normal x: the hardware estimate refined by two
// Newton steps r <- r + r (1 - x r) (error ~2^-26 -> 2^-52 -> round-off),
// instead of the full IEEE division sequence
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// ---------------------------------------------------------------------------
// Lattice tables
// ---------------------------------------------------------------------------
template <int Q> struct Lat;

template <> struct Lat<9> {
  static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  // opposite velocity (bounce-back) and vertical mirror (free-slip)
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  static constexpr int mir[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};
  // weights 4/9, 1/9, 1/36 (Sec. 4.2)
  static __host__ __device__ constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

template <> struct Lat<3> {
  static constexpr int cx[3] = {0, -1, 1};
  static constexpr int cy[3] = {0, 0, 0};
  static constexpr int opp[3] = {0, 2, 1};
  static constexpr int mir[3] = {0, 1, 2};
  // weights 2/3, 1/6, 1/6 (Sec. 4.1)
  static __host__ __device__ constexpr double w(int i) { return i == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
};

enum : int { BC_PERIODIC = 0, BC_ZEROGRAD = 1, BC_FREESLIP = 2, BC_INLET_EQ = 3, BC_OUTLET_EQ = 4,
             BC_OUTLET_EQ_PREV = 5 };
enum : int { QE_POLY = 0, QE_ENTROPIC_MM = 1, QE_ENTROPIC_M = 2 };

// Geometry and per-step parameters passed by value to every step kernel.
struct Geom {
  int64_t nx, ny, pitch, plane;  // pitch = nx rounded up to 64; plane = pitch * ny elements
  int32_t bc[4];                 // west, east, south, north
  int64_t sx0, sy0, sx1, sy1;    // solid square [sx0, sx1) x [sy0, sy1); empty if sx1 <= sx0
  double feq_in[9];              // inlet quasiequilibrium (FP64; cast at use)
  double beta2;                  // 2 beta
  double delta;                  // Ehrenfests' tolerance
  int32_t ds_on;                 // 0 when delta = +inf: no Delta S work at all
  int32_t kmax;                  // k
  int32_t out_qe;                // outlet quasiequilibrium: QE_POLY or QE_ENTROPIC_MM
  int32_t pad0;
  double inv_nx, inv_pitch;      // 1 / nx, 1 / pitch (site index -> coordinates)
};

// q = floor(s / d) and r = s - q d for 0 <= s < 2^40 and 0 < d < 2^32: the
// quotient from the FP64 reciprocal (its error, below 2^-50 s / d < 1e-5,
// moves it by at most one) corrected by one step either way; a 64-bit
// integer division would take a long instruction sequence per site
__device__ __forceinline__ void divmod(int64_t s, int64_t d, double inv_d, int64_t& q, int64_t& r) {
  q = (int64_t)((double)s * inv_d);
  r = s - q * d;
  if (r < 0) {
    --q;
    r += d;
  } else if (r >= d) {
    ++q;
    r -= d;
  }
}

// State layout: tiles of 64 sites of one row.  Population i of site (x, y)
// lives at ((y * (pitch / 64) + x / 64) * Q + i) * 64 + x % 64, so a
// wavefront's 64 sites read each population as one contiguous run and the Q
// runs of a tile are adjacent (fewer concurrent DRAM streams than Q separate
// planes).  x must lie in [0, pitch).
template <int Q>
__device__ __forceinline__ int64_t sidx(const Geom& g, int64_t x, int64_t y, int i) {
  return ((y * (g.pitch >> 6) + (x >> 6)) * Q + i) * 64 + (x & 63);
}

// Row-relative addressing of the same layout: a row of tiles holds
// pitch * Q elements (below 2^32 bytes, since nx <= 2^25), so a site's
// populations sit at a per-row base (uniform over a workgroup that covers
// part of one row) plus a 32-bit byte offset per column plus 64 * i elements.
template <typename T, int Q>
__device__ __forceinline__ uint32_t col_bytes(int64_t x) {
  const uint32_t xx = (uint32_t)x;
  return ((xx >> 6) * (uint32_t)(Q * 64) + (xx & 63u)) * (uint32_t)sizeof(T);
}

__device__ __forceinline__ bool is_solid(const Geom& g, int64_t x, int64_t y) {
  return x >= g.sx0 && x < g.sx1 && y >= g.sy0 && y < g.sy1;
}

// ---------------------------------------------------------------------------
// Moments and quasiequilibria (evaluated in T = float or double)
// ---------------------------------------------------------------------------
template <int Q, typename T> struct Moments {
  T rho, jx, jy, e2;
};

template <int Q, typename T>
__device__ __forceinline__ Moments<Q, T> moments(const T* f) {
  Moments<Q, T> m;
  if constexpr (Q == 9) {
    // fixed summation order i = 0..8
    m.rho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    m.jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    m.jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    m.e2 = (f[1] + f[2] + f[3] + f[4]) + T(2) * (f[5] + f[6] + f[7] + f[8]);
  } else {
    m.rho = f[0] + f[1] + f[2];
    m.jx = f[2] - f[1];
    m.jy = T(0);
    m.e2 = f[1] + f[2];
  }
  return m;
}

// Polynomial quasiequilibrium.  D1Q3: Sec. 4.1's formulas.  D2Q9: the
// second-order polynomial W_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u) of the
// LBGK literature the paper cites for it.  Written as f*_i = W_i rho p_i;
// the brackets p_i are returned for the Delta S screen.
template <int Q, typename T>
__device__ __forceinline__ void qe_poly_br(T rho, T ux, T uy, T* fs, T* p) {
  if constexpr (Q == 9) {
    const T uu = ux * ux + uy * uy;
    const T base = T(1) - T(1.5) * uu;  // 1 - 3/2 u.u
    const T r0 = rho * T(4.0 / 9.0), r1 = rho * T(1.0 / 9.0), r2 = rho * T(1.0 / 36.0);
    p[0] = base;
    // axis velocities: c.u = +-ux, +-uy
    const T ax = base + T(4.5) * ux * ux, ay = base + T(4.5) * uy * uy;
    p[1] = ax + T(3) * ux;
    p[3] = ax - T(3) * ux;
    p[2] = ay + T(3) * uy;
    p[4] = ay - T(3) * uy;
    // diagonals: c.u = +-(ux + uy), +-(ux - uy)
    const T a = ux + uy, b = ux - uy;
    const T dp = base + T(4.5) * a * a, dq = base + T(4.5) * b * b;
    p[5] = dp + T(3) * a;  // NE  (+1,+1)
    p[7] = dp - T(3) * a;  // SW  (-1,-1)
    p[8] = dq + T(3) * b;  // SE  (+1,-1)
    p[6] = dq - T(3) * b;  // NW  (-1,+1)
    fs[0] = r0 * p[0];
    #pragma unroll
    for (int i = 1; i < 5; ++i) fs[i] = r1 * p[i];
    #pragma unroll
    for (int i = 5; i < 9; ++i) fs[i] = r2 * p[i];
  } else {
    const T u = ux;
    p[0] = T(1) - T(1.5) * u * u;
    p[1] = T(1) - T(3) * u + T(3) * u * u;
    p[2] = T(1) + T(3) * u + T(3) * u * u;
    fs[0] = (T(2) * rho / T(3)) * p[0];
    fs[1] = (rho / T(6)) * p[1];
    fs[2] = (rho / T(6)) * p[2];
  }
}

template <int Q, typename T>
__device__ __forceinline__ void qe_poly(T rho, T ux, T uy, T* fs) {
  T p[Q];
  qe_poly_br<Q, T>(rho, ux, uy, fs, p);
}

// Entropic quasiequilibrium with mass and momentum constraints, closed
// form: D2Q9 product formula of Sec. 4.2; D1Q3 its 1-D factor (Sec. 4.1's
// explicit formulas with the right-hand sides of f2 and f3 in the order that
// reproduces +rho u).
template <typename T> __device__ __forceinline__ T dsqrt(T x) {
  if constexpr (sizeof(T) == 4) return __builtin_sqrtf(x);
  else return __builtin_sqrt(x);
}

template <int Q, typename T>
__device__ __forceinline__ void qe_entropic_mm(T rho, T ux, T uy, T* fs) {
  const T sx = dsqrt(T(1) + T(3) * ux * ux);
  const T ax = T(2) - sx;                      // weight factor of the rest component
  const T bx = (T(2) * ux + sx) / (T(1) - ux);  // X = factor of a +1 component
  if constexpr (Q == 3) {
    // rho (2/3, 1/6, 1/6) * (2 - s) * X^{v}
    const T base = rho * ax;
    fs[0] = base * T(2.0 / 3.0);
    fs[1] = base * T(1.0 / 6.0) / bx;
    fs[2] = base * T(1.0 / 6.0) * bx;
  } else {
    const T sy = dsqrt(T(1) + T(3) * uy * uy);
    const T ay = T(2) - sy;
    const T by = (T(2) * uy + sy) / (T(1) - uy);
    const T ibx = T(1) / bx, iby = T(1) / by;
    const T base = rho * ax * ay;
    const T b1 = base * T(1.0 / 9.0), b2 = base * T(1.0 / 36.0);
    fs[0] = base * T(4.0 / 9.0);
    fs[1] = b1 * bx;
    fs[3] = b1 * ibx;
    fs[2] = b1 * by;
    fs[4] = b1 * iby;
    fs[5] = b2 * bx * by;
    fs[6] = b2 * ibx * by;
    fs[7] = b2 * ibx * iby;
    fs[8] = b2 * bx * iby;
  }
}

template <typename T> __device__ __forceinline__ T inv_of(T x) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(x);
  else return T(1) / x;
}

template <int Q, int QE, typename T>
__device__ __forceinline__ void qe_eval(const Moments<Q, T>& m, T* fs) {
  const T inv = inv_of(m.rho);
  const T ux = m.jx * inv, uy = m.jy * inv;
  if constexpr (QE == QE_POLY) qe_poly<Q, T>(m.rho, ux, uy, fs);
  else qe_entropic_mm<Q, T>(m.rho, ux, uy, fs);
}

// ---------------------------------------------------------------------------
// Nonequilibrium entropy
// ---------------------------------------------------------------------------
// Per population, with s = (f - f*)/(f + f*), sigma = f + f*:
//   f ln(f/f*) - f + f* = sigma s^2 [1 + s (1 + s) G(s^2)],
//   G(t) = sum_{j >= 0} t^j / (2j + 3)
// (from the series of artanh; every term is non-negative, no cancellation).

// FP32 screen: returns a value that is >= Delta S (1 - 2e-3) up to FP32
// rounding for sites with every |s| <= 1/2, and +inf when some |s| > 1/2,
// some f < 0, f* <= 0, or a value is not finite.  The caller re-evaluates
// screened sites in FP64.
template <int Q>
__device__ __forceinline__ float dS_screen(const float* f, const float* fs) {
  float acc = 0.0f;
  bool wild = false;
  #pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float a = f[i], b = fs[i];
    const float d = a - b, sg = a + b;
    const float s = d * __builtin_amdgcn_rcpf(sg);
    const float t = s * s;
    const float h = 1.0f + (s + t) * (1.0f / 3.0f + t * (0.2f + t * (1.0f / 7.0f)));
    acc += (d * s) * h;
    wild |= !(a >= 0.0f) | !(b > 0.0f) | !(__builtin_fabsf(s) <= 0.5f);
  }
  return wild ? __builtin_inff() : acc;
}

// FP32 screen for the polynomial quasiequilibrium f*_i = W_i rho p_i, free
// of reciprocals: with a = f_i, b = f*_i > 0, a ln(a/b) - a + b <= (a-b)^2/b
// (from ln x <= x - 1), and 1/p <= 2p^2 - 5p + 4 for p in [1/2, 3/2], so
//   Delta S <= (1/rho) sum_i (f_i - f*_i)^2 (2 p_i^2 - 5 p_i + 4) / W_i.
// Returns +inf when some f_i < 0, some p_i is outside [1/2, 3/2] (this
// includes f*_i <= 0), or a value is not finite.
template <int Q>
__device__ __forceinline__ float dS_bound_poly(const float* f, const float* fs, const float* p, float inv_rho) {
  float acc = 0.0f;
  float fmin = f[0], pmin = p[0], pmax = p[0];
  #pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float d = f[i] - fs[i];
    const float q = __builtin_fmaf(p[i], __builtin_fmaf(2.0f, p[i], -5.0f), 4.0f);
    acc = __builtin_fmaf(d * d * (float)(1.0 / Lat<Q>::w(i)), q, acc);
    if (i > 0) {
      fmin = fminf(fmin, f[i]);
      pmin = fminf(pmin, p[i]);
      pmax = fmaxf(pmax, p[i]);
    }
  }
  const float u = acc * inv_rho;
  const bool ok = fmin >= 0.0f && pmin >= 0.5f && pmax <= 1.5f && u <= 3.0e38f;
  return ok ? u : __builtin_inff();
}

// ELBM (eq. (elbmLB)): alpha is the nontrivial root of
// S(f + alpha (f* - f)) = S(f), by bisection to 1e-15.  For an entropic f*
// with the conserved moments of f the entropy difference equals, exactly,
//   H(a) = sum_i f_i [a x_i ln(1 + x_i) - phi(a x_i)],  x_i = f*_i / f_i - 1,
//   phi(y) = (1 + y) ln(1 + y) - y,
// a form free of cancellation (every term is O(x^2)); phi by its Taylor
// series sum_{k>=2} (-1)^k y^k / (k (k-1)) for |y| < 0.1.  The root lies in
// (1, a_max], a_max keeping every population >= 0 (capped at 1000); a site
// with some f_i <= 0 or f*_i <= 0, or with f = f*, takes a = 2.
__device__ __forceinline__ double elbm_phi(double y) {
  if (__builtin_fabs(y) < 0.1) {
    // Horner on y^2 sum_{k=2}^{19} c_k y^(k-2), c_k = (-1)^k / (k (k-1))
    double s = -1.0 / (19.0 * 18.0);
    #pragma unroll
    for (int k = 18; k >= 2; --k) s = s * y + ((k & 1) ? -1.0 : 1.0) / (double)(k * (k - 1));
    return s * y * y;
  }
  return (1.0 + y) * ::log1p(y) - y;
}

template <int Q>
__device__ __forceinline__ double elbm_alpha(const double* f, const double* fs) {
  double x[Q], px[Q];
  double amax = 1000.0;
  bool moving = false;
  #pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (!(f[i] > 0.0) || !(fs[i] > 0.0)) return 2.0;
    x[i] = fs[i] / f[i] - 1.0;
    px[i] = f[i] * x[i] * ::log1p(x[i]);  // f psi(x)
    moving |= x[i] != 0.0;
    if (x[i] < 0.0) amax = fmin(amax, -1.0 / x[i]);
  }
  if (!moving) return 2.0;
  auto H = [&](double a) {
    double h = 0.0;
    #pragma unroll
    for (int i = 0; i < Q; ++i) h += a * px[i] - f[i] * elbm_phi(a * x[i]);
    return h;
  };
  double lo = 1.0, hi = amax;
  if (H(hi) >= 0.0) return hi;
  for (int it = 0; it < 80 && hi - lo > 1e-15; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (H(mid) > 0.0) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// FP64 Delta S (Sec. 3.3 Kullback form, generalised by -f + f* so that it
// stays >= 0 when masses differ by round-off); +inf for f < 0 or f* <= 0.
// Per population, for |s| <= 1/16 (t <= 2^-8) the series of G is cut after
// t^6: the first term dropped, t^7 / 17 <= 2^-56 / 17, is < 1e-17 of G's
// leading 1/3 and enters the bracket multiplied by |s (1 + s)| < 0.07; 14
// terms for |s| <= 1/4; the logarithm beyond.
//
// The bracket sg t (1 + s (1 + s) G(t)) of one population, with G cut after
// t^6 (short) or t^13 (long):
template <bool LONG>
__device__ __forceinline__ double dS_series(double sg, double s) {
  const double t = s * s;
  double G;
  if constexpr (LONG) {
    G = 1.0 / 29.0;
    G = G * t + 1.0 / 27.0;
    G = G * t + 1.0 / 25.0;
    G = G * t + 1.0 / 23.0;
    G = G * t + 1.0 / 21.0;
    G = G * t + 1.0 / 19.0;
    G = G * t + 1.0 / 17.0;
    G = G * t + 1.0 / 15.0;
  } else {
    G = 1.0 / 15.0;
  }
  G = G * t + 1.0 / 13.0;
  G = G * t + 1.0 / 11.0;
  G = G * t + 1.0 / 9.0;
  G = G * t + 1.0 / 7.0;
  G = G * t + 1.0 / 5.0;
  G = G * t + 1.0 / 3.0;
  return sg * t * (1.0 + s * (1.0 + s) * G);
}

// Delta S of one site.  The order of the series is chosen per population
// for the whole wavefront: when every active lane's s lies within 1/16 (or
// 1/4) the wavefront evaluates the short (or long) series, each accurate to
// round-off wherever it is used, as one straight-line sequence instead of
// every branch that some lane needs; otherwise each lane takes its own form
// (series by its own |s|, or the logarithm).
template <int Q>
__device__ __forceinline__ double dS_fp64(const double* f, const double* fs) {
  double acc = 0.0;
  bool bad = false;
  #pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double a = f[i], b = fs[i];
    const double sg = a + b, s = (a - b) * rcp64(sg);
    const double as = __builtin_fabs(s);
    const bool pos = a > 0.0 && b > 0.0;  // false for a NaN
    if (__all(pos && as <= 0.0625)) {
      acc += dS_series<false>(sg, s);
    } else if (__all(pos && as <= 0.25)) {
      acc += dS_series<true>(sg, s);
    } else if (!(a >= 0.0) || !(b > 0.0)) {
      bad = true;
    } else if (a == 0.0) {
      acc += b;
    } else if (as <= 0.0625) {
      acc += dS_series<false>(sg, s);
    } else if (as <= 0.25) {
      acc += dS_series<true>(sg, s);
    } else {
      acc += a * ::log(a / b) - a + b;
    }
  }
  return bad ? __builtin_inf() : acc;
}

}  // namespace lbm
