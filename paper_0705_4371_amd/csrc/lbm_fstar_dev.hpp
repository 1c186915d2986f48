// lbm_fstar_dev.hpp -- device helpers of the f*_M Newton iteration in the
// product form f*_i = A g(vx_i) g(vy_i), g(0) = 1, g(+-1) = Z X^{+-1}
// (Y for the y factor), shared by the solver and the time-step kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"

namespace lbm {

template <typename T> struct FS {
  T a, X, Y, Z;  // a = A / rho
};

// gradient g = m(f)/rho - M/rho and Hessian (upper triangle, row-major
// 00 01 02 03 11 12 13 22 23 33) of the dual, scaled by 1/rho
template <typename T>
__device__ __forceinline__ void fsys(const FS<T>& s, T u1, T u2, T e, T* g, T* H) {
  T ix, iy;
  if constexpr (sizeof(T) == 4) { ix = __builtin_amdgcn_rcpf(s.X); iy = __builtin_amdgcn_rcpf(s.Y); }
  else { ix = rcp64(s.X); iy = rcp64(s.Y); }
  const T qx = s.Z * (s.X + ix), px = s.Z * (s.X - ix), nx = T(1) + qx;
  const T qy = s.Z * (s.Y + iy), py = s.Z * (s.Y - iy), ny = T(1) + qy;
  const T a = s.a;
  const T r = a * nx * ny, jx = a * px * ny, jy = a * nx * py;
  const T ee = a * (qx * ny + nx * qy);
  g[0] = r - T(1);
  g[1] = jx - u1;
  g[2] = jy - u2;
  g[3] = ee - e;
  H[0] = r;
  H[1] = jx;
  H[2] = jy;
  H[3] = ee;
  H[4] = a * qx * ny;
  H[5] = a * px * py;
  H[6] = a * px * (ny + qy);
  H[7] = a * nx * qy;
  H[8] = a * py * (nx + qx);
  H[9] = a * (qx * ny + T(2) * qx * qy + nx * qy);
}

// the gradient alone (the convergence test)
template <typename T>
__device__ __forceinline__ void fsys_grad(const FS<T>& s, T u1, T u2, T e, T* g) {
  T ix, iy;
  if constexpr (sizeof(T) == 4) { ix = __builtin_amdgcn_rcpf(s.X); iy = __builtin_amdgcn_rcpf(s.Y); }
  else { ix = rcp64(s.X); iy = rcp64(s.Y); }
  const T qx = s.Z * (s.X + ix), px = s.Z * (s.X - ix), nx = T(1) + qx;
  const T qy = s.Z * (s.Y + iy), py = s.Z * (s.Y - iy), ny = T(1) + qy;
  const T a = s.a;
  g[0] = a * nx * ny - T(1);
  g[1] = a * px * ny - u1;
  g[2] = a * nx * py - u2;
  g[3] = a * (qx * ny + nx * qy) - e;
}

template <typename T> __device__ __forceinline__ T recip(T x) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(x);
  else return rcp64(x);
}

// solve H d = -g (H symmetric positive definite) by LDL^T
template <typename T>
__device__ __forceinline__ void fsolve(const T* H, const T* g, T* d) {
  const T D0 = H[0], i0 = recip(D0);
  const T l10 = H[1] * i0, l20 = H[2] * i0, l30 = H[3] * i0;
  const T D1 = H[4] - l10 * H[1], i1 = recip(D1);
  const T l21 = (H[5] - l20 * H[1]) * i1, l31 = (H[6] - l30 * H[1]) * i1;
  const T D2 = H[7] - l20 * H[2] - l21 * l21 * D1, i2 = recip(D2);
  const T l32 = (H[8] - l30 * H[2] - l31 * l21 * D1) * i2;
  const T D3 = H[9] - l30 * H[3] - l31 * l31 * D1 - l32 * l32 * D2, i3 = recip(D3);
  // L y = -g
  const T y0 = -g[0];
  const T y1 = -g[1] - l10 * y0;
  const T y2 = -g[2] - l20 * y0 - l21 * y1;
  const T y3 = -g[3] - l30 * y0 - l31 * y1 - l32 * y2;
  // D L^T d = y
  d[3] = y3 * i3;
  d[2] = y2 * i2 - l32 * d[3];
  d[1] = y1 * i1 - l21 * d[2] - l31 * d[3];
  d[0] = y0 * i0 - l10 * d[1] - l20 * d[2] - l30 * d[3];
}

template <typename T> __device__ __forceinline__ T resid(const T* g) {
  T r = __builtin_fabs(g[0]);
  r = fmax(r, (T)__builtin_fabs(g[1]));
  r = fmax(r, (T)__builtin_fabs(g[2]));
  r = fmax(r, (T)__builtin_fabs(g[3]));
  return r;
}

// exp(d) for the FP64 phase: Taylor polynomial when |d| < 1e-3 (truncation
// d^5/120 < 1e-17), the library exp otherwise
__device__ __forceinline__ double exp_step(double d) {
  if (__builtin_fabs(d) < 1e-3)
    return 1.0 + d * (1.0 + 0.5 * d * (1.0 + (1.0 / 3.0) * d * (1.0 + 0.25 * d)));
  return ::exp(d);
}

__device__ __forceinline__ bool feasible(double rho, double u1, double u2, double e) {
  return rho > 0.0 && e > __builtin_fabs(u1) + __builtin_fabs(u2) && e < 2.0;
}

// closed-form mass-momentum start (Sec. 4.2): Z = 1/4,
// X = (2u + sqrt(1 + 3u^2)) / (1 - u), a = (4/9)(2 - s_x)(2 - s_y)
template <typename T>
__device__ __forceinline__ FS<T> closed_form(T u1, T u2) {
  const T sx = sqrt(T(1) + T(3) * u1 * u1), sy = sqrt(T(1) + T(3) * u2 * u2);
  FS<T> s;
  s.a = T(4.0 / 9.0) * (T(2) - sx) * (T(2) - sy);
  s.X = (T(2) * u1 + sx) / (T(1) - u1);
  s.Y = (T(2) * u2 + sy) / (T(1) - u2);
  s.Z = T(0.25);
  return s;
}


// Newton polish in FP64 from the product-form state s (a = A / rho) for
// moments M: `iters` undamped steps, for the ranking of screened sites
__device__ __forceinline__ FS<double> polish64(FS<double> s, double u1, double u2, double e, int iters) {
  double g[4], H[10], d[4];
  for (int it = 0; it < iters; ++it) {
    fsys<double>(s, u1, u2, e, g, H);
    if (resid(g) < 1e-15) break;
    fsolve<double>(H, g, d);
    s.a *= exp_step(d[0]);
    s.X *= exp_step(d[1]);
    s.Y *= exp_step(d[2]);
    s.Z *= exp_step(d[3]);
  }
  return s;
}

// One more undamped FP64 Newton update from a converged state: from a
// residual <= 1e-10 the update leaves ~1e-20 in exact arithmetic, so the
// maximiser of Sec. 2 is reached to FP64 round-off.  Returns the residual
// at the updated state.
__device__ __forceinline__ double polish_once(FS<double>& s, double u1, double u2, double e) {
  double g[4], H[10], d[4];
  fsys<double>(s, u1, u2, e, g, H);
  fsolve<double>(H, g, d);
  s.a *= exp_step(d[0]);
  s.X *= exp_step(d[1]);
  s.Y *= exp_step(d[2]);
  s.Z *= exp_step(d[3]);
  fsys_grad<double>(s, u1, u2, e, g);
  return resid(g);
}

// f*_i = rho a g(vx) g(vy) on D2Q9 (paper numbering) from the product-form state
template <typename T>
__device__ __forceinline__ void fstar_pop(T rho_a, T X, T Y, T Z, T* fs) {
  const T ix = T(1) / X, iy = T(1) / Y;
  const T gxp = Z * X, gxm = Z * ix, gyp = Z * Y, gym = Z * iy;
  fs[0] = rho_a;
  fs[1] = rho_a * gxp;
  fs[2] = rho_a * gyp;
  fs[3] = rho_a * gxm;
  fs[4] = rho_a * gym;
  fs[5] = rho_a * gxp * gyp;
  fs[6] = rho_a * gxm * gyp;
  fs[7] = rho_a * gxm * gym;
  fs[8] = rho_a * gxp * gym;
}

}  // namespace lbm
