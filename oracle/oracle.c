/*
 * oracle.c -- plain FP64 CPU reference (see oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  Written for a
 * reader who checks it against the paper by eye: one site at a time, in
 * site-index order, no blocking, no fusion.
 *
 * Parity pins for every function live in tests/test_oracle_*.py.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Velocity sets and weights                                                */
/* ------------------------------------------------------------------------ */

/*
 * D1Q3 (Sec. 4.1): velocities {0, -1, +1}; f1 static, f2 left-moving,
 * f3 right-moving.  Weights 2/3, 1/6, 1/6: the polynomial quasiequilibrium
 * of Sec. 4.1 at u = 0, and the 4:1:1 weights inside the entropy H of the
 * same section.
 *
 * D2Q9 (Sec. 4.2): v_0 = 0; v_i = (cos((i-1) pi/2), sin((i-1) pi/2)) for
 * i = 1..4; v_i = sqrt(2) (cos((i-5) pi/2 + pi/4), sin(...)) for i = 5..8.
 * The integer components are obtained by evaluating that formula and
 * rounding.  Weights W_0 = 4/9, W_1..4 = 1/9, W_5..8 = 1/36 (Sec. 4.2).
 */
int or_velocities(int Q, int32_t* vx, int32_t* vy, double* w)
{
  if (Q == 3) {
    const int32_t v[3] = {0, -1, 1};
    const double W[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
    for (int i = 0; i < 3; ++i) {
      vx[i] = v[i];
      vy[i] = 0;
      w[i] = W[i];
    }
    return 0;
  }
  if (Q == 9) {
    const double pi = 3.14159265358979323846;
    vx[0] = 0;
    vy[0] = 0;
    w[0] = 4.0 / 9.0;
    for (int i = 1; i <= 4; ++i) {
      double a = (i - 1) * pi / 2.0;
      vx[i] = (int32_t)lround(cos(a));
      vy[i] = (int32_t)lround(sin(a));
      w[i] = 1.0 / 9.0;
    }
    for (int i = 5; i <= 8; ++i) {
      double a = (i - 5) * pi / 2.0 + pi / 4.0;
      vx[i] = (int32_t)lround(sqrt(2.0) * cos(a));
      vy[i] = (int32_t)lround(sqrt(2.0) * sin(a));
      w[i] = 1.0 / 36.0;
    }
    return 0;
  }
  return -1;
}

/* index of the velocity (cx, cy) in the set, or -1 */
static int or_find(int Q, int cx, int cy)
{
  int32_t vx[9], vy[9];
  double w[9];
  or_velocities(Q, vx, vy, w);
  for (int i = 0; i < Q; ++i)
    if (vx[i] == cx && vy[i] == cy) return i;
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Moments (Sec. 2: M = (rho, rho u1, rho u2, 2E); discrete sums Sec. 4)    */
/* ------------------------------------------------------------------------ */
void or_moments(int Q, const double* f, double* M)
{
  int32_t vx[9], vy[9];
  double w[9];
  or_velocities(Q, vx, vy, w);
  M[0] = M[1] = M[2] = M[3] = 0.0;
  for (int i = 0; i < Q; ++i) {
    M[0] += f[i];
    M[1] += vx[i] * f[i];
    M[2] += vy[i] * f[i];
    M[3] += (double)(vx[i] * vx[i] + vy[i] * vy[i]) * f[i];
  }
}

/* ------------------------------------------------------------------------ */
/* Quasiequilibria                                                          */
/* ------------------------------------------------------------------------ */

/*
 * Polynomial quasiequilibrium.
 * D1Q3: the three formulas printed in Sec. 4.1.
 * D2Q9: the standard second-order polynomial of the cited LBGK literature
 *   f*_i = W_i rho (1 + 3 v_i.u + 9/2 (v_i.u)^2 - 3/2 u.u);
 *   the paper gives it only by reference; its pins are the exact moments
 *   and its u2 = 0 marginal, which is the D1Q3 formula of Sec. 4.1.
 */
void or_qe_poly(int Q, double rho, double u1, double u2, double* fs)
{
  if (Q == 3) {
    double u = u1;
    fs[0] = (2.0 * rho / 3.0) * (1.0 - 3.0 * u * u / 2.0);
    fs[1] = (rho / 6.0) * (1.0 - 3.0 * u + 3.0 * u * u);
    fs[2] = (rho / 6.0) * (1.0 + 3.0 * u + 3.0 * u * u);
    return;
  }
  int32_t vx[9], vy[9];
  double w[9];
  or_velocities(9, vx, vy, w);
  double uu = u1 * u1 + u2 * u2;
  for (int i = 0; i < 9; ++i) {
    double cu = vx[i] * u1 + vy[i] * u2;
    fs[i] = w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/*
 * Entropic quasiequilibrium under mass and momentum constraints.
 * D1Q3: Sec. 4.1's explicit formulas, with the printed right-hand sides of
 *   f2 and f3 exchanged: as printed, f2 - f3 yields rho u for the
 *   left-moving f2, i.e. momentum -rho u.  The exchanged pair reproduces
 *   +rho u and is the 1-D factor of the D2Q9 formula below.
 * D2Q9: Sec. 4.2's product formula
 *   f*_i = rho W_i prod_j (2 - sqrt(1+3u_j^2)) ((2u_j + sqrt(1+3u_j^2))/(1-u_j))^{v_ij}.
 */
void or_qe_entropic_mm(int Q, double rho, double u1, double u2, double* fs)
{
  if (Q == 3) {
    double s = sqrt(1.0 + 3.0 * u1 * u1);
    fs[0] = (2.0 * rho / 3.0) * (2.0 - s);
    fs[1] = (rho / 6.0) * ((-3.0 * u1 - 1.0) + 2.0 * s); /* left-moving */
    fs[2] = (rho / 6.0) * ((3.0 * u1 - 1.0) + 2.0 * s);  /* right-moving */
    return;
  }
  int32_t vx[9], vy[9];
  double w[9];
  or_velocities(9, vx, vy, w);
  double u[2] = {u1, u2};
  for (int i = 0; i < 9; ++i) {
    int v[2] = {vx[i], vy[i]};
    double p = rho * w[i];
    for (int j = 0; j < 2; ++j) {
      double s = sqrt(1.0 + 3.0 * u[j] * u[j]);
      double base = (2.0 * u[j] + s) / (1.0 - u[j]);
      p *= (2.0 - s) * pow(base, (double)v[j]);
    }
    fs[i] = p;
  }
}

/*
 * Entropic quasiequilibrium with the energy row, f*_M (Sec. 2, argmax
 * problem, with M = (rho, rho u1, rho u2, 2E); Sec. 3.3: ln f*_k is linear
 * in the moment rows with Lagrange multipliers mu_j).  D2Q9 only.
 *
 * With the rows m_i = (1, vx_i, vy_i, |v_i|^2), f*_i = exp(mu . m_i) (the
 * weights W_i are absorbed into mu_0 and mu_3 since ln W_i is itself a
 * combination of the rows 1 and |v|^2).
 */
void or_fstar_from_mu(const double* mu, double* fs)
{
  int32_t vx[9], vy[9];
  double w[9];
  or_velocities(9, vx, vy, w);
  for (int i = 0; i < 9; ++i)
    fs[i] = exp(mu[0] + mu[1] * vx[i] + mu[2] * vy[i] + mu[3] * (vx[i] * vx[i] + vy[i] * vy[i]));
}

/*
 * A moment vector is realisable by positive D2Q9 populations iff rho > 0
 * and |u1| + |u2| < 2E/rho < 2 (each |v|^2 is 0, 1 or 2, and |v|^2 >=
 * |vx| + |vy|).
 */
int or_fstar_feasible(const double* M)
{
  if (!(M[0] > 0.0)) return 0;
  double u1 = M[1] / M[0], u2 = M[2] / M[0], e = M[3] / M[0];
  return (e > fabs(u1) + fabs(u2)) && (e < 2.0);
}

static void or_solve4(double A[4][4], double* b, double* x)
{
  /* Gaussian elimination with partial pivoting on a 4x4 system */
  int p[4] = {0, 1, 2, 3};
  for (int c = 0; c < 4; ++c) {
    int best = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(A[p[r]][c]) > fabs(A[p[best]][c])) best = r;
    int t = p[c];
    p[c] = p[best];
    p[best] = t;
    for (int r = c + 1; r < 4; ++r) {
      double m = A[p[r]][c] / A[p[c]][c];
      for (int cc = c; cc < 4; ++cc) A[p[r]][cc] -= m * A[p[c]][cc];
      b[p[r]] -= m * b[p[c]];
    }
  }
  for (int c = 3; c >= 0; --c) {
    double s = b[p[c]];
    for (int cc = c + 1; cc < 4; ++cc) s -= A[p[c]][cc] * x[cc];
    x[c] = s / A[p[c]][c];
  }
}

/* dual objective phi(mu) = sum_i exp(mu . m_i) - mu . M */
static double or_phi(const double* mu, const double* M)
{
  double fs[9];
  or_fstar_from_mu(mu, fs);
  double s = 0.0;
  for (int i = 0; i < 9; ++i) s += fs[i];
  return s - (mu[0] * M[0] + mu[1] * M[1] + mu[2] * M[2] + mu[3] * M[3]);
}

/*
 * Damped Newton on the convex dual: minimise phi(mu); its gradient is
 * m(f(mu)) - M and its Hessian sum_i f_i m_i m_i^T.  Start: the isothermal
 * rest state at the site's density, mu = (ln(4 rho/9), 0, 0, -ln 4), i.e.
 * f_i = rho W_i.  Armijo backtracking while the residual exceeds 1e-3.
 * Residual: max_j |m_j(f) - M_j| / rho.  Returns the iteration count, or
 * -1 for an infeasible M, -2 if max_iter is reached.
 */
int or_fstar_newton(const double* M, double tol, int max_iter, double* mu, double* resid)
{
  if (!or_fstar_feasible(M)) {
    *resid = INFINITY;
    return -1;
  }
  mu[0] = log(4.0 * M[0] / 9.0);
  mu[1] = 0.0;
  mu[2] = 0.0;
  mu[3] = -log(4.0);
  return or_fstar_newton_from(M, tol, max_iter, mu, resid);
}

/* the same damped Newton from the multipliers in mu on entry */
int or_fstar_newton_from(const double* M, double tol, int max_iter, double* mu, double* resid)
{
  *resid = INFINITY;
  if (!or_fstar_feasible(M)) return -1;
  int32_t vx[9], vy[9];
  double w[9];
  or_velocities(9, vx, vy, w);
  double m[9][4];
  for (int i = 0; i < 9; ++i) {
    m[i][0] = 1.0;
    m[i][1] = vx[i];
    m[i][2] = vy[i];
    m[i][3] = vx[i] * vx[i] + vy[i] * vy[i];
  }
  for (int it = 0; it <= max_iter; ++it) {
    double fs[9];
    or_fstar_from_mu(mu, fs);
    double g[4] = {-M[0], -M[1], -M[2], -M[3]};
    double H[4][4] = {{0}};
    for (int i = 0; i < 9; ++i)
      for (int a = 0; a < 4; ++a) {
        g[a] += fs[i] * m[i][a];
        for (int b = 0; b < 4; ++b) H[a][b] += fs[i] * m[i][a] * m[i][b];
      }
    double r = 0.0;
    for (int a = 0; a < 4; ++a)
      if (fabs(g[a]) / M[0] > r) r = fabs(g[a]) / M[0];
    *resid = r;
    if (r <= tol) return it;
    if (it == max_iter) break;
    double rhs[4] = {-g[0], -g[1], -g[2], -g[3]}, d[4];
    or_solve4(H, rhs, d);
    double t = 1.0;
    if (r > 1e-3) {
      double phi0 = or_phi(mu, M);
      double slope = g[0] * d[0] + g[1] * d[1] + g[2] * d[2] + g[3] * d[3];
      for (int ls = 0; ls < 60; ++ls) {
        double trial[4];
        for (int a = 0; a < 4; ++a) trial[a] = mu[a] + t * d[a];
        if (or_phi(trial, M) <= phi0 + 1e-4 * t * slope) break;
        t *= 0.5;
      }
    }
    for (int a = 0; a < 4; ++a) mu[a] += t * d[a];
  }
  return -2;
}

/*
 * Gradient m(f(mu)) - M and Hessian sum_i f_i m_i m_i^T of the dual at mu;
 * returns the residual max_j |g_j| / rho.
 */
static double or_fstar_gh(const double* M, const double* mu, double* g, double H[4][4])
{
  int32_t vx[9], vy[9];
  double w[9], fs[9];
  or_velocities(9, vx, vy, w);
  or_fstar_from_mu(mu, fs);
  for (int a = 0; a < 4; ++a) {
    g[a] = -M[a];
    for (int b = 0; b < 4; ++b) H[a][b] = 0.0;
  }
  for (int i = 0; i < 9; ++i) {
    double m[4] = {1.0, vx[i], vy[i], vx[i] * vx[i] + vy[i] * vy[i]};
    for (int a = 0; a < 4; ++a) {
      g[a] += fs[i] * m[a];
      for (int b = 0; b < 4; ++b) H[a][b] += fs[i] * m[a] * m[b];
    }
  }
  double r = 0.0;
  for (int a = 0; a < 4; ++a)
    if (fabs(g[a]) / M[0] > r) r = fabs(g[a]) / M[0];
  return r;
}

/*
 * One more undamped Newton update from converged multipliers.  From a
 * residual of 1e-13 Newton's quadratic convergence leaves O(1e-26) in exact
 * arithmetic, so the update carries mu to the maximiser of Sec. 2 up to FP64
 * round-off; it is kept only if the residual does not grow.  Returns the
 * final residual.
 */
double or_fstar_polish(const double* M, double* mu)
{
  double g[4], H[4][4], g1[4], H1[4][4];
  double r0 = or_fstar_gh(M, mu, g, H);
  double rhs[4] = {-g[0], -g[1], -g[2], -g[3]}, d[4], trial[4];
  or_solve4(H, rhs, d);
  for (int a = 0; a < 4; ++a) trial[a] = mu[a] + d[a];
  double r1 = or_fstar_gh(M, trial, g1, H1);
  if (!(r1 <= r0)) return r0;
  for (int a = 0; a < 4; ++a) mu[a] = trial[a];
  return r1;
}

/*
 * Independent route to f*_M through its product structure: on D2Q9,
 * |v|^2 = vx^2 + vy^2, so f*_i = A g(vx_i) g(vy_i) with g(0) = 1,
 * g(+-1) = Z X^{+-1} (and Y for the y factor), (A, X, Y, Z) = exp(mu).
 * For fixed Z each velocity component fixes X (a quadratic), the energy per
 * mass e_x(Z) + e_y(Z) is increasing in Z, and the energy constraint is
 * solved by bisection on ln Z in long double.
 */
static long double or_xfactor(long double u, long double Z, long double* e)
{
  /* positive root of Z(1-u) X^2 - u X - Z(1+u) = 0, in the form free of
     cancellation for either sign of u */
  long double D = sqrtl(u * u + 4.0L * Z * Z * (1.0L - u * u));
  long double X = u >= 0.0L ? (u + D) / (2.0L * Z * (1.0L - u)) : (2.0L * Z * (1.0L + u)) / (D - u);
  long double q = Z * (X + 1.0L / X);
  *e = q / (1.0L + q);
  return X;
}

int or_fstar_scalar(const double* M, double* mu)
{
  if (!or_fstar_feasible(M)) return -1;
  long double rho = M[0], u1 = M[1] / (long double)M[0], u2 = M[2] / (long double)M[0];
  long double e = M[3] / (long double)M[0];
  long double lo = -80.0L, hi = 80.0L;
  for (int it = 0; it < 400; ++it) {
    long double mid = 0.5L * (lo + hi), ex, ey;
    long double Z = expl(mid);
    or_xfactor(u1, Z, &ex);
    or_xfactor(u2, Z, &ey);
    if (ex + ey < e) lo = mid;
    else hi = mid;
  }
  long double lz = 0.5L * (lo + hi), Z = expl(lz), ex, ey;
  long double X = or_xfactor(u1, Z, &ex);
  long double Y = or_xfactor(u2, Z, &ey);
  long double nx = 1.0L + Z * (X + 1.0L / X), ny = 1.0L + Z * (Y + 1.0L / Y);
  mu[0] = (double)logl(rho / (nx * ny));
  mu[1] = (double)logl(X);
  mu[2] = (double)logl(Y);
  mu[3] = (double)lz;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Nonequilibrium entropy                                                   */
/* ------------------------------------------------------------------------ */
/*
 * Delta S = S(f*) - S(f) for the perfect entropy S = -sum f ln(f/W)
 * (Sec. 3.3).  Written as sum_i [f_i ln(f_i/f*_i) - f_i + f*_i], which is
 * the Kullback form of Sec. 3.3 whenever sum f = sum f*, stays >= 0 when
 * the masses differ by round-off, and vanishes only at f = f*.
 * A site with some f_i < 0 or f*_i <= 0 has no finite entropy: +inf.
 * A population f_i = 0 contributes its limit f*_i.
 */
long double or_delta_S(int Q, const double* f, const double* fs)
{
  long double acc = 0.0L;
  for (int i = 0; i < Q; ++i) {
    long double a = f[i], b = fs[i];
    if (!(a >= 0.0L) || !(b > 0.0L)) return INFINITY;
    if (a == 0.0L) acc += b;
    else acc += a * logl(a / b) - a + b;
  }
  return acc;
}

/* perfect entropy S(f) = -sum f ln(f/W) in long double (used by ELBM) */
static long double or_entropy(int Q, const long double* f)
{
  int32_t vx[9], vy[9];
  double w[9];
  or_velocities(Q, vx, vy, w);
  long double s = 0.0L;
  for (int i = 0; i < Q; ++i) {
    if (f[i] < 0.0L) return -INFINITY;
    if (f[i] > 0.0L) s -= f[i] * logl(f[i] / (long double)w[i]);
  }
  return s;
}

/*
 * ELBM (Sec. 3.2 and Sec. 4.1): alpha is the nontrivial root of
 * S(f + alpha (f* - f)) = S(f), found by bisection to an accuracy of 1e-15.
 *
 * Evaluation without cancellation.  With x_i = f*_i / f_i - 1 (f, f* > 0)
 * and S(g) = -sum g ln(g/W):
 *   S(f + a (f* - f)) - S(f)
 *     = -a sum f x ln(f/W) - sum f (1 + a x) ln(1 + a x).
 * For an entropic f* with the conserved moments of f, ln(f* / W) lies in the
 * span of the moment rows, so sum (f* - f) ln(f* / W) = 0 and
 * sum f x ln(f/W) = -sum f x ln(1 + x); with sum (f* - f) = 0 (mass row)
 *   H(a) = sum_i f_i [a psi(x_i) - phi(a x_i)],
 *   psi(x) = x ln(1 + x),  phi(y) = (1 + y) ln(1 + y) - y,
 * in which every term is O(x^2); phi uses its Taylor series
 * sum_{k>=2} (-1)^k y^k / (k (k-1)) for |y| < 0.1.  H(1) is Delta S, H is
 * concave with its maximum at a = 1, and the root lies in (1, a_max], a_max
 * the largest a that keeps every population non-negative (capped at 1000);
 * if H(a_max) >= 0 there is no root below it and a_max is returned.
 * A site with some f_i <= 0 or f*_i <= 0 has no entropy to conserve; it, and
 * a site at f = f*, takes the LBGK mirror a = 2.
 */
static long double or_phi_elbm(long double y)
{
  if (fabsl(y) < 0.1L) {
    long double s = 0.0L, p = y * y;
    for (int k = 2; k <= 22; ++k) {
      s += ((k & 1) ? -p : p) / (long double)(k * (k - 1));
      p *= y;
    }
    return s;
  }
  return (1.0L + y) * log1pl(y) - y;
}

long double or_elbm_H(int Q, const double* f, const double* fs, long double a)
{
  long double h = 0.0L;
  for (int i = 0; i < Q; ++i) {
    long double x = (long double)fs[i] / (long double)f[i] - 1.0L;
    h += (long double)f[i] * (a * x * log1pl(x) - or_phi_elbm(a * x));
  }
  return h;
}

double or_elbm_alpha(int Q, const double* f, const double* fs)
{
  long double amax = 1000.0L;
  int moving = 0;
  for (int i = 0; i < Q; ++i) {
    if (!(f[i] > 0.0) || !(fs[i] > 0.0)) return 2.0;
    long double x = (long double)fs[i] / (long double)f[i] - 1.0L;
    if (x != 0.0L) moving = 1;
    if (x < 0.0L && -1.0L / x < amax) amax = -1.0L / x;
  }
  if (!moving) return 2.0;
  long double lo = 1.0L, hi = amax;
  if (or_elbm_H(Q, f, fs, hi) >= 0.0L) return (double)hi;
  while (hi - lo > 1e-15L) {
    long double mid = 0.5L * (lo + hi);
    if (or_elbm_H(Q, f, fs, mid) > 0.0L) lo = mid;
    else hi = mid;
  }
  return (double)(0.5L * (lo + hi));
}

/* ------------------------------------------------------------------------ */
/* Lattice                                                                  */
/* ------------------------------------------------------------------------ */

static int or_solid(const or_cfg* c, int64_t x, int64_t y)
{
  return c->solid_w > 0 && c->solid_h > 0 && x >= c->solid_x0 && x < c->solid_x0 + c->solid_w &&
         y >= c->solid_y0 && y < c->solid_y0 + c->solid_h;
}

/* quasiequilibrium of the configured kind for one site; returns 1 on a
   closed-form fallback of the f*_M solve */
static int or_site_qe(const or_cfg* c, const double* M, double* fs)
{
  double rho = M[0], u1 = M[1] / M[0], u2 = M[2] / M[0];
  if (c->qe == OR_QE_POLY) {
    or_qe_poly(c->Q, rho, u1, u2, fs);
    return 0;
  }
  if (c->qe == OR_QE_ENTROPIC_MM) {
    or_qe_entropic_mm(c->Q, rho, u1, u2, fs);
    return 0;
  }
  double mu[4], r;
  int it = or_fstar_newton(M, 1e-13, 100, mu, &r);
  if (it < 0) {
    /* infeasible or unconverged: mass-momentum closed form */
    or_qe_entropic_mm(c->Q, rho, u1, u2, fs);
    return 1;
  }
  or_fstar_polish(M, mu);
  or_fstar_from_mu(mu, fs);
  return 0;
}

/* inlet quasiequilibrium (entropic configurations use the mass-momentum
   closed form, which is f*_M at the isothermal energy) */
static void or_inlet_qe(const or_cfg* c, double* fs)
{
  if (c->qe == OR_QE_POLY) or_qe_poly(c->Q, c->inlet_rho, c->inlet_u1, c->inlet_u2, fs);
  else or_qe_entropic_mm(c->Q, c->inlet_rho, c->inlet_u1, c->inlet_u2, fs);
}

/*
 * Where f_i(x, y, t+1) comes from (free flight, Sec. 3, with the boundary
 * rules of Sec. 4.2 as read for these configurations):
 *   returns 1: the post-collision population *pj at (*px, *py);
 *   returns 0: the inlet quasiequilibrium value of population i;
 *   returns 2: the outlet rule: population i of the quasiequilibrium at the
 *     density and velocity of f(*px, y, t+1), *px the penultimate column.
 * Rules, in this order:
 *   x outside: periodic wrap | zero-gradient: the value that the adjacent
 *     inner column receives | inlet: quasiequilibrium at the inlet state |
 *     outlet: quasiequilibrium of the penultimate column (Sec. 4.2);
 *   y outside: periodic wrap | free-slip: specular reflection, i.e. the
 *     population with the mirrored vertical velocity leaving from
 *     (x - cx, y) | zero-gradient: the value the adjacent inner row receives;
 *   source inside the solid: halfway bounce-back, the opposite population
 *     leaving (x, y).
 */
static int or_source(const or_cfg* c, const int32_t* vx, const int32_t* vy, int64_t x, int64_t y,
                     int i, int64_t* px, int64_t* py, int* pj)
{
  int64_t nx = c->nx, ny = c->ny;
  int64_t sx = x - vx[i], sy = y - vy[i];
  int j = i;
  if (sx < 0 || sx >= nx) {
    int b = sx < 0 ? c->bc[0] : c->bc[1];
    if (b == OR_BC_PERIODIC) sx = ((sx % nx) + nx) % nx;
    else if (b == OR_BC_INLET_EQ) return 0;
    else if (b == OR_BC_OUTLET_EQ || b == OR_BC_OUTLET_EQ_PREV) {
      *px = sx < 0 ? 1 : nx - 2;
      *py = y;
      *pj = i;
      return 2;
    } else return or_source(c, vx, vy, sx < 0 ? x + 1 : x - 1, y, i, px, py, pj);
  }
  if (sy < 0 || sy >= ny) {
    int b = sy < 0 ? c->bc[2] : c->bc[3];
    if (b == OR_BC_PERIODIC) sy = ((sy % ny) + ny) % ny;
    else if (b == OR_BC_FREESLIP) {
      j = or_find(c->Q, vx[i], -vy[i]);
      sy = y;
    } else if (b == OR_BC_INLET_EQ) return 0;
    else return or_source(c, vx, vy, x, sy < 0 ? y + 1 : y - 1, i, px, py, pj);
  }
  if (or_solid(c, sx, sy)) {
    j = or_find(c->Q, -vx[i], -vy[i]);
    sx = x;
    sy = y;
  }
  *px = sx;
  *py = sy;
  *pj = j;
  return 1;
}

/* Post-collision values: either a stored field (N-site planes) or, when
   fpost is NULL, evaluated from the pre-collision field f_in at the one
   site, with the caller's set of sites returned to quasiequilibrium. */
typedef struct {
  const or_cfg* c;
  const double* fpost;
  const double* f_in;
  const int64_t* sel;
  int64_t nsel;
  double beta;
} or_post;

static double or_post_value(const or_post* P, int64_t s, int j)
{
  const or_cfg* c = P->c;
  int Q = c->Q;
  int64_t N = c->nx * c->ny;
  if (P->fpost) return P->fpost[(int64_t)j * N + s];
  double f[9], fs[9], M[4];
  for (int q = 0; q < Q; ++q) f[q] = P->f_in[(int64_t)q * N + s];
  or_moments(Q, f, M);
  or_site_qe(c, M, fs);
  int chosen = 0;
  for (int64_t r = 0; r < P->nsel; ++r)
    if (P->sel[r] == s) chosen = 1;
  if (chosen) return fs[j];
  double a = 2.0;
  if (c->collision == OR_COLL_ELBM) a = or_elbm_alpha(Q, f, fs);
  return f[j] + a * P->beta * (fs[j] - f[j]);
}

/* f_i(x, y, t+1) of a fluid site: free flight of the post-collision field
   with the boundary rules of or_source */
static double or_new_value(const or_post* P, const int32_t* vx, const int32_t* vy, int64_t x, int64_t y,
                           int i)
{
  const or_cfg* c = P->c;
  int64_t px, py;
  int j;
  int r = or_source(c, vx, vy, x, y, i, &px, &py, &j);
  if (r == 1) return or_post_value(P, py * c->nx + px, j);
  double fs[9];
  if (r == 0) {
    or_inlet_qe(c, fs);
    return fs[i];
  }
  /* outlet: density and velocity of the penultimate column, either of its
     new state at t+1 (OR_BC_OUTLET_EQ) or of its state at t
     (OR_BC_OUTLET_EQ_PREV; the collision keeps these moments) */
  double g[9], M[4];
  int b = x == 0 ? c->bc[0] : c->bc[1];
  int64_t N = c->nx * c->ny;
  for (int q = 0; q < c->Q; ++q)
    g[q] = b == OR_BC_OUTLET_EQ_PREV ? P->f_in[(int64_t)q * N + py * c->nx + px] : or_new_value(P, vx, vy, px, py, q);
  or_moments(c->Q, g, M);
  double u2 = c->Q == 9 ? M[2] / M[0] : 0.0;
  if (c->qe == OR_QE_POLY) or_qe_poly(c->Q, M[0], M[1] / M[0], u2, fs);
  else or_qe_entropic_mm(c->Q, M[0], M[1] / M[0], u2, fs);
  return fs[i];
}

/* f(x, 0) = quasiequilibrium of the initial fields at fluid sites, 0 in the solid */
int or_init(const or_cfg* c, const double* rho0, const double* u0, const double* twoE0, double* f)
{
  int Q = c->Q;
  int64_t N = c->nx * c->ny;
  for (int64_t s = 0; s < N; ++s) {
    int64_t x = s % c->nx, y = s / c->nx;
    double fs[9];
    if (or_solid(c, x, y)) {
      for (int i = 0; i < Q; ++i) fs[i] = 0.0;
    } else if (c->qe == OR_QE_ENTROPIC_M && twoE0) {
      double M[4] = {rho0[s], rho0[s] * u0[s], rho0[s] * u0[N + s], rho0[s] * twoE0[s]};
      or_site_qe(c, M, fs);
    } else {
      double u2 = Q == 9 ? u0[N + s] : 0.0;
      if (c->qe == OR_QE_POLY) or_qe_poly(Q, rho0[s], u0[s], u2, fs);
      else or_qe_entropic_mm(Q, rho0[s], u0[s], u2, fs);
    }
    for (int i = 0; i < Q; ++i) f[(int64_t)i * N + s] = fs[i];
  }
  return 0;
}

typedef struct {
  long double dS;
  int64_t s;
} or_cand;

/* order: larger Delta S first, then lower site index */
static int or_cand_cmp(const void* a, const void* b)
{
  const or_cand* x = (const or_cand*)a;
  const or_cand* y = (const or_cand*)b;
  if (x->dS > y->dS) return -1;
  if (x->dS < y->dS) return 1;
  return (x->s > y->s) - (x->s < y->s);
}

/*
 * One time step of LBGK with Ehrenfests' steps (Sec. 3.2, Sec. 4.1):
 *  1. at every fluid site: M = m(f), f* = f*(M), Delta S(f);
 *  2. C = {s : Delta S(s) > delta}; if |C| <= k all of C is selected,
 *     otherwise the k sites with the largest Delta S (ties: lower site
 *     index s = x + nx y);
 *  3. selected sites are returned to quasiequilibrium, f' = f*; all other
 *     fluid sites take the LBGK step f' = f + 2 beta (f* - f)
 *     (or, for ELBM, f + alpha beta (f* - f));
 *  4. free flight of f' with the boundary rules of or_source gives f(t+1).
 * beta = 1/(1 + 6 nu) from nu = c_s^2 (1/(2 beta) - 1/2), c_s^2 = 1/3.
 * dS (optional) receives Delta S per site (0 in the solid); sel (optional,
 * capacity k) the selected sites in rank order.
 */
int or_step(const or_cfg* c, const double* f_in, double* f_out, double* dS, int64_t* sel,
            or_step_info* info)
{
  int Q = c->Q;
  int64_t nx = c->nx, ny = c->ny, N = nx * ny;
  int32_t vx[9], vy[9];
  double w[9];
  or_velocities(Q, vx, vy, w);
  double beta = 1.0 / (1.0 + 6.0 * c->nu);

  double* fst = (double*)malloc(sizeof(double) * (size_t)Q * (size_t)N);
  double* fpost = (double*)malloc(sizeof(double) * (size_t)Q * (size_t)N);
  long double* dsl = (long double*)malloc(sizeof(long double) * (size_t)N);
  unsigned char* chosen = (unsigned char*)calloc((size_t)N, 1);
  or_cand* cand = (or_cand*)malloc(sizeof(or_cand) * (size_t)(N > 0 ? N : 1));
  if (!fst || !fpost || !dsl || !chosen || !cand) {
    free(fst);
    free(fpost);
    free(dsl);
    free(chosen);
    free(cand);
    return -2;
  }
  memset(info, 0, sizeof(*info));

  /* 1. moments, quasiequilibrium, nonequilibrium entropy (the site loops
     carry OpenMP pragmas for a separate timing build; the plain build runs
     them in site-index order) */
  double sums[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t n_fallback = 0, n_invalid = 0;
#pragma omp parallel for schedule(static) reduction(+ : sums[:4], n_fallback, n_invalid)
  for (int64_t s = 0; s < N; ++s) {
    int64_t x = s % nx, y = s / nx;
    dsl[s] = 0.0L;
    if (or_solid(c, x, y)) continue;
    double f[9], fs[9], M[4];
    for (int i = 0; i < Q; ++i) f[i] = f_in[(int64_t)i * N + s];
    or_moments(Q, f, M);
    for (int a = 0; a < 4; ++a) sums[a] += M[a];
    n_fallback += or_site_qe(c, M, fs);
    for (int i = 0; i < Q; ++i) fst[(int64_t)i * N + s] = fs[i];
    dsl[s] = or_delta_S(Q, f, fs);
    if (isinf(dsl[s])) n_invalid++;
  }
  for (int a = 0; a < 4; ++a) info->sums[a] = sums[a];
  info->n_fallback = n_fallback;
  info->n_invalid = n_invalid;
  /* the candidates C = {s : Delta S(s) > delta}, in site-index order */
  int64_t nc = 0;
  for (int64_t s = 0; s < N; ++s) {
    if (or_solid(c, s % nx, s / nx)) continue;
    if (dsl[s] > (long double)c->delta) {
      cand[nc].dS = dsl[s];
      cand[nc].s = s;
      nc++;
    }
  }

  /* 2. selection */
  info->n_above = nc;
  int64_t take = nc;
  if (nc > c->k) {
    qsort(cand, (size_t)nc, sizeof(or_cand), or_cand_cmp);
    take = c->k;
  } else {
    qsort(cand, (size_t)nc, sizeof(or_cand), or_cand_cmp); /* rank order for the report */
  }
  if (take < 0) take = 0;
  for (int64_t r = 0; r < take; ++r) {
    chosen[cand[r].s] = 1;
    if (sel) sel[r] = cand[r].s;
  }
  info->n_selected = take;

  /* 3. collision or Ehrenfests' step */
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    int64_t x = s % nx, y = s / nx;
    if (or_solid(c, x, y)) {
      for (int i = 0; i < Q; ++i) fpost[(int64_t)i * N + s] = 0.0;
      continue;
    }
    double f[9], fs[9];
    for (int i = 0; i < Q; ++i) {
      f[i] = f_in[(int64_t)i * N + s];
      fs[i] = fst[(int64_t)i * N + s];
    }
    double a = 2.0;
    if (c->collision == OR_COLL_ELBM && !chosen[s]) a = or_elbm_alpha(Q, f, fs);
    for (int i = 0; i < Q; ++i)
      fpost[(int64_t)i * N + s] = chosen[s] ? fs[i] : f[i] + a * beta * (fs[i] - f[i]);
  }

  /* 4. free flight with boundary rules */
  or_post P = {c, fpost, f_in, NULL, 0, beta};
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    int64_t x = s % nx, y = s / nx;
    for (int i = 0; i < Q; ++i)
      f_out[(int64_t)i * N + s] = or_solid(c, x, y) ? 0.0 : or_new_value(&P, vx, vy, x, y, i);
  }

  if (dS)
    for (int64_t s = 0; s < N; ++s) dS[s] = (double)dsl[s];
  free(fst);
  free(fpost);
  free(dsl);
  free(chosen);
  free(cand);
  return 0;
}

/*
 * The same time step evaluated only at the output sites `sites` (out:
 * [ns][Q]), with the set of sites returned to quasiequilibrium given by the
 * caller (sel, nsel).  Each output population is the post-collision value of
 * its free-flight source (or_source), computed from that source site alone.
 */
int or_step_sites(const or_cfg* c, const double* f_in, const int64_t* sites, int64_t ns, const int64_t* sel,
                  int64_t nsel, double* out)
{
  int Q = c->Q;
  int64_t nx = c->nx;
  int32_t vx[9], vy[9];
  double w[9];
  or_velocities(Q, vx, vy, w);
  or_post P = {c, NULL, f_in, sel, nsel, 1.0 / (1.0 + 6.0 * c->nu)};
  for (int64_t k = 0; k < ns; ++k) {
    int64_t x = sites[k] % nx, y = sites[k] / nx;
    for (int i = 0; i < Q; ++i)
      out[k * Q + i] = or_solid(c, x, y) ? 0.0 : or_new_value(&P, vx, vy, x, y, i);
  }
  return 0;
}

/* Delta S of one site of a lattice (pre-collision populations f_in) */
double or_site_dS(const or_cfg* c, const double* f_in, int64_t site)
{
  int Q = c->Q;
  int64_t N = c->nx * c->ny;
  double f[9], fs[9], M[4];
  for (int q = 0; q < Q; ++q) f[q] = f_in[(int64_t)q * N + site];
  or_moments(Q, f, M);
  or_site_qe(c, M, fs);
  return (double)or_delta_S(Q, f, fs);
}

/* ------------------------------------------------------------------------ */
/* Shedding frequency of a recorded signal (Sec. 4.2, Strouhal number)      */
/* ------------------------------------------------------------------------ */
/*
 * power[k] = |sum_j x_j exp(-2 pi i j k / n)|^2 for k = 0 .. n/2: the
 * discrete Fourier transform written out, summed in long double, each
 * angle reduced exactly to 2 pi ((j k) mod n) / n.  O(n) per bin
 * (or_dft_power_at), O(n^2) for the whole spectrum.
 */
double or_dft_power_at(const double* x, int64_t n, int64_t k)
{
  const long double two_pi = 6.283185307179586476925286766559L;
  long double re = 0.0L, im = 0.0L;
  for (int64_t j = 0; j < n; ++j) {
    long double ang = two_pi * (long double)((j * k) % n) / (long double)n;
    re += (long double)x[j] * cosl(ang);
    im -= (long double)x[j] * sinl(ang);
  }
  return (double)(re * re + im * im);
}

void or_dft_power(const double* x, int64_t n, double* power)
{
  for (int64_t k = 0; k <= n / 2; ++k) power[k] = or_dft_power_at(x, n, k);
}

/* ------------------------------------------------------------------------ */
/* MLP 4 -> 64 -> 64 -> 4 with SiLU: the learned warm start                  */
/* ------------------------------------------------------------------------ */
/*
 * Parameter layout (4740 values):
 *   W1 [64][4] @0, b1 [64] @256, W2 [64][64] @320, b2 [64] @4416,
 *   W3 [4][64] @4480, b3 [4] @4736.
 * With bf16 != 0 the BF16 rounding points of the GPU kernels are emulated:
 * inputs, weights, hidden activations (after SiLU) and the back-propagated
 * deltas that enter a product are rounded to BF16 (round to nearest even,
 * through FP32); sums are in FP64; biases, bias gradients and SiLU stay
 * unrounded.
 */
enum { OW1 = 0, OB1 = 256, OW2 = 320, OB2 = 4416, OW3 = 4480, OB3 = 4736 };

double or_bf16_round(double xd)
{
  float x = (float)xd;
  if (x != x) return xd;
  uint32_t b;
  memcpy(&b, &x, 4);
  uint32_t lsb = (b >> 16) & 1u;
  b = (b + 0x7FFFu + lsb) & 0xFFFF0000u;
  float r;
  memcpy(&r, &b, 4);
  return (double)r;
}

static double or_sig(double z) { return 1.0 / (1.0 + exp(-z)); }

typedef struct {
  double xb[4], z1[64], h1[64], z2[64], h2[64], y[4];
} or_act;

static void or_mlp_one(const double* p, const double* x, int bf16, or_act* a)
{
#define RB(v) (bf16 ? or_bf16_round(v) : (v))
  for (int k = 0; k < 4; ++k) a->xb[k] = RB(x[k]);
  for (int j = 0; j < 64; ++j) {
    double s = 0.0;
    for (int k = 0; k < 4; ++k) s += RB(p[OW1 + j * 4 + k]) * a->xb[k];
    a->z1[j] = s + p[OB1 + j];
    a->h1[j] = RB(a->z1[j] * or_sig(a->z1[j]));
  }
  for (int j = 0; j < 64; ++j) {
    double s = 0.0;
    for (int k = 0; k < 64; ++k) s += RB(p[OW2 + j * 64 + k]) * a->h1[k];
    a->z2[j] = s + p[OB2 + j];
    a->h2[j] = RB(a->z2[j] * or_sig(a->z2[j]));
  }
  for (int o = 0; o < 4; ++o) {
    double s = 0.0;
    for (int k = 0; k < 64; ++k) s += RB(p[OW3 + o * 64 + k]) * a->h2[k];
    a->y[o] = s + p[OB3 + o];
  }
#undef RB
}

/* forward over n samples x[n][4] -> y[n][4]; returns 0 */
double or_mlp_forward(const double* p, const double* x, int64_t n, double* y, int bf16)
{
  or_act a;
  for (int64_t b = 0; b < n; ++b) {
    or_mlp_one(p, x + 4 * b, bf16, &a);
    for (int o = 0; o < 4; ++o) y[4 * b + o] = a.y[o];
  }
  return 0.0;
}

/*
 * Mean squared error L = (1/(4n)) sum_b sum_o (y_bo - t_bo)^2 and its
 * gradient with respect to all 4740 parameters (back-propagation through
 * the three layers; SiLU'(z) = sig(z) (1 + z (1 - sig(z)))).
 */
double or_mlp_loss_grad(const double* p, const double* x, const double* t, int64_t n,
                        double* grad, int bf16)
{
#define RB(v) (bf16 ? or_bf16_round(v) : (v))
  memset(grad, 0, sizeof(double) * OR_MLP_NPARAM);
  double loss = 0.0;
  or_act a;
  for (int64_t b = 0; b < n; ++b) {
    or_mlp_one(p, x + 4 * b, bf16, &a);
    double g[4], gb[4];
    for (int o = 0; o < 4; ++o) {
      double d = a.y[o] - t[4 * b + o];
      loss += d * d;
      g[o] = 2.0 * d / (4.0 * (double)n);
      if (bf16) g[o] = (double)(float)g[o];
      gb[o] = RB(g[o]);
    }
    /* layer 3 */
    for (int o = 0; o < 4; ++o) {
      for (int k = 0; k < 64; ++k) grad[OW3 + o * 64 + k] += gb[o] * a.h2[k];
      grad[OB3 + o] += g[o];
    }
    double dz2[64], dz2b[64];
    for (int k = 0; k < 64; ++k) {
      double s = 0.0;
      for (int o = 0; o < 4; ++o) s += RB(p[OW3 + o * 64 + k]) * gb[o];
      double sg = or_sig(a.z2[k]);
      dz2[k] = s * sg * (1.0 + a.z2[k] * (1.0 - sg));
      dz2b[k] = RB(dz2[k]);
    }
    /* layer 2 */
    for (int j = 0; j < 64; ++j) {
      for (int k = 0; k < 64; ++k) grad[OW2 + j * 64 + k] += dz2b[j] * a.h1[k];
      grad[OB2 + j] += dz2[j];
    }
    double dz1[64], dz1b[64];
    for (int k = 0; k < 64; ++k) {
      double s = 0.0;
      for (int j = 0; j < 64; ++j) s += RB(p[OW2 + j * 64 + k]) * dz2b[j];
      double sg = or_sig(a.z1[k]);
      dz1[k] = s * sg * (1.0 + a.z1[k] * (1.0 - sg));
      dz1b[k] = RB(dz1[k]);
    }
    /* layer 1 */
    for (int j = 0; j < 64; ++j) {
      for (int k = 0; k < 4; ++k) grad[OW1 + j * 4 + k] += dz1b[j] * a.xb[k];
      grad[OB1 + j] += dz1[j];
    }
  }
#undef RB
  return loss / (4.0 * (double)n);
}

/* Adam (Kingma and Ba): step number t >= 1, bias-corrected moments */
void or_adam_step(double* p, double* m, double* v, const double* g, int64_t n, int64_t t,
                  double lr, double b1, double b2, double eps)
{
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ------------------------------------------------------------------------ */
/* Inputs and outputs of the warm-start network                             */
/* ------------------------------------------------------------------------ */
/*
 * The network proposes a start for the f*_M solve of Sec. 2 (argmax with
 * M = (rho, rho u1, rho u2, 2E)).  Its inputs are the moments per unit mass
 * u1, u2, 2E/rho and |u|^2; its outputs are the multipliers with the
 * density taken out, (mu0 - ln rho, mu1, mu2, mu3).  By the density
 * scaling of f*_M (M -> lambda M leaves (mu1, mu2, mu3) and mu0 - ln rho
 * unchanged, since f* is linear in A = exp(mu0) for fixed X, Y, Z) both
 * depend on (u1, u2, 2E/rho) only.  They are mapped to O(1) by
 * x = (v - shift) * scale with the 16 constants norm[0..3] (input shifts),
 * norm[4..7] (input scales), norm[8..11] (output shifts), norm[12..15]
 * (output scales).  The normalised inputs are rounded to FP32, the
 * precision in which the network receives them.  Arrays: M and mu
 * [4][n] (component-major), X, T and Y [n][4] (sample-major).
 */
void or_mlp_features(const double* M, int64_t n, const float* norm, double* X)
{
  for (int64_t s = 0; s < n; ++s) {
    double rho = M[s];
    double u1 = M[n + s] / rho, u2 = M[2 * n + s] / rho, e = M[3 * n + s] / rho;
    double v[4] = {u1, u2, e, u1 * u1 + u2 * u2};
    for (int k = 0; k < 4; ++k) X[4 * s + k] = (double)(float)((v[k] - (double)norm[k]) * (double)norm[4 + k]);
  }
}

void or_mlp_targets(const double* M, const double* mu, int64_t n, const float* norm, double* T)
{
  for (int64_t s = 0; s < n; ++s) {
    double v[4] = {mu[s] - log(M[s]), mu[n + s], mu[2 * n + s], mu[3 * n + s]};
    for (int k = 0; k < 4; ++k) T[4 * s + k] = (v[k] - (double)norm[8 + k]) * (double)norm[12 + k];
  }
}

/* network outputs Y back to (mu0 - ln rho, mu1, mu2, mu3), out [4][n] */
void or_mlp_unnormalise(const double* Y, int64_t n, const float* norm, double* out)
{
  for (int64_t s = 0; s < n; ++s)
    for (int k = 0; k < 4; ++k) out[k * n + s] = Y[4 * s + k] / (double)norm[12 + k] + (double)norm[8 + k];
}

/* ------------------------------------------------------------------------ */
/* Conservation sums                                                        */
/* ------------------------------------------------------------------------ */
/*
 * Sums over the fluid sites of a state f of the moments rho, rho u1, rho u2
 * and 2E (Sec. 2: the collision conserves mass and momentum, Sec. 3.1; the
 * Ehrenfests' step returns a site to the quasiequilibrium with the same
 * moments), accumulated in long double site by site in index order.
 */
void or_sums(const or_cfg* c, const double* f, double* sums)
{
  int Q = c->Q;
  int64_t N = c->nx * c->ny;
  long double acc[4] = {0.0L, 0.0L, 0.0L, 0.0L};
  for (int64_t s = 0; s < N; ++s) {
    if (or_solid(c, s % c->nx, s / c->nx)) continue;
    double g[9], M[4];
    for (int i = 0; i < Q; ++i) g[i] = f[(int64_t)i * N + s];
    or_moments(Q, g, M);
    for (int a = 0; a < 4; ++a) acc[a] += M[a];
  }
  for (int a = 0; a < 4; ++a) sums[a] = (double)acc[a];
}

/* ------------------------------------------------------------------------ */
/* f*_M of a whole moment field (timing of the CPU baseline)                */
/* ------------------------------------------------------------------------ */
/*
 * Solves n sites M [4][n] to the residual tol by the damped Newton above,
 * from the rest start (start = 0), from the mass-momentum closed form of
 * Sec. 4.2 (start = 1: mu = (ln(4 rho (2 - s_x)(2 - s_y) / 9), ln X, ln Y,
 * -ln 4), the multipliers of that formula, since W_i = (4/9) (1/4)^{|v|^2}),
 * or from the values in mu on entry (start = 2).  iters [n] receives the
 * Newton updates (-1 infeasible, -2 unconverged).  Returns the number of
 * sites that did not converge.
 */
int64_t or_fstar_field(const double* M, int64_t n, double tol, int start, double* mu, int32_t* iters)
{
  int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : bad)
  for (int64_t s = 0; s < n; ++s) {
    double m[4] = {M[s], M[n + s], M[2 * n + s], M[3 * n + s]}, x[4] = {0.0, 0.0, 0.0, 0.0}, r;
    int it;
    if (start == 0) {
      it = or_fstar_newton(m, tol, 100, x, &r);
    } else {
      if (start == 1) {
        double u1 = m[1] / m[0], u2 = m[2] / m[0];
        double sx = sqrt(1.0 + 3.0 * u1 * u1), sy = sqrt(1.0 + 3.0 * u2 * u2);
        x[0] = log(4.0 * m[0] * (2.0 - sx) * (2.0 - sy) / 9.0);
        x[1] = log((2.0 * u1 + sx) / (1.0 - u1));
        x[2] = log((2.0 * u2 + sy) / (1.0 - u2));
        x[3] = -log(4.0);
      } else {
        for (int a = 0; a < 4; ++a) x[a] = mu[a * n + s];
      }
      it = or_fstar_newton_from(m, tol, 100, x, &r);
    }
    for (int a = 0; a < 4; ++a) mu[a * n + s] = x[a];
    iters[s] = it;
    if (it < 0) bad++;
  }
  return bad;
}
