/*
 * oracle.h -- plain, slow FP64 CPU reference for the Ehrenfests'-step
 * regularised lattice Boltzmann method of Brownlee, Gorban and Levesley,
 * "Stable simulation of fluid flow with high-Reynolds number using
 * Ehrenfests' steps" (2007), and for the learned warm start of its
 * entropic quasiequilibrium solve.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library; every constant below is
 * typed from the paper.
 *
 * Layout convention for population arrays: f[i][y][x], x fastest, no
 * padding, i in the paper's numbering (D1Q3: rest, left, right -- Sec. 4.1;
 * D2Q9: rest, E, N, W, S, NE, NW, SW, SE -- Sec. 4.2).
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_QE_POLY = 0, OR_QE_ENTROPIC_MM = 1, OR_QE_ENTROPIC_M = 2 };
enum { OR_BC_PERIODIC = 0, OR_BC_ZEROGRAD = 1, OR_BC_FREESLIP = 2, OR_BC_INLET_EQ = 3, OR_BC_OUTLET_EQ = 4,
       OR_BC_OUTLET_EQ_PREV = 5 };
enum { OR_COLL_LBGK = 0, OR_COLL_ELBM = 1 };

typedef struct {
  int32_t Q;          /* 3 or 9 */
  int32_t qe;         /* OR_QE_* */
  int32_t collision;  /* OR_COLL_* */
  int32_t pad0;
  int64_t nx, ny;
  double nu;          /* kinematic viscosity; beta = 1/(1+6 nu) */
  double delta;       /* Ehrenfests' tolerance on Delta S */
  int64_t k;          /* maximum number of Ehrenfests' steps per time step */
  int32_t bc[4];      /* west, east, south, north */
  double inlet_rho, inlet_u1, inlet_u2;
  int64_t solid_x0, solid_y0, solid_w, solid_h;
} or_cfg;

typedef struct {
  int64_t n_above;     /* sites with Delta S > delta */
  int64_t n_selected;  /* sites returned to quasiequilibrium */
  int64_t n_invalid;   /* sites with Delta S = +inf (negative f or f* <= 0) */
  int64_t n_fallback;  /* entropic f*_M sites that fell back to the closed form */
  double sums[4];      /* FP64 sums over fluid sites of rho, rho u1, rho u2, 2E (pre-collision) */
} or_step_info;

/* velocity set and weights */
int or_velocities(int Q, int32_t* vx, int32_t* vy, double* w);

/* moments M = (rho, rho u1, rho u2, 2E) of one site */
void or_moments(int Q, const double* f, double* M);

/* quasiequilibria */
void or_qe_poly(int Q, double rho, double u1, double u2, double* fs);
void or_qe_entropic_mm(int Q, double rho, double u1, double u2, double* fs);
int or_fstar_feasible(const double* M);
int or_fstar_newton(const double* M, double tol, int max_iter, double* mu, double* resid);
int or_fstar_newton_from(const double* M, double tol, int max_iter, double* mu, double* resid);
/* a whole moment field [4][n] (start 0 rest, 1 closed form, 2 mu on entry) */
int64_t or_fstar_field(const double* M, int64_t n, double tol, int start, double* mu, int32_t* iters);
int or_fstar_scalar(const double* M, double* mu);
/* one more Newton update from converged multipliers (kept if the residual does not grow) */
double or_fstar_polish(const double* M, double* mu);
void or_fstar_from_mu(const double* mu, double* fs);

/* nonequilibrium entropy (generalised Kullback form), long double */
long double or_delta_S(int Q, const double* f, const double* fs);

/* ELBM entropic involution parameter and its entropy function */
double or_elbm_alpha(int Q, const double* f, const double* fs);
long double or_elbm_H(int Q, const double* f, const double* fs, long double a);

/* whole lattice */
int or_init(const or_cfg* c, const double* rho0, const double* u0, const double* twoE0, double* f);
int or_step(const or_cfg* c, const double* f_in, double* f_out, double* dS,
            int64_t* sel, or_step_info* info);

int or_step_sites(const or_cfg* c, const double* f_in, const int64_t* sites, int64_t ns, const int64_t* sel,
                  int64_t nsel, double* out);
double or_site_dS(const or_cfg* c, const double* f_in, int64_t site);
/* sums over fluid sites of rho, rho u1, rho u2, 2E of a state f (long double accumulation) */
void or_sums(const or_cfg* c, const double* f, double* sums);

/* power spectrum of a real signal by the DFT's definition, bins 0..n/2 */
void or_dft_power(const double* x, int64_t n, double* power);
double or_dft_power_at(const double* x, int64_t n, int64_t k);

/* MLP 4 -> 64 -> 64 -> 4 (SiLU), parameters flat (see oracle.c) */
enum { OR_MLP_NPARAM = 4740 };
double or_mlp_forward(const double* p, const double* x, int64_t n, double* y, int bf16);
double or_mlp_loss_grad(const double* p, const double* x, const double* t, int64_t n,
                        double* grad, int bf16);
void or_adam_step(double* p, double* m, double* v, const double* g, int64_t n,
                  int64_t t, double lr, double b1, double b2, double eps);
double or_bf16_round(double x);

/* inputs (u1, u2, 2E/rho, |u|^2) and outputs (mu0 - ln rho, mu1, mu2, mu3)
   of the warm-start network, normalised with norm[16] (see oracle.c) */
void or_mlp_features(const double* M, int64_t n, const float* norm, double* X);
void or_mlp_targets(const double* M, const double* mu, int64_t n, const float* norm, double* T);
void or_mlp_unnormalise(const double* Y, int64_t n, const float* norm, double* out);

#ifdef __cplusplus
}
#endif
#endif
