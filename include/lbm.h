/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for lattice Boltzmann
 * steps regularised by Ehrenfests' steps (Brownlee, Gorban, Levesley,
 * "Stable simulation of fluid flow with high-Reynolds number using
 * Ehrenfests' steps", 2007), and for the entropic quasiequilibrium f*_M
 * with its learned (MLP) Newton warm start.
 *
 * Conventions for every entry point:
 *  - Return value: LBM_OK (0) or a negative LBM_E_* code.  No exception,
 *    abort or exit crosses this boundary.  lbm_last_error() returns a
 *    thread-local message for the last failure.
 *  - Arguments are validated on the host before any HIP call, so invalid
 *    arguments yield LBM_E_INVAL even on a machine without a GPU.
 *  - Array arguments marked "device" are device pointers owned by the
 *    caller; they must stay valid until the work queued on the context's
 *    stream has completed.  Arguments marked "host" are host memory.
 *  - Population arrays have the layout f[i][y][x] (x fastest, no padding)
 *    with the paper's numbering: D1Q3 (rest, left, right) from Sec. 4.1;
 *    D2Q9 (rest, E, N, W, S, NE, NW, SW, SE) from Sec. 4.2.  Their element
 *    type is float for LBM_FP32 contexts and double for LBM_FP64 contexts.
 *  - Site index s = x + nx * y.
 *  - A context is bound to one HIP stream and is not thread-safe.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_E_INVAL = -1,     /* invalid argument or configuration            */
  LBM_E_NOMEM = -2,     /* device allocation failed                     */
  LBM_E_DEVICE = -3,    /* a HIP call failed (no device, launch error)  */
  LBM_E_NONFINITE = -4, /* non-finite populations were detected         */
  LBM_E_NOCONV = -5,    /* f*_M solve left sites above the tolerance    */
  LBM_E_STATE = -6      /* call not valid in the context's state        */
};

enum { LBM_D1Q3 = 3, LBM_D2Q9 = 9 };
/* quasiequilibrium: polynomial (Sec. 4.1 / cited D2Q9 form), entropic with
   mass and momentum (closed forms of Sec. 4.1 and Sec. 4.2), entropic with
   mass, momentum and energy f*_M (Sec. 2 argmax with M = (rho, rho u, 2E)) */
enum { LBM_QE_POLY = 0, LBM_QE_ENTROPIC_MM = 1, LBM_QE_ENTROPIC_M = 2 };
enum { LBM_FP32 = 0, LBM_FP64 = 1 };
/* boundary rules (Sec. 4.2's channel); west/east accept PERIODIC, ZEROGRAD,
   INLET_EQ (incoming populations = quasiequilibrium of the inlet state),
   OUTLET_EQ (incoming populations = quasiequilibrium at the density and
   velocity of the new state of the penultimate column), OUTLET_EQ_PREV (the
   same at the density and velocity of that column one step earlier: the
   other reading of Sec. 4.2's outlet; both need nx >= 3 and the solid clear
   of both columns); south/north accept PERIODIC, ZEROGRAD, FREESLIP
   (specular reflection).  Corners take the west/east rule. */
enum { LBM_BC_PERIODIC = 0, LBM_BC_ZEROGRAD = 1, LBM_BC_FREESLIP = 2, LBM_BC_INLET_EQ = 3,
       LBM_BC_OUTLET_EQ = 4, LBM_BC_OUTLET_EQ_PREV = 5 };
/* collision: LBGK (eq. lbgkLB), f' = f + 2 beta (f* - f); or ELBM
   (eq. elbmLB), f' = f + alpha beta (f* - f) with alpha the nontrivial root
   of S(f + alpha (f* - f)) = S(f) by bisection to 1e-15 (entropic
   quasiequilibria only) */
enum { LBM_COLL_LBGK = 0, LBM_COLL_ELBM = 1 };
/* f*_M Newton start: isothermal rest state at the site density; the
   mass-momentum closed form of Sec. 4.2; the warm-start network; the
   multipliers already held (previous time step / contents of mu) */
enum { LBM_START_DEFAULT = 0, LBM_START_CLOSED_FORM = 1, LBM_START_MLP = 2, LBM_START_PREV = 3,
       LBM_START_PLAIN = 4 };
/* how the ranking and selection of a step are launched (the result is the
   same): MANY (and AUTO) spread them over many workgroups in three kernels,
   whose cost grows gently with the number of sites above delta; ONE runs
   them in a single workgroup in one kernel, about 3 us per step cheaper on
   a healthy lattice of ~10^5-10^6 sites but slow when many sites are above
   delta (an outbreak: ~0.3 ms per step at 5 x 10^5 screened sites) */
enum { LBM_SELECT_AUTO = 0, LBM_SELECT_ONE = 1, LBM_SELECT_MANY = 2 };

typedef struct lbm_ctx lbm_ctx; /* opaque; owns all device memory it allocates */
typedef struct lbm_mlp lbm_mlp; /* opaque; owns weights and optimiser state    */

typedef struct lbm_config {
  int32_t lattice;    /* LBM_D1Q3 or LBM_D2Q9                                   */
  int32_t qe;         /* LBM_QE_*                                               */
  int32_t precision;  /* LBM_FP32 or LBM_FP64: storage and collision arithmetic */
  int32_t collision;  /* LBM_COLL_*                                             */
  int64_t nx, ny;     /* lattice size; D1Q3 requires ny == 1; 2 <= nx <= 2^25, ny >= 1,
                         nx * ny < 2^32 - 1 */
  double nu;          /* kinematic viscosity > 0; beta = 1/(1 + 6 nu)           */
  double delta;       /* Ehrenfests' tolerance on Delta S, >= 0 (+inf: off)     */
  int32_t k;          /* at most k Ehrenfests' steps per time step, >= 0        */
  int32_t fstar_start;/* LBM_START_* (LBM_QE_ENTROPIC_M only): start of the
                         per-site Newton solve in every step; the residual
                         target is 1e-10 (FP32 contexts) or 1e-13 (FP64)      */
  int32_t bc[4];      /* west, east, south, north                               */
  int32_t select_mode;/* LBM_SELECT_*                                           */
  int32_t reserved;   /* 0                                                      */
  double inlet_rho;   /* inlet state for LBM_BC_INLET_EQ                        */
  double inlet_u[2];
  int64_t solid_x0, solid_y0, solid_w, solid_h; /* solid square (w == 0: none)  */
  const lbm_mlp* net; /* warm-start network for LBM_START_MLP, else NULL; must
                         outlive the context                                   */
  void* stream;       /* hipStream_t used for all work of the context (0: null) */
} lbm_config;

typedef struct lbm_es_stats {
  int64_t step;          /* time steps taken since init / set_populations          */
  int64_t n_above_delta; /* last step: sites with Delta S > delta                  */
  int64_t n_selected;    /* last step: sites returned to quasiequilibrium          */
  int64_t n_invalid;     /* last step: sites with Delta S = +inf (f < 0 or f* <= 0) */
  int64_t n_fallback;    /* last step, f*_M only: sites whose first Newton pass
                            missed the tolerance (re-solved by damped Newton from
                            the rest start) plus infeasible sites (closed form)   */
  int64_t total_selected;/* all steps since init                                   */
  int64_t nonfinite;     /* sticky: a step met non-finite populations              */
  int64_t newton_updates;/* last step, f*_M only: Newton updates over fluid sites  */
  int64_t n_failed;      /* last step, f*_M only: sites whose damped fallback also
                            missed the residual target (their last iterate is
                            used); 0 in a healthy run                             */
  double kth_dS;         /* last step: smallest selected Delta S (0 if none)       */
  double max_dS;         /* last step: largest Delta S above delta (0 if none)     */
  double mass, mom[2], energy; /* FP64 sums over fluid sites of rho, rho u1,
                                  rho u2, 2E of the current pre-collision state
                                  f(x, t) (conservation diagnostics)            */
  double max_resid;      /* last step, f*_M only: largest final residual
                            max_j |m_j(f*) - M_j| / rho of a converged site    */
} lbm_es_stats;

/* Fills *cfg with defaults: D2Q9, polynomial QE, FP32, LBGK, 64 x 64
   periodic, nu = 1e-3, delta = +inf, k = 0. */
void lbm_config_default(lbm_config* cfg);

/* Host-only validation of a configuration (no HIP call). */
int lbm_validate_config(const lbm_config* cfg);

/*
 * Creates a context and sets f(x, 0) to the configured quasiequilibrium of
 * the initial fields (Sec. 4.1 / Sec. 4.2 initial states).
 *   rho0  device double [ny][nx]
 *   u0    device double [2][ny][nx] (D1Q3: [1][ny][nx])
 *   twoE0 device double [ny][nx], 2E/rho, required for LBM_QE_ENTROPIC_M,
 *         else NULL
 * Solid sites hold zero populations.  *out receives the context.
 */
int lbm_init(const lbm_config* cfg, const double* rho0, const double* u0, const double* twoE0,
             lbm_ctx** out);

/*
 * Advances nsteps >= 0 time steps of eq. (ESLB) (LBGK with Ehrenfests'
 * steps; Sec. 3.2 "return to quasiequilibrium" for the selected sites):
 * per step, at every fluid site the moments, f* and
 * Delta S = sum_i f_i ln(f_i / f*_i) - f_i + f*_i (Sec. 3.3, +inf if some
 * f_i < 0 or f*_i <= 0) are computed; the sites with Delta S > delta are
 * ranked (largest first, ties by lower site index); at most k of them are
 * set to f*, all other fluid sites take f + 2 beta (f* - f); then free
 * flight with the boundary rules.  Queued asynchronously on the context's
 * stream; returns LBM_E_NONFINITE without queuing work once a previous
 * lbm_ehrenfest_stats call has reported non-finite values.
 */
int lbm_step(lbm_ctx* ctx, int64_t nsteps);

/*
 * Moments of the current pre-collision state f(x, t), FP64, into device
 * double arrays [ny][nx] (any pointer may be NULL): rho, rho u1, rho u2
 * (u is [2][ny][nx]: rho u1 then rho u2), 2E (Sec. 2, M = (rho, rho u1,
 * rho u2, 2E)).  Solid sites give zeros.
 */
int lbm_moments(lbm_ctx* ctx, double* rho, double* rhou, double* twoE);

/* Current pre-collision populations f(x, t) into a device array of the
   context's precision [Q][ny][nx]; zeros at solid sites. */
int lbm_get_populations(lbm_ctx* ctx, void* f);

/* Replaces the state by the pre-collision populations f(x, t) given in a
   device array [Q][ny][nx]; resets the sticky non-finite flag and the step
   counter; returns LBM_E_NONFINITE if f holds a non-finite value. */
int lbm_set_populations(lbm_ctx* ctx, const void* f);

/*
 * Synchronises the context's stream and reports the last step's
 * Ehrenfests' statistics (host *out).  sel (host, may be NULL) receives up
 * to sel_cap selected site indices in rank order (Delta S descending, site
 * ascending), sel_dS (host, may be NULL) their FP64 Delta S.
 */
int lbm_ehrenfest_stats(lbm_ctx* ctx, lbm_es_stats* out, int64_t* sel, double* sel_dS,
                        int64_t sel_cap);

/*
 * Synchronises and copies the last step's candidate list -- every fluid
 * site with FP64 Delta S > delta, in no particular order -- into host
 * arrays sites / dS of capacity cap; *n receives the full count.
 */
int lbm_candidates(lbm_ctx* ctx, int64_t* sites, double* dS, int64_t cap, int64_t* n);

/*
 * f*_M solver of a context (LBM_QE_ENTROPIC_M): residual target tol of the
 * FP64 phase (default 1e-10 in FP32 contexts, 1e-13 in FP64 contexts),
 * target tol32 of the FP32 phase (2e-6) and the update budgets of the first
 * pass (max32 = 16, max64 = 6).  A site that
 * misses tol within the budgets is solved again by the damped FP64 Newton
 * fallback from the rest start (Sec. 3.3's multipliers; counted in
 * lbm_es_stats.n_fallback).  Returns LBM_E_INVAL for another quasiequilibrium
 * or out-of-range values (0 <= max32 <= 64, 1 <= max64 <= 64); waits for the
 * context's stream (captured step graphs are rebuilt).
 */
int lbm_set_fstar_tolerance(lbm_ctx* ctx, double tol, double tol32, int32_t max32, int32_t max64);

/*
 * Kernel timing for measurement: with on != 0, lbm_step launches the step
 * kernels directly (no graph replay) and brackets each fused step kernel
 * with HIP events on the context's stream; lbm_kernel_time synchronises and
 * returns the summed duration in ms and the number of timed launches of
 * that kernel since timing was switched on.
 */
int lbm_set_timing(lbm_ctx* ctx, int on);
int lbm_kernel_time(lbm_ctx* ctx, double* ms, int64_t* launches);

/* Lattice geometry actually allocated: row pitch in elements (>= nx, a
   multiple of 64) and bytes of one population buffer. */
int lbm_layout(const lbm_ctx* ctx, int64_t* pitch, int64_t* buffer_bytes);

/* ------------------------------------------------------------------------
 * Shedding frequency (Sec. 4.2, Strouhal-Reynolds relationship): the
 * x-velocity is recorded at a monitoring point during the run and the
 * dominant frequency of the final quarter of the signal is taken from its
 * discrete Fourier transform; St = L f / u_inf.
 * ------------------------------------------------------------------------ */
/*
 * Monitoring point at fluid site (x, y): every later time step records the
 * density and velocity (rho, u1, u2) of the pre-collision state f(x, t) at
 * that site, FP64, into a ring of `capacity` samples owned by the context
 * (24 B per sample, device memory).  Replaces a previous probe and resets
 * its count; capacity 0 removes the probe.  LBM_E_INVAL for a site outside
 * the lattice or in the solid, or capacity outside [0, 2^31].
 */
int lbm_probe_set(lbm_ctx* ctx, int64_t x, int64_t y, int64_t capacity);
/* samples recorded since lbm_probe_set (host *total); 0 without a probe */
int lbm_probe_count(const lbm_ctx* ctx, int64_t* total);
/*
 * Copies the last n samples, oldest first, into out (device double [3][n]:
 * rho, then u1, then u2), queued on the context's stream.  n must not
 * exceed min(count, capacity) (LBM_E_INVAL); LBM_E_STATE without a probe.
 */
int lbm_probe_read(lbm_ctx* ctx, double* out, int64_t n);
/*
 * Power spectrum of a real signal x (device double [n], 1 <= n <= 2^31):
 * power[k] = |sum_j x_j exp(-2 pi i j k / n)|^2 for k = 0..n/2 (device
 * double [n/2 + 1]), FP64, queued on `stream` (hipStream_t, 0: null
 * stream).  peak (host, optional) receives the bin k >= 1 of largest power
 * (lowest k on ties; 0 when n == 1); asking for it synchronises the stream.
 */
int lbm_dft_power(const double* x, int64_t n, double* power, int64_t* peak, void* stream);

/* ------------------------------------------------------------------------
 * Entropic quasiequilibrium with the energy row, f*_M (Sec. 2: the
 * maximiser of S(f) = -sum_i f_i ln(f_i / W_i) (Sec. 3.3) under
 * m(f) = M = (rho, rho u1, rho u2, 2E); Sec. 3.3: ln f*_i = sum_j mu_j m_ji).
 * D2Q9 rows m_i = (1, vx_i, vy_i, |v_i|^2), so f*_i = exp(mu . m_i) with the
 * weights absorbed into mu.  Per site: Newton on the four multipliers, FP32
 * iterations then FP64 iterations until max_j |m_j(f*) - M_j| / rho <= tol
 * (default 1e-10); sites that miss it are re-solved by FP64 damped Newton
 * from the isothermal rest start.  M outside the realisable set
 * (2E/rho not in (|u1| + |u2|, 2), or rho <= 0) is reported as infeasible and
 * receives the mass-momentum closed form of Sec. 4.2.
 * ------------------------------------------------------------------------ */
typedef struct lbm_fstar lbm_fstar; /* opaque solver workspace (device scratch) */

typedef struct lbm_solve_stats {
  int64_t n;             /* sites solved                                        */
  int64_t n_infeasible;  /* M outside the realisable set                        */
  int64_t n_fallback;    /* sites re-solved by the damped FP64 Newton           */
  int64_t n_failed;      /* sites above tol after the fallback                  */
  int64_t iter_hist[16]; /* first-pass Newton updates (FP32 + FP64) per feasible
                            site; the last bin counts 15 or more                */
  double mean_fp32_iters, mean_fp64_iters; /* per feasible site, first pass    */
  double max_resid;      /* largest final residual of a converged site          */
} lbm_solve_stats;

/* Workspace for up to max_n sites, bound to a HIP stream. */
int lbm_fstar_create(int64_t max_n, void* stream, lbm_fstar** out);
/* Residual target tol (FP64), FP32-phase target tol32, iteration budgets. */
int lbm_fstar_set_tolerance(lbm_fstar* s, double tol, double tol32, int32_t max32, int32_t max64);
/*
 * Solves n sites.  M: device double [4][n] (rho, rho u1, rho u2, 2E);
 * mu: device double [4][n] output; start: LBM_START_DEFAULT (isothermal
 * rest state at the site density), LBM_START_CLOSED_FORM (mass-momentum
 * closed form of Sec. 4.2), LBM_START_MLP (network net), LBM_START_PREV
 * (the values in mu on entry) or LBM_START_PLAIN (no FP32 phase: plain FP64
 * Newton with Armijo damping from the rest start at every site, the
 * method's fallback, up to 200 updates: the reference solve of Sec. 3.3's
 * Newton that the other starts are compared with; solver only, not a time
 * step option); iters, status:
 * optional device uint8 [n] (Newton updates; 0 ok, 1 fallback ok,
 * 2 infeasible, 3 failed).  stats (host, optional) synchronises the stream
 * and returns LBM_E_NOCONV if any site failed; without stats the call is
 * asynchronous.
 */
int lbm_fstar_solve(lbm_fstar* s, const double* M, int64_t n, double* mu, int32_t start,
                    const lbm_mlp* net, uint8_t* iters, uint8_t* status, lbm_solve_stats* stats);
void lbm_fstar_free(lbm_fstar* s);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * lbm_fstar_solve without a solver handle.  Arguments as lbm_fstar_solve,
 * with the tolerances of lbm_fstar_set_tolerance given directly, queued on
 * `stream` (hipStream_t, 0: null stream); the same kernels, so the same
 * results bit for bit.  It allocates nothing: its scratch (failure counter,
 * statistics, failure list for up to LBM_FSTAR_STATIC_MAX_N sites, network
 * start for up to LBM_FSTAR_STATIC_MLP_MAX sites: 48 MB) is static device
 * memory of the library, one copy per GPU, held until the process ends,
 * and cleared by a kernel at the start of every call (no memset).  All calls
 * on one GPU share that scratch: calls that overlap in time on one GPU
 * (other streams, other threads) race and must not be issued.  Limits
 * (LBM_E_INVAL beyond them): n <= LBM_FSTAR_STATIC_MAX_N, and
 * n <= LBM_FSTAR_STATIC_MLP_MAX for LBM_START_MLP.  stats (host, optional)
 * synchronises the stream (and returns LBM_E_NOCONV if a site failed); with
 * stats == NULL the call only queues kernels.
 */
#define LBM_FSTAR_STATIC_MLP_MAX (1 << 20)
#define LBM_FSTAR_STATIC_MAX_N (1 << 23)
int lbm_fstar_solve_static(const double* M, int64_t n, double* mu, int32_t start, const lbm_mlp* net,
                           double tol, double tol32, int32_t max32, int32_t max64, uint8_t* iters,
                           uint8_t* status, lbm_solve_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Learned Newton warm start: MLP 4 -> 64 -> 64 -> 4, SiLU, BF16 matrix-core
 * products with FP32 accumulation, FP32 master weights and Adam moments.
 * Parameters (4740 floats): W1 [64][4], b1 [64], W2 [64][64], b2 [64],
 * W3 [4][64], b3 [4].  Features of a site: (u1, u2, 2E/rho, |u|^2),
 * x_k = (feature_k - in_shift_k) * in_scale_k; targets
 * (mu0 - ln rho, mu1, mu2, mu3), y_k = (target_k - out_shift_k) * out_scale_k.
 * ------------------------------------------------------------------------ */
/* Kaiming-uniform weights from SplitMix64(seed), zero biases, identity norm. */
int lbm_mlp_create(uint64_t seed, lbm_mlp** out);
int lbm_mlp_get_params(const lbm_mlp* net, float* host_params);
/* sets the weights (host float [4740]) and clears the Adam state */
int lbm_mlp_set_params(lbm_mlp* net, const float* host_params);
/* host float [16]: in_shift[4], in_scale[4], out_shift[4], out_scale[4] */
int lbm_mlp_set_norm(lbm_mlp* net, const float* norm16);
int lbm_mlp_get_norm(const lbm_mlp* net, float* norm16);
/* Y = net(X) for normalised features; X, Y device float [n][4] */
int lbm_mlp_forward(const lbm_mlp* net, const float* X, int64_t n, float* Y, void* stream);
/* gradient of L = (1/(4n)) sum (net(X) - T)^2 into device float grad[4740];
   loss (device float, optional) receives L; fixed-order (deterministic) */
int lbm_mlp_loss_grad(lbm_mlp* net, const float* X, const float* T, int64_t n, float* grad,
                      float* loss, void* stream);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) */
int lbm_mlp_adam_step(lbm_mlp* net, const float* grad, double lr, void* stream);
/* epochs of shuffled minibatch Adam over n samples (X, T device [n][4]);
   loss_per_epoch (host float [epochs], optional): mean batch loss */
int lbm_mlp_train(lbm_mlp* net, const float* X, const float* T, int64_t n, int32_t epochs,
                  int32_t batch, double lr, uint64_t shuffle_seed, float* loss_per_epoch,
                  void* stream);
/* Training pairs of the network from moments M and multipliers mu (device
   double [4][n] each, mu optional): X (device float [n][4]) receives the
   normalised features (u1, u2, 2E/rho, |u|^2) of M, the inputs that the
   warm start computes; T (device float [n][4], required with mu) the
   normalised targets (mu0 - ln rho, mu1, mu2, mu3).  Queued on stream. */
int lbm_mlp_pairs(const lbm_mlp* net, const double* M, const double* mu, int64_t n, float* X, float* T,
                  void* stream);
/* The network start of the f*_M solve (the same kernel as
   LBM_START_MLP): for moments M (device double [4][n]) writes warm (device
   float [4][n]) = (mu0 - ln rho, mu1, mu2, mu3), the network output on the
   features of M, unnormalised.  Queued on stream; n = 0 does nothing (M
   and warm may then be NULL); LBM_E_INVAL for a NULL net, NULL M or warm
   with n > 0, or n < 0. */
int lbm_mlp_warm_start(const lbm_mlp* net, const double* M, int64_t n, float* warm, void* stream);
void lbm_mlp_free(lbm_mlp* net);

/* sizeof(lbm_config) and sizeof(lbm_es_stats) as compiled into the
   library, so that bindings can check their struct layouts (host only). */
void lbm_struct_sizes(int64_t* config_size, int64_t* stats_size);

void lbm_free(lbm_ctx* ctx);
const char* lbm_strerror(int code);
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
