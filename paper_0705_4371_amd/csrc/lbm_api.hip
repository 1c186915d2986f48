// lbm_api.hip -- C ABI (include/lbm.h) over the gfx950 step kernels.
//
// Host-side responsibilities: argument validation before any HIP call,
// device buffers (two population buffers plus the Ehrenfests' ranking
// scratch), the buffer swap, hipGraph capture of runs of steps, optional HIP
// event timing of the fused step kernel, and the statistics read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_launch.hpp"
#include "lbm_internal.hpp"

using namespace lbm;

static thread_local char g_err[512] = "";

static int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

// shared with the f*_M / MLP entry points (lbm_api_learn.hip)
int lbm_internal_fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(LBM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// graph replays cover this many steps (even, so the state returns to its buffer)
static constexpr int GRAPH_STEPS = 32;

struct lbm_ctx {
  lbm_config cfg;
  StepArgs args;        // template; A/B set per launch
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;          // buffer holding the state
  bool canonical = true;
  int64_t step = 0;
  bool nonfinite_seen = false;
  // pinned host copy of the device words C_NONFINITE .. C_BADSTEP, refreshed
  // asynchronously after every lbm_step call (so that lbm_step can refuse
  // without waiting for the stream)
  volatile uint32_t* hflag = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
  double time_ms = 0.0;
  int64_t launches = 0;
  int64_t N = 0, pitch = 0, plane = 0;
  size_t elem = 4;
  // scratch
  uint32_t* ctr = nullptr;
  uint32_t* screen = nullptr;
  unsigned long long* part = nullptr;
  Cand* cand = nullptr;
  Cand* bnd = nullptr;
  uint32_t* hist = nullptr;
  uint32_t* sel = nullptr;
  double* sel_ds = nullptr;
  DevStats* st = nullptr;
  double* partials = nullptr;
  // f*_M quasiequilibrium (LBM_QE_ENTROPIC_M)
  double* Mbuf = nullptr;
  double* mubuf = nullptr;
  float* warm = nullptr;
  uint32_t* fctr = nullptr;
  uint32_t* fail_list = nullptr;
  FstarStats* fstats = nullptr;
  FstarArgs fa{};
  int fkind = START_REST;
  // monitoring point
  double* probe_buf = nullptr;
  unsigned long long* probe_n = nullptr;
  int64_t probe_total = 0;  // samples recorded since lbm_probe_set
};

extern "C" {

const char* lbm_last_error(void) { return g_err; }

const char* lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "ok";
    case LBM_E_INVAL: return "invalid argument";
    case LBM_E_NOMEM: return "device allocation failed";
    case LBM_E_DEVICE: return "HIP device error";
    case LBM_E_NONFINITE: return "non-finite populations";
    case LBM_E_NOCONV: return "f*_M solve did not converge";
    case LBM_E_STATE: return "invalid state for this call";
    default: return "unknown error";
  }
}

void lbm_config_default(lbm_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->lattice = LBM_D2Q9;
  c->qe = LBM_QE_POLY;
  c->precision = LBM_FP32;
  c->collision = LBM_COLL_LBGK;
  c->nx = 64;
  c->ny = 64;
  c->nu = 1e-3;
  c->delta = INFINITY;
  c->k = 0;
  c->fstar_start = LBM_START_DEFAULT;
  for (int i = 0; i < 4; ++i) c->bc[i] = LBM_BC_PERIODIC;
  c->inlet_rho = 1.0;
}

int lbm_validate_config(const lbm_config* c) {
  if (!c) return fail(LBM_E_INVAL, "config is NULL");
  if (c->lattice != LBM_D1Q3 && c->lattice != LBM_D2Q9)
    return fail(LBM_E_INVAL, "lattice must be LBM_D1Q3 (3) or LBM_D2Q9 (9), got %d", c->lattice);
  if (c->qe != LBM_QE_POLY && c->qe != LBM_QE_ENTROPIC_MM && c->qe != LBM_QE_ENTROPIC_M)
    return fail(LBM_E_INVAL, "qe must be one of LBM_QE_*, got %d", c->qe);
  if (c->qe == LBM_QE_ENTROPIC_M) {
    if (c->lattice != LBM_D2Q9) return fail(LBM_E_INVAL, "LBM_QE_ENTROPIC_M needs D2Q9");
    if (c->fstar_start != LBM_START_DEFAULT && c->fstar_start != LBM_START_CLOSED_FORM &&
        c->fstar_start != LBM_START_MLP && c->fstar_start != LBM_START_PREV)
      return fail(LBM_E_INVAL, "fstar_start must be one of LBM_START_*");
    if (c->fstar_start == LBM_START_MLP && !c->net) return fail(LBM_E_INVAL, "LBM_START_MLP needs cfg->net");
  }
  if (c->precision != LBM_FP32 && c->precision != LBM_FP64)
    return fail(LBM_E_INVAL, "precision must be LBM_FP32 or LBM_FP64, got %d", c->precision);
  if (c->collision != LBM_COLL_LBGK && c->collision != LBM_COLL_ELBM)
    return fail(LBM_E_INVAL, "collision must be LBM_COLL_LBGK or LBM_COLL_ELBM, got %d", c->collision);
  if (c->collision == LBM_COLL_ELBM && c->qe == LBM_QE_POLY)
    return fail(LBM_E_INVAL, "ELBM needs an entropic quasiequilibrium (LBM_QE_ENTROPIC_MM or _M)");
  if (c->nx < 2 || c->ny < 1) return fail(LBM_E_INVAL, "need nx >= 2 and ny >= 1 (got %lld x %lld)",
                                         (long long)c->nx, (long long)c->ny);
  if (c->lattice == LBM_D1Q3 && c->ny != 1) return fail(LBM_E_INVAL, "D1Q3 requires ny == 1");
  if (c->nx > (int64_t)1 << 25 || c->ny > (int64_t)1 << 31 || c->nx * c->ny >= (int64_t)0xFFFFFFFFll)
    return fail(LBM_E_INVAL, "lattice too large: nx <= 2^25 and nx * ny below 2^32 - 1 are required");
  if (!(c->nu >= 0.0)) return fail(LBM_E_INVAL, "nu must be >= 0 (got %g)", c->nu);
  if (!(c->delta >= 0.0)) return fail(LBM_E_INVAL, "delta must be >= 0 or +inf (got %g)", c->delta);
  if (c->k < 0) return fail(LBM_E_INVAL, "k must be >= 0 (got %d)", c->k);
  if (c->select_mode != LBM_SELECT_AUTO && c->select_mode != LBM_SELECT_ONE && c->select_mode != LBM_SELECT_MANY)
    return fail(LBM_E_INVAL, "select_mode must be one of LBM_SELECT_* (got %d)", c->select_mode);
  for (int s = 0; s < 4; ++s) {
    const int b = c->bc[s];
    const bool ok = s < 2 ? (b == LBM_BC_PERIODIC || b == LBM_BC_ZEROGRAD || b == LBM_BC_INLET_EQ ||
                             b == LBM_BC_OUTLET_EQ || b == LBM_BC_OUTLET_EQ_PREV)
                          : (b == LBM_BC_PERIODIC || b == LBM_BC_ZEROGRAD || b == LBM_BC_FREESLIP);
    if (!ok) return fail(LBM_E_INVAL, "boundary rule %d not allowed on side %d", b, s);
  }
  if ((c->bc[0] == LBM_BC_PERIODIC) != (c->bc[1] == LBM_BC_PERIODIC))
    return fail(LBM_E_INVAL, "west and east must both be periodic or both not");
  if ((c->bc[2] == LBM_BC_PERIODIC) != (c->bc[3] == LBM_BC_PERIODIC))
    return fail(LBM_E_INVAL, "south and north must both be periodic or both not");
  if (c->bc[2] != LBM_BC_PERIODIC && c->ny < 2)
    return fail(LBM_E_INVAL, "non-periodic south/north rules need ny >= 2");
  if (c->lattice == LBM_D1Q3 && c->bc[2] != LBM_BC_PERIODIC)
    return fail(LBM_E_INVAL, "D1Q3 has no y direction: south/north must be LBM_BC_PERIODIC");
  if ((c->bc[0] == LBM_BC_INLET_EQ || c->bc[1] == LBM_BC_INLET_EQ)) {
    if (!(c->inlet_rho > 0.0) || !std::isfinite(c->inlet_u[0]) || !std::isfinite(c->inlet_u[1]))
      return fail(LBM_E_INVAL, "inlet state must have rho > 0 and finite velocity");
    if (c->qe == LBM_QE_ENTROPIC_MM && (std::fabs(c->inlet_u[0]) >= 1.0 || std::fabs(c->inlet_u[1]) >= 1.0))
      return fail(LBM_E_INVAL, "entropic inlet state needs |u_j| < 1");
  }
  const bool out_w = c->bc[0] == LBM_BC_OUTLET_EQ || c->bc[0] == LBM_BC_OUTLET_EQ_PREV;
  const bool out_e = c->bc[1] == LBM_BC_OUTLET_EQ || c->bc[1] == LBM_BC_OUTLET_EQ_PREV;
  if ((out_w || out_e) && c->nx < 3) return fail(LBM_E_INVAL, "the outlet rule needs nx >= 3");
  if (c->solid_w < 0 || c->solid_h < 0) return fail(LBM_E_INVAL, "solid size must be >= 0");
  if (c->solid_w > 0 && c->solid_h > 0) {
    if (c->lattice == LBM_D1Q3) return fail(LBM_E_INVAL, "solid obstacles need D2Q9");
    if (c->solid_x0 < 0 || c->solid_y0 < 0 || c->solid_x0 + c->solid_w > c->nx ||
        c->solid_y0 + c->solid_h > c->ny)
      return fail(LBM_E_INVAL, "solid square must lie inside the lattice");
    if ((out_w && c->solid_x0 < 2) || (out_e && c->solid_x0 + c->solid_w > c->nx - 2))
      return fail(LBM_E_INVAL, "the solid must keep clear of an outlet column and its penultimate column");
  }
  return LBM_OK;
}

static void qe_host(int Q, int qe, double rho, double ux, double uy, double* fs) {
  if (qe == LBM_QE_POLY) {
    if (Q == 3) {
      fs[0] = (2.0 * rho / 3.0) * (1.0 - 1.5 * ux * ux);
      fs[1] = (rho / 6.0) * (1.0 - 3.0 * ux + 3.0 * ux * ux);
      fs[2] = (rho / 6.0) * (1.0 + 3.0 * ux + 3.0 * ux * ux);
    } else {
      static const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
      const double uu = ux * ux + uy * uy;
      for (int i = 0; i < 9; ++i) {
        const double w = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        const double cu = cx[i] * ux + cy[i] * uy;
        fs[i] = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      }
    }
  } else {
    const double sx = std::sqrt(1.0 + 3.0 * ux * ux), X = (2.0 * ux + sx) / (1.0 - ux);
    if (Q == 3) {
      fs[0] = rho * (2.0 - sx) * (2.0 / 3.0);
      fs[1] = rho * (2.0 - sx) / 6.0 / X;
      fs[2] = rho * (2.0 - sx) / 6.0 * X;
    } else {
      static const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
      const double sy = std::sqrt(1.0 + 3.0 * uy * uy), Y = (2.0 * uy + sy) / (1.0 - uy);
      for (int i = 0; i < 9; ++i) {
        const double w = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        fs[i] = rho * w * (2.0 - sx) * (2.0 - sy) * std::pow(X, cx[i]) * std::pow(Y, cy[i]);
      }
    }
  }
}

static void ctx_release(lbm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (int p = 0; p < 2; ++p) {
    if (c->gexec[p]) (void)hipGraphExecDestroy(c->gexec[p]);
    if (c->graph[p]) (void)hipGraphDestroy(c->graph[p]);
  }
  for (auto& e : c->ev_used) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  for (auto& e : c->ev_free) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  void* ptrs[] = {c->buf[0], c->buf[1], c->ctr, c->part, c->screen, c->cand, c->bnd, c->hist, c->sel, c->sel_ds,
                  c->st, c->partials, c->Mbuf, c->mubuf, c->warm, c->fctr, c->fail_list, c->fstats,
                  c->probe_buf, c->probe_n};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->hflag) (void)hipHostFree((void*)c->hflag);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
}

static StepArgs args_for(const lbm_ctx* c, int src, int dst) {
  StepArgs a = c->args;
  a.A = c->buf[src];
  a.B = c->buf[dst];
  a.dst = dst;
  return a;
}

// After a step met non-finite values the step kernels stop (see
// raise_nonfinite): the buffer that step read holds the last finite state.
// Synchronises, and if the device has halted, makes that buffer (and its
// layout and step number) the context's state; returns whether it had.
static int take_halt(lbm_ctx* c, bool* halted) {
  *halted = c->nonfinite_seen;
  if (c->nonfinite_seen) return LBM_OK;
  uint32_t w[C_COUNT];
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemcpy(w, c->ctr, sizeof(w), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(LBM_E_DEVICE, "halt check: %s", hipGetErrorString(e));
  if (!w[C_NONFINITE]) return LBM_OK;
  const uint32_t tag = w[C_NONFINITE] - 1u;
  c->cur = 1 - (int)(tag & 1u);
  c->canonical = (tag & 2u) != 0u;
  c->step = (int64_t)w[C_BADSTEP] - 1;
  if (c->probe_n) {
    unsigned long long pn = 0;
    e = hipMemcpy(&pn, c->probe_n, sizeof(pn), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(LBM_E_DEVICE, "halt check: %s", hipGetErrorString(e));
    c->probe_total = (int64_t)pn;
  }
  c->nonfinite_seen = true;
  *halted = true;
  return LBM_OK;
}

// one time step from buffer src into buffer dst.  For the f*_M
// quasiequilibrium with a network start the moments of every site go to
// memory, the network and the Newton solve run, then the step kernel; the
// other starts solve and collide in one kernel.
static hipError_t step_once(const lbm_ctx* c, int src, int dst, bool pull, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1) {
  const StepArgs a = args_for(c, src, dst);
  if (c->cfg.qe == LBM_QE_ENTROPIC_M) {
    if (c->fkind != START_WARM) return launch_fstep(a, c->fa, c->fkind, pull, s, e0, e1);
    hipError_t e = launch_moments_M(a, pull, s);
    if (e == hipSuccess) e = launch_mlp_warm(c->cfg.net->params, c->cfg.net->norm, c->Mbuf, c->N, c->warm, s);
    if (e == hipSuccess) e = launch_fstar(c->fa, c->fkind, s);
    if (e != hipSuccess) return e;
  }
  return launch_step(a, pull, s, e0, e1);
}

int lbm_init(const lbm_config* cfg, const double* rho0, const double* u0, const double* twoE0,
             lbm_ctx** out) {
  if (!out) return fail(LBM_E_INVAL, "out is NULL");
  *out = nullptr;
  int rc = lbm_validate_config(cfg);
  if (rc) return rc;
  if (!rho0 || !u0) return fail(LBM_E_INVAL, "rho0 and u0 are required");
  if (cfg->qe == LBM_QE_ENTROPIC_M && !twoE0) return fail(LBM_E_INVAL, "twoE0 is required for f*_M");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(LBM_E_DEVICE, "no HIP device");

  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_E_NOMEM, "host allocation failed");
  c->cfg = *cfg;
  const int Q = cfg->lattice;
  c->elem = cfg->precision == LBM_FP64 ? 8 : 4;
  c->N = cfg->nx * cfg->ny;
  c->pitch = (cfg->nx + 63) / 64 * 64;
  c->plane = c->pitch * cfg->ny;
  c->stream = (hipStream_t)cfg->stream;

  StepArgs& a = c->args;
  std::memset(&a, 0, sizeof(a));
  Geom& g = a.g;
  g.nx = cfg->nx;
  g.ny = cfg->ny;
  g.pitch = c->pitch;
  g.plane = c->plane;
  g.inv_nx = 1.0 / (double)cfg->nx;
  g.inv_pitch = 1.0 / (double)c->pitch;
  for (int s = 0; s < 4; ++s) g.bc[s] = cfg->bc[s];
  if (cfg->solid_w > 0 && cfg->solid_h > 0) {
    g.sx0 = cfg->solid_x0;
    g.sy0 = cfg->solid_y0;
    g.sx1 = cfg->solid_x0 + cfg->solid_w;
    g.sy1 = cfg->solid_y0 + cfg->solid_h;
  } else {
    g.sx0 = g.sx1 = g.sy0 = g.sy1 = -4;
  }
  double feq[9] = {0};
  if (cfg->bc[0] == LBM_BC_INLET_EQ || cfg->bc[1] == LBM_BC_INLET_EQ)
    qe_host(Q, cfg->qe, cfg->inlet_rho, cfg->inlet_u[0], Q == 9 ? cfg->inlet_u[1] : 0.0, feq);
  for (int i = 0; i < 9; ++i) g.feq_in[i] = feq[i];
  g.beta2 = 2.0 / (1.0 + 6.0 * cfg->nu);
  g.delta = cfg->delta;
  g.ds_on = std::isinf(cfg->delta) ? 0 : 1;
  g.out_qe = cfg->qe == LBM_QE_POLY ? QE_POLY : QE_ENTROPIC_MM;
  // at most N sites can be selected: "fewer than k: all of them"
  g.kmax = (int32_t)std::min<int64_t>(cfg->k, c->N);
  // FP32 screen threshold delta (1 - 1e-2) - 64 eps32 sqrt(delta rho)
  const double dclamp = std::min(cfg->delta, 3.0e38);
  a.thr_a = (float)(0.99 * dclamp);
  a.thr_b = (float)(64.0 * std::ldexp(1.0, -24) * std::sqrt(dclamp));
  a.ntx = (cfg->nx + STEP_TX - 1) / STEP_TX;
  a.nblocks = a.ntx * cfg->ny;
  a.prec = cfg->precision;
  a.coll = cfg->collision;
  a.Q = Q;
  a.qe = cfg->qe;
  a.probe = -1;
  a.probe_cap = 1;
  a.one_wg = cfg->select_mode == LBM_SELECT_ONE;

  const size_t bytes = (size_t)Q * (size_t)c->plane * c->elem;
  const size_t ncap = (size_t)c->N;
  const size_t kcap = (size_t)std::max<int64_t>(g.kmax, 1);
#define ALLOC(ptr, nbytes)                                                              \
  do {                                                                                \
    if (hipMalloc((void**)&(ptr), (nbytes)) != hipSuccess) {                          \
      ctx_release(c);                                                                 \
      return fail(LBM_E_NOMEM, "hipMalloc of %zu bytes failed", (size_t)(nbytes));    \
    }                                                                                 \
  } while (0)
  ALLOC(c->buf[0], bytes);
  ALLOC(c->buf[1], bytes);
  ALLOC(c->ctr, sizeof(uint32_t) * C_COUNT);
  ALLOC(c->screen, sizeof(uint32_t) * ncap);
  ALLOC(c->part, sizeof(unsigned long long) * 2 * PART_BLOCKS);
  ALLOC(c->cand, sizeof(Cand) * ncap);
  ALLOC(c->bnd, sizeof(Cand) * ncap);
  ALLOC(c->hist, sizeof(uint32_t) * HIST_WORDS);
  ALLOC(c->sel, sizeof(uint32_t) * kcap);
  ALLOC(c->sel_ds, sizeof(double) * kcap);
  ALLOC(c->st, sizeof(DevStats));
  ALLOC(c->partials, sizeof(double) * 4 * SUM_BLOCKS);
  {
    void* hp = nullptr;
    if (hipHostMalloc(&hp, 4 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
      ctx_release(c);
      return fail(LBM_E_NOMEM, "pinned host word");
    }
    c->hflag = (volatile uint32_t*)hp;
    for (int i = 0; i < 4; ++i) c->hflag[i] = 0u;
  }
  if (cfg->qe == LBM_QE_ENTROPIC_M) {
    ALLOC(c->Mbuf, sizeof(double) * 4 * ncap);
    ALLOC(c->mubuf, sizeof(double) * 4 * ncap);
    ALLOC(c->fctr, 16);
    ALLOC(c->fail_list, sizeof(uint32_t) * ncap);
    ALLOC(c->fstats, sizeof(FstarStats) * FSTAR_STAT_SLOTS);
    if (cfg->fstar_start == LBM_START_MLP) ALLOC(c->warm, sizeof(float) * 4 * ncap);
    FstarArgs& f = c->fa;
    f.M = c->Mbuf;
    f.n = c->N;
    f.mu = c->mubuf;
    f.prod = 1;  // the time step keeps the product-form state, not the multipliers
    f.warm = c->warm;
    f.iters = nullptr;
    f.status = nullptr;
    f.ctr = c->fctr;
    f.fail_list = c->fail_list;
    f.stats = c->fstats;
    f.tol = cfg->precision == LBM_FP64 ? 1e-13 : 1e-10;
    f.tol32 = 2e-6f;
    f.max32 = 16;
    f.max64 = 6;
    // FP64 contexts carry every solve to round-off (one more Newton update)
    f.polish = cfg->precision == LBM_FP64 ? 1 : 0;
    c->fkind = cfg->fstar_start == LBM_START_CLOSED_FORM ? START_CLOSED
               : cfg->fstar_start == LBM_START_MLP        ? START_WARM
               : cfg->fstar_start == LBM_START_PREV       ? START_PREV
                                                          : START_REST;
    // the fused step's grid: the workgroups the device holds at once
    a.fgrid[0] = a.fgrid[1] = 0;
    if (c->fkind != START_WARM) {
      const bool elbm = cfg->collision == LBM_COLL_ELBM;
      a.fgrid[0] = fstep_resident(cfg->precision, c->fkind, false, elbm);
      a.fgrid[1] = fstep_resident(cfg->precision, c->fkind, true, elbm);
    }
    a.Mbuf = c->Mbuf;
    a.mu = c->mubuf;
  }
#undef ALLOC
  a.ctr = c->ctr;
  a.screen = c->screen;
  a.part = c->part;
  a.cand = c->cand;
  a.bnd = c->bnd;
  a.hist = c->hist;
  a.sel = c->sel;
  a.sel_ds = c->sel_ds;
  a.st = c->st;
  a.partials = c->partials;

  hipError_t e = launch_clear(args_for(c, 0, 0), c->stream);
  if (cfg->qe == LBM_QE_ENTROPIC_M) {
    // f(x, 0) = f*_M of the initial moments (rest start, then the fallback)
    if (e == hipSuccess) e = launch_init_M_moments(args_for(c, 1, 0), rho0, u0, twoE0, c->stream);
    if (e == hipSuccess) e = launch_fstar(c->fa, START_REST, c->stream);
    if (e == hipSuccess) e = launch_init_M_pops(args_for(c, 1, 0), c->stream);
  } else if (e == hipSuccess) {
    e = launch_init(args_for(c, 1, 0), rho0, u0, twoE0, c->stream);
  }
  if (e != hipSuccess) {
    ctx_release(c);
    return fail(LBM_E_DEVICE, "init kernels: %s", hipGetErrorString(e));
  }
  c->cur = 0;
  c->canonical = true;
  *out = c;
  return LBM_OK;
}

void lbm_free(lbm_ctx* ctx) { ctx_release(ctx); }

void lbm_struct_sizes(int64_t* config_size, int64_t* stats_size) {
  if (config_size) *config_size = (int64_t)sizeof(lbm_config);
  if (stats_size) *stats_size = (int64_t)sizeof(lbm_es_stats);
}

static int step_run(lbm_ctx* c, int64_t n);

static int ensure_graph(lbm_ctx* c, int from) {
  if (c->gexec[from]) return LBM_OK;
  if (!c->cap) HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  int s = from;
  hipError_t err = hipSuccess;
  for (int t = 0; t < GRAPH_STEPS && err == hipSuccess; ++t) {
    err = step_once(c, s, 1 - s, true, c->cap, nullptr, nullptr);
    s = 1 - s;
  }
  hipGraph_t gr = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->cap, &gr);
  if (err != hipSuccess || e2 != hipSuccess) {
    if (gr) (void)hipGraphDestroy(gr);
    return fail(LBM_E_DEVICE, "graph capture: %s", hipGetErrorString(err != hipSuccess ? err : e2));
  }
  c->graph[from] = gr;
  HIPCHK(hipGraphInstantiate(&c->gexec[from], gr, nullptr, nullptr, 0));
  return LBM_OK;
}

static int timed_launch(lbm_ctx* c, bool pull) {
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (!c->ev_free.empty()) {
    ev = c->ev_free.back();
    c->ev_free.pop_back();
  } else {
    HIPCHK(hipEventCreate(&ev.first));
    HIPCHK(hipEventCreate(&ev.second));
  }
  c->ev_used.push_back(ev);
  HIPCHK(step_once(c, c->cur, 1 - c->cur, pull, c->stream, ev.first, ev.second));
  return LBM_OK;
}

static int drain_events(lbm_ctx* c) {
  if (c->ev_used.empty()) return LBM_OK;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (auto& e : c->ev_used) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e.first, e.second));
    c->time_ms += ms;
    c->launches++;
    c->ev_free.push_back(e);
  }
  c->ev_used.clear();
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  if (n < 0) return fail(LBM_E_INVAL, "nsteps must be >= 0");
  int rc;
  if (!c->nonfinite_seen && c->hflag[0] != 0u) {
    bool h = false;
    if ((rc = take_halt(c, &h))) return rc;
  }
  if (c->nonfinite_seen)
    return fail(LBM_E_NONFINITE, "step %lld met non-finite populations (the state of step %lld is kept); "
                "set new populations", (long long)(c->step + 1), (long long)c->step);
  rc = step_run(c, n);
  // refresh the host copy of the halt words behind the queued steps
  HIPCHK(hipMemcpyAsync((void*)c->hflag, c->ctr + C_NONFINITE, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                        c->stream));
  return rc;
}

static int step_run(lbm_ctx* c, int64_t n) {
  int rc;
  while (n > 0) {
    if (c->canonical || c->timing) {
      const bool pull = !c->canonical;
      if (c->timing) {
        if ((rc = timed_launch(c, pull))) return rc;
        if (c->ev_used.size() >= 1024 && (rc = drain_events(c))) return rc;
      } else {
        HIPCHK(step_once(c, c->cur, 1 - c->cur, pull, c->stream, nullptr, nullptr));
      }
      c->cur = 1 - c->cur;
      c->canonical = false;
      c->step++;
      c->probe_total++;
      n--;
      continue;
    }
    if (n >= GRAPH_STEPS) {
      if ((rc = ensure_graph(c, c->cur))) return rc;
      HIPCHK(hipGraphLaunch(c->gexec[c->cur], c->stream));
      c->step += GRAPH_STEPS;
      c->probe_total += GRAPH_STEPS;
      n -= GRAPH_STEPS;
      continue;
    }
    HIPCHK(step_once(c, c->cur, 1 - c->cur, true, c->stream, nullptr, nullptr));
    c->cur = 1 - c->cur;
    c->step++;
    c->probe_total++;
    n--;
  }
  return LBM_OK;
}

int lbm_get_populations(lbm_ctx* c, void* f) {
  if (!c || !f) return fail(LBM_E_INVAL, "ctx and f are required");
  bool h;
  int rc = take_halt(c, &h);
  if (rc) return rc;
  HIPCHK(launch_get(args_for(c, c->cur, c->cur), !c->canonical, f, c->stream));
  return LBM_OK;
}

int lbm_set_populations(lbm_ctx* c, const void* f) {
  if (!c || !f) return fail(LBM_E_INVAL, "ctx and f are required");
  HIPCHK(launch_clear(args_for(c, c->cur, c->cur), c->stream));
  HIPCHK(launch_set(args_for(c, c->cur, c->cur), f, c->stream));
  uint32_t flags[C_COUNT];
  HIPCHK(hipMemcpyAsync(flags, c->ctr, sizeof(flags), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->canonical = true;
  c->step = 0;
  c->nonfinite_seen = false;
  for (int i = 0; i < 4; ++i) c->hflag[i] = 0u;
  if (flags[C_SETBAD]) {
    c->nonfinite_seen = true;
    return fail(LBM_E_NONFINITE, "populations hold non-finite values");
  }
  return LBM_OK;
}

int lbm_moments(lbm_ctx* c, double* rho, double* rhou, double* e2) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  bool h;
  int rc = take_halt(c, &h);
  if (rc) return rc;
  HIPCHK(launch_moments(args_for(c, c->cur, c->cur), !c->canonical, rho, rhou, e2, c->stream));
  return LBM_OK;
}

int lbm_ehrenfest_stats(lbm_ctx* c, lbm_es_stats* out, int64_t* sel, double* sel_dS, int64_t cap) {
  if (!c || !out) return fail(LBM_E_INVAL, "ctx and out are required");
  if (cap < 0) return fail(LBM_E_INVAL, "sel_cap must be >= 0");
  bool halted;
  int rc = take_halt(c, &halted);
  if (rc) return rc;
  HIPCHK(launch_sums(args_for(c, c->cur, c->cur), !c->canonical, c->stream));
  DevStats st;
  uint32_t ctr[C_COUNT];
  HIPCHK(hipMemcpyAsync(&st, c->st, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(ctr, c->ctr, sizeof(ctr), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::memset(out, 0, sizeof(*out));
  out->step = c->step;
  out->n_above_delta = (int64_t)st.n_above;
  out->n_selected = (int64_t)st.n_sel;
  out->n_invalid = (int64_t)st.n_invalid;
  out->n_fallback = 0;
  out->newton_updates = 0;
  if (c->cfg.qe == LBM_QE_ENTROPIC_M) {
    FstarStats slots[FSTAR_STAT_SLOTS];
    HIPCHK(hipMemcpy(slots, c->fstats, sizeof(slots), hipMemcpyDeviceToHost));
    const FstarStats fs = fstar_stats_total(slots);
    out->n_fallback = (int64_t)(fs.fallback + fs.infeasible);
    out->newton_updates = (int64_t)(fs.sum32 + fs.sum64);
    out->n_failed = (int64_t)fs.failed;
    std::memcpy(&out->max_resid, &fs.maxres_bits, sizeof(double));
  }
  out->total_selected = (int64_t)st.total_sel;
  out->nonfinite = halted ? 1 : 0;
  out->kth_dS = st.kth;
  out->max_dS = st.max;
  out->mass = st.sums[0];
  out->mom[0] = st.sums[1];
  out->mom[1] = st.sums[2];
  out->energy = st.sums[3];
  if ((sel || sel_dS) && st.n_sel > 0 && cap > 0) {
    std::vector<uint32_t> s(st.n_sel);
    std::vector<double> d(st.n_sel);
    HIPCHK(hipMemcpy(s.data(), c->sel, sizeof(uint32_t) * st.n_sel, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(d.data(), c->sel_ds, sizeof(double) * st.n_sel, hipMemcpyDeviceToHost));
    std::vector<size_t> order(st.n_sel);
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) {
      if (d[x] != d[y]) return d[x] > d[y];
      return s[x] < s[y];
    });
    const int64_t m = std::min<int64_t>(cap, (int64_t)st.n_sel);
    for (int64_t i = 0; i < m; ++i) {
      if (sel) sel[i] = s[order[i]];
      if (sel_dS) sel_dS[i] = d[order[i]];
    }
  }
  return LBM_OK;
}

int lbm_candidates(lbm_ctx* c, int64_t* sites, double* dS, int64_t cap, int64_t* n) {
  if (!c || !n) return fail(LBM_E_INVAL, "ctx and n are required");
  if (cap < 0) return fail(LBM_E_INVAL, "cap must be >= 0");
  DevStats st;
  HIPCHK(hipMemcpyAsync(&st, c->st, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *n = (int64_t)st.n_above;
  // the entries of the screened sites, Delta S < 0 marking non-candidates
  if (cap > 0 && st.n_above > 0) {
    std::vector<Cand> v((size_t)st.n_screened);
    HIPCHK(hipMemcpy(v.data(), c->cand, sizeof(Cand) * v.size(), hipMemcpyDeviceToHost));
    int64_t m = 0;
    for (size_t i = 0; i < v.size() && m < cap; ++i) {
      if (!(v[i].ds >= 0.0)) continue;
      if (sites) sites[m] = v[i].site;
      if (dS) dS[m] = v[i].ds;
      ++m;
    }
  }
  return LBM_OK;
}

int lbm_set_timing(lbm_ctx* c, int on) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  int rc = drain_events(c);
  if (rc) return rc;
  c->timing = on != 0;
  c->time_ms = 0.0;
  c->launches = 0;
  return LBM_OK;
}

int lbm_kernel_time(lbm_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return fail(LBM_E_INVAL, "ctx, ms and launches are required");
  int rc = drain_events(c);
  if (rc) return rc;
  *ms = c->time_ms;
  *launches = c->launches;
  return LBM_OK;
}

// the captured graphs hold the kernel arguments: drop them when those change
static int drop_graphs(lbm_ctx* c) {
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int p = 0; p < 2; ++p) {
    if (c->gexec[p]) (void)hipGraphExecDestroy(c->gexec[p]);
    if (c->graph[p]) (void)hipGraphDestroy(c->graph[p]);
    c->gexec[p] = nullptr;
    c->graph[p] = nullptr;
  }
  return LBM_OK;
}

int lbm_set_fstar_tolerance(lbm_ctx* c, double tol, double tol32, int32_t max32, int32_t max64) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  if (c->cfg.qe != LBM_QE_ENTROPIC_M) return fail(LBM_E_INVAL, "the context does not use LBM_QE_ENTROPIC_M");
  if (!(tol > 0.0) || !(tol32 > 0.0) || max32 < 0 || max64 < 1 || max32 > 64 || max64 > 64)
    return fail(LBM_E_INVAL, "need tol > 0, tol32 > 0, 0 <= max32 <= 64, 1 <= max64 <= 64");
  int rc = drop_graphs(c);
  if (rc) return rc;
  c->fa.tol = tol;
  c->fa.tol32 = (float)tol32;
  c->fa.max32 = max32;
  c->fa.max64 = max64;
  return LBM_OK;
}

int lbm_probe_set(lbm_ctx* c, int64_t x, int64_t y, int64_t capacity) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  if (capacity < 0 || capacity > ((int64_t)1 << 31))
    return fail(LBM_E_INVAL, "capacity must be in [0, 2^31] (got %lld)", (long long)capacity);
  const lbm_config& cf = c->cfg;
  if (capacity > 0) {
    if (x < 0 || x >= cf.nx || y < 0 || y >= cf.ny)
      return fail(LBM_E_INVAL, "probe (%lld, %lld) outside the lattice", (long long)x, (long long)y);
    if (cf.solid_w > 0 && cf.solid_h > 0 && x >= cf.solid_x0 && x < cf.solid_x0 + cf.solid_w &&
        y >= cf.solid_y0 && y < cf.solid_y0 + cf.solid_h)
      return fail(LBM_E_INVAL, "probe (%lld, %lld) lies in the solid", (long long)x, (long long)y);
  }
  int rc = drop_graphs(c);
  if (rc) return rc;
  if (c->probe_buf) (void)hipFree(c->probe_buf);
  if (c->probe_n) (void)hipFree(c->probe_n);
  c->probe_buf = nullptr;
  c->probe_n = nullptr;
  c->args.probe = -1;
  c->args.probe_buf = nullptr;
  c->args.probe_n = nullptr;
  c->args.probe_cap = 1;
  c->probe_total = 0;
  if (capacity == 0) return LBM_OK;
  if (hipMalloc((void**)&c->probe_buf, sizeof(double) * 3 * (size_t)capacity) != hipSuccess ||
      hipMalloc((void**)&c->probe_n, sizeof(unsigned long long)) != hipSuccess) {
    if (c->probe_buf) (void)hipFree(c->probe_buf);
    c->probe_buf = nullptr;
    c->probe_n = nullptr;
    return fail(LBM_E_NOMEM, "probe buffer of %lld samples", (long long)capacity);
  }
  HIPCHK(hipMemsetAsync(c->probe_n, 0, sizeof(unsigned long long), c->stream));
  HIPCHK(hipMemsetAsync(c->probe_buf, 0, sizeof(double) * 3 * (size_t)capacity, c->stream));
  c->args.probe = x + y * cf.nx;
  c->args.probe_buf = c->probe_buf;
  c->args.probe_n = c->probe_n;
  c->args.probe_cap = capacity;
  return LBM_OK;
}

int lbm_probe_count(const lbm_ctx* c, int64_t* total) {
  if (!c || !total) return fail(LBM_E_INVAL, "ctx and total are required");
  *total = c->args.probe >= 0 ? c->probe_total : 0;
  return LBM_OK;
}

int lbm_probe_read(lbm_ctx* c, double* out, int64_t n) {
  if (!c || !out) return fail(LBM_E_INVAL, "ctx and out are required");
  if (c->args.probe < 0) return fail(LBM_E_STATE, "no probe is set");
  const int64_t cap = c->args.probe_cap;
  if (n < 0 || n > std::min(c->probe_total, cap))
    return fail(LBM_E_INVAL, "n = %lld exceeds the %lld samples held", (long long)n,
                (long long)std::min(c->probe_total, cap));
  if (n == 0) return LBM_OK;
  const int64_t first = (c->probe_total - n) % cap;  // ring slot of the oldest sample wanted
  const int64_t n1 = std::min(n, cap - first);
  for (int comp = 0; comp < 3; ++comp) {
    const double* src = c->probe_buf + comp * cap;
    double* dst = out + comp * n;
    HIPCHK(hipMemcpyAsync(dst, src + first, sizeof(double) * (size_t)n1, hipMemcpyDeviceToDevice, c->stream));
    if (n1 < n)
      HIPCHK(hipMemcpyAsync(dst + n1, src, sizeof(double) * (size_t)(n - n1), hipMemcpyDeviceToDevice,
                            c->stream));
  }
  return LBM_OK;
}

int lbm_dft_power(const double* x, int64_t n, double* power, int64_t* peak, void* stream) {
  if (!x || !power) return fail(LBM_E_INVAL, "x and power are required");
  if (n < 1 || n > ((int64_t)1 << 31)) return fail(LBM_E_INVAL, "n must be in [1, 2^31] (got %lld)", (long long)n);
  hipStream_t s = (hipStream_t)stream;
  int64_t* dpeak = nullptr;
  if (peak && hipMalloc((void**)&dpeak, sizeof(int64_t)) != hipSuccess)
    return fail(LBM_E_NOMEM, "peak index");
  hipError_t e = launch_dft_power(x, n, power, dpeak, s);
  if (e == hipSuccess && peak) e = hipMemcpyAsync(peak, dpeak, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && peak) e = hipStreamSynchronize(s);
  if (dpeak) (void)hipFree(dpeak);
  if (e != hipSuccess) return fail(LBM_E_DEVICE, "dft: %s", hipGetErrorString(e));
  return LBM_OK;
}

int lbm_layout(const lbm_ctx* c, int64_t* pitch, int64_t* bytes) {
  if (!c) return fail(LBM_E_INVAL, "ctx is NULL");
  if (pitch) *pitch = c->pitch;
  if (bytes) *bytes = (int64_t)c->cfg.lattice * c->plane * (int64_t)c->elem;
  return LBM_OK;
}

}  // extern "C"
