// lbm_api_learn.hip -- C ABI of the entropic quasiequilibrium solver f*_M
// and of its learned Newton warm start (MLP 4 -> 64 -> 64 -> 4).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_fstar.hpp"
#include "lbm_internal.hpp"

using namespace lbm;

// the thread-local error text lives in lbm_api.hip
extern "C" const char* lbm_last_error(void);
int lbm_internal_fail(int code, const char* fmt, ...);

#define HIPCHK(expr)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return lbm_internal_fail(LBM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// SplitMix64 (Steele, Lea and Flood 2014)
static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
static double u01(uint64_t seed, uint64_t i) {
  return (double)(splitmix64(seed * 0x9E3779B97F4A7C15ull ^ i) >> 11) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Scratch of lbm_fstar_solve_static, in the library's own device memory
// (each GPU holds one copy until the process ends): the failure counter at
// byte 0, the FSTAR_STAT_SLOTS copies of the statistics at byte 256, the
// failure list (uint32 [n]) for up to LBM_FSTAR_STATIC_MAX_N sites from
// byte STATIC_FAIL_OFF, and the network's start (float [4][n]) for up to
// LBM_FSTAR_STATIC_MLP_MAX sites from byte STATIC_WARM_OFF: 48 MB in all.
// In host code `scratch` names a host-side stand-in; its device address is
// taken once per device with hipGetSymbolAddress and only that address is
// used.
// ---------------------------------------------------------------------------
constexpr size_t STATIC_STATS_OFF = 256;
constexpr size_t STATIC_FAIL_OFF = 4096;
constexpr size_t STATIC_WARM_OFF = STATIC_FAIL_OFF + sizeof(uint32_t) * (size_t)LBM_FSTAR_STATIC_MAX_N;
constexpr size_t STATIC_BYTES = STATIC_WARM_OFF + sizeof(float) * 4 * (size_t)LBM_FSTAR_STATIC_MLP_MAX;
static_assert(STATIC_STATS_OFF + sizeof(FstarStats) * FSTAR_STAT_SLOTS <= STATIC_FAIL_OFF, "scratch layout");
static_assert(STATIC_WARM_OFF % 256 == 0, "scratch layout");

static __device__ __align__(256) unsigned char scratch[STATIC_BYTES];

constexpr int STATIC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_ptr[STATIC_MAX_DEVICES];

// the current device's address of `scratch` (looked up once per device)
static int static_scratch(unsigned char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lbm_internal_fail(LBM_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= STATIC_MAX_DEVICES) return lbm_internal_fail(LBM_E_DEVICE, "device %d not supported", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return lbm_internal_fail(LBM_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

static void fill_solve_stats(const FstarStats& h, int64_t n, lbm_solve_stats* st) {
  std::memset(st, 0, sizeof(*st));
  st->n = n;
  st->n_infeasible = (int64_t)h.infeasible;
  st->n_fallback = (int64_t)h.fallback;
  st->n_failed = (int64_t)h.failed;
  for (int i = 0; i < 16; ++i) st->iter_hist[i] = (int64_t)h.hist[i];
  const double nf = (double)(n - (int64_t)h.infeasible);
  st->mean_fp32_iters = nf > 0 ? (double)h.sum32 / nf : 0.0;
  st->mean_fp64_iters = nf > 0 ? (double)h.sum64 / nf : 0.0;
  double mr;
  std::memcpy(&mr, &h.maxres_bits, 8);
  st->max_resid = mr;
}

extern "C" {

// ---------------------------------------------------------------------------
// f*_M solver
// ---------------------------------------------------------------------------
int lbm_fstar_create(int64_t max_n, void* stream, lbm_fstar** out) {
  if (!out) return lbm_internal_fail(LBM_E_INVAL, "out is NULL");
  *out = nullptr;
  if (max_n < 1 || max_n >= (int64_t)0xFFFFFFFFll) return lbm_internal_fail(LBM_E_INVAL, "max_n must be in [1, 2^32 - 1)");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return lbm_internal_fail(LBM_E_DEVICE, "no HIP device");
  lbm_fstar* s = new (std::nothrow) lbm_fstar();
  if (!s) return lbm_internal_fail(LBM_E_NOMEM, "host allocation failed");
  s->cap = max_n;
  s->stream = (hipStream_t)stream;
  bool ok = hipMalloc((void**)&s->ctr, 16) == hipSuccess &&
            hipMalloc((void**)&s->fail_list, sizeof(uint32_t) * (size_t)max_n) == hipSuccess &&
            hipMalloc((void**)&s->warm, sizeof(float) * 4 * (size_t)max_n) == hipSuccess &&
            hipMalloc((void**)&s->stats, sizeof(FstarStats) * FSTAR_STAT_SLOTS) == hipSuccess;
  if (!ok) {
    lbm_fstar_free(s);
    return lbm_internal_fail(LBM_E_NOMEM, "solver workspace allocation failed");
  }
  *out = s;
  return LBM_OK;
}

void lbm_fstar_free(lbm_fstar* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  if (s->ctr) (void)hipFree(s->ctr);
  if (s->fail_list) (void)hipFree(s->fail_list);
  if (s->warm) (void)hipFree(s->warm);
  if (s->stats) (void)hipFree(s->stats);
  delete s;
}

int lbm_fstar_set_tolerance(lbm_fstar* s, double tol, double tol32, int32_t max32, int32_t max64) {
  if (!s) return lbm_internal_fail(LBM_E_INVAL, "solver is NULL");
  if (!(tol > 0.0) || !(tol32 > 0.0) || max32 < 0 || max64 < 1 || max32 > 64 || max64 > 64)
    return lbm_internal_fail(LBM_E_INVAL, "need tol > 0, tol32 > 0, 0 <= max32 <= 64, 1 <= max64 <= 64");
  s->tol = tol;
  s->tol32 = (float)tol32;
  s->max32 = max32;
  s->max64 = max64;
  return LBM_OK;
}

int lbm_fstar_solve(lbm_fstar* s, const double* M, int64_t n, double* mu, int32_t start, const lbm_mlp* net,
                    uint8_t* iters, uint8_t* status, lbm_solve_stats* st) {
  if (!s || !M || !mu) return lbm_internal_fail(LBM_E_INVAL, "solver, M and mu are required");
  if (n < 0 || n > s->cap) return lbm_internal_fail(LBM_E_INVAL, "n must be in [0, max_n]");
  if (start != LBM_START_DEFAULT && start != LBM_START_CLOSED_FORM && start != LBM_START_MLP &&
      start != LBM_START_PREV && start != LBM_START_PLAIN)
    return lbm_internal_fail(LBM_E_INVAL, "start must be one of LBM_START_*");
  if (start == LBM_START_MLP && !net) return lbm_internal_fail(LBM_E_INVAL, "LBM_START_MLP needs a network");
  FstarArgs a{};
  a.M = M;
  a.n = n;
  a.mu = mu;
  a.warm = s->warm;
  a.iters = iters;
  a.status = status;
  a.ctr = s->ctr;
  a.fail_list = s->fail_list;
  a.stats = s->stats;
  a.tol = s->tol;
  a.tol32 = s->tol32;
  a.max32 = s->max32;
  a.max64 = s->max64;
  int kind = START_REST;
  if (start == LBM_START_CLOSED_FORM) kind = START_CLOSED;
  if (start == LBM_START_PREV) kind = START_PREV;
  if (start == LBM_START_PLAIN) kind = START_PLAIN;
  if (start == LBM_START_MLP) {
    kind = START_WARM;
    if (n > 0) HIPCHK(launch_mlp_warm(net->params, net->norm, M, n, s->warm, s->stream));
  }
  HIPCHK(launch_fstar(a, kind, s->stream));
  if (st) {
    FstarStats slots[FSTAR_STAT_SLOTS];
    HIPCHK(hipMemcpyAsync(slots, s->stats, sizeof(slots), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    const FstarStats h = fstar_stats_total(slots);
    fill_solve_stats(h, n, st);
    if (h.failed) return lbm_internal_fail(LBM_E_NOCONV, "%llu sites above the tolerance", (unsigned long long)h.failed);
  }
  return LBM_OK;
}

int lbm_fstar_solve_static(const double* M, int64_t n, double* mu, int32_t start, const lbm_mlp* net, double tol,
                           double tol32, int32_t max32, int32_t max64, uint8_t* iters, uint8_t* status,
                           lbm_solve_stats* st, void* stream) {
  if (!M || !mu) return lbm_internal_fail(LBM_E_INVAL, "M and mu are required");
  if (n < 0 || n > LBM_FSTAR_STATIC_MAX_N)
    return lbm_internal_fail(LBM_E_INVAL, "n must be in [0, %lld] (got %lld)", (long long)LBM_FSTAR_STATIC_MAX_N,
                             (long long)n);
  if (start != LBM_START_DEFAULT && start != LBM_START_CLOSED_FORM && start != LBM_START_MLP &&
      start != LBM_START_PREV && start != LBM_START_PLAIN)
    return lbm_internal_fail(LBM_E_INVAL, "start must be one of LBM_START_*");
  if (start == LBM_START_MLP && !net) return lbm_internal_fail(LBM_E_INVAL, "LBM_START_MLP needs a network");
  if (start == LBM_START_MLP && n > LBM_FSTAR_STATIC_MLP_MAX)
    return lbm_internal_fail(LBM_E_INVAL,
                             "LBM_START_MLP: the static scratch holds the network start of at most %d sites "
                             "(got %lld); use lbm_fstar_solve",
                             LBM_FSTAR_STATIC_MLP_MAX, (long long)n);
  if (!(tol > 0.0) || !(tol32 > 0.0) || max32 < 0 || max64 < 1 || max32 > 64 || max64 > 64)
    return lbm_internal_fail(LBM_E_INVAL, "need tol > 0, tol32 > 0, 0 <= max32 <= 64, 1 <= max64 <= 64");
  unsigned char* base = nullptr;
  int rc = static_scratch(&base);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  FstarArgs a{};
  a.M = M;
  a.n = n;
  a.mu = mu;
  float* warm = (float*)(base + STATIC_WARM_OFF);
  a.warm = warm;
  a.iters = iters;
  a.status = status;
  a.ctr = (uint32_t*)base;
  a.fail_list = (uint32_t*)(base + STATIC_FAIL_OFF);
  a.stats = (FstarStats*)(base + STATIC_STATS_OFF);
  a.tol = tol;
  a.tol32 = (float)tol32;
  a.max32 = max32;
  a.max64 = max64;
  int kind = START_REST;
  if (start == LBM_START_CLOSED_FORM) kind = START_CLOSED;
  if (start == LBM_START_PREV) kind = START_PREV;
  if (start == LBM_START_PLAIN) kind = START_PLAIN;
  if (start == LBM_START_MLP) {
    kind = START_WARM;
    if (n > 0) HIPCHK(launch_mlp_warm(net->params, net->norm, M, n, warm, s));
  }
  HIPCHK(launch_fstar(a, kind, s));
  if (st) {
    FstarStats slots[FSTAR_STAT_SLOTS];
    HIPCHK(hipMemcpyAsync(slots, a.stats, sizeof(slots), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const FstarStats h = fstar_stats_total(slots);
    fill_solve_stats(h, n, st);
    if (h.failed) return lbm_internal_fail(LBM_E_NOCONV, "%llu sites above the tolerance", (unsigned long long)h.failed);
  }
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// MLP
// ---------------------------------------------------------------------------
int lbm_mlp_pairs(const lbm_mlp* net, const double* M, const double* mu, int64_t n, float* X, float* T,
                  void* stream) {
  if (!net || !M || !X) return lbm_internal_fail(LBM_E_INVAL, "net, M and X are required");
  if (mu && !T) return lbm_internal_fail(LBM_E_INVAL, "T is required with mu");
  if (n < 0) return lbm_internal_fail(LBM_E_INVAL, "n must be >= 0");
  HIPCHK(launch_mlp_pairs(net->norm, M, mu, n, X, T, (hipStream_t)stream));
  return LBM_OK;
}

int lbm_mlp_warm_start(const lbm_mlp* net, const double* M, int64_t n, float* warm, void* stream) {
  if (n < 0) return lbm_internal_fail(LBM_E_INVAL, "n must be >= 0");
  if (!net || (n > 0 && (!M || !warm))) return lbm_internal_fail(LBM_E_INVAL, "net, M and warm are required");
  if (n > 0) HIPCHK(launch_mlp_warm(net->params, net->norm, M, n, warm, (hipStream_t)stream));
  return LBM_OK;
}

void lbm_mlp_free(lbm_mlp* net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  float* ptrs[] = {net->params, net->m, net->v, net->grad, net->partials, net->loss};
  for (float* p : ptrs)
    if (p) (void)hipFree(p);
  delete net;
}

int lbm_mlp_create(uint64_t seed, lbm_mlp** out) {
  if (!out) return lbm_internal_fail(LBM_E_INVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return lbm_internal_fail(LBM_E_DEVICE, "no HIP device");
  lbm_mlp* net = new (std::nothrow) lbm_mlp();
  if (!net) return lbm_internal_fail(LBM_E_NOMEM, "host allocation failed");
  const size_t pb = sizeof(float) * MLP_NPARAM;
  bool ok = hipMalloc((void**)&net->params, pb) == hipSuccess && hipMalloc((void**)&net->m, pb) == hipSuccess &&
            hipMalloc((void**)&net->v, pb) == hipSuccess && hipMalloc((void**)&net->grad, pb) == hipSuccess &&
            hipMalloc((void**)&net->partials, sizeof(float) * MLP_GRAD_MAX_BLOCKS * (MLP_NPARAM + 1)) == hipSuccess;
  if (!ok) {
    lbm_mlp_free(net);
    return lbm_internal_fail(LBM_E_NOMEM, "network allocation failed");
  }
  // Kaiming-uniform weights (bound sqrt(6 / fan_in)), zero biases
  std::vector<float> p(MLP_NPARAM, 0.0f);
  struct { int off, n, fan_in; } layers[3] = {{MLP_OW1, 256, 4}, {MLP_OW2, 4096, 64}, {MLP_OW3, 256, 64}};
  for (auto& L : layers) {
    const double b = std::sqrt(6.0 / L.fan_in);
    for (int i = 0; i < L.n; ++i) p[L.off + i] = (float)((2.0 * u01(seed, (uint64_t)(L.off + i)) - 1.0) * b);
  }
  std::vector<float> z(MLP_NPARAM, 0.0f);
  if (hipMemcpy(net->params, p.data(), pb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(net->m, z.data(), pb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(net->v, z.data(), pb, hipMemcpyHostToDevice) != hipSuccess) {
    lbm_mlp_free(net);
    return lbm_internal_fail(LBM_E_DEVICE, "network upload failed");
  }
  for (int k = 0; k < 4; ++k) {
    net->norm.in_shift[k] = 0.f;
    net->norm.in_scale[k] = 1.f;
    net->norm.out_shift[k] = 0.f;
    net->norm.out_scale[k] = 1.f;
  }
  *out = net;
  return LBM_OK;
}

int lbm_mlp_get_params(const lbm_mlp* net, float* host) {
  if (!net || !host) return lbm_internal_fail(LBM_E_INVAL, "net and host buffer are required");
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(host, net->params, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost));
  return LBM_OK;
}

int lbm_mlp_set_params(lbm_mlp* net, const float* host) {
  if (!net || !host) return lbm_internal_fail(LBM_E_INVAL, "net and host buffer are required");
  for (int i = 0; i < MLP_NPARAM; ++i)
    if (!std::isfinite(host[i])) return lbm_internal_fail(LBM_E_INVAL, "parameter %d is not finite", i);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(net->params, host, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice));
  std::vector<float> z(MLP_NPARAM, 0.0f);
  HIPCHK(hipMemcpy(net->m, z.data(), sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(net->v, z.data(), sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice));
  net->t = 0;
  return LBM_OK;
}

int lbm_mlp_set_norm(lbm_mlp* net, const float* norm16) {
  if (!net || !norm16) return lbm_internal_fail(LBM_E_INVAL, "net and norm are required");
  for (int k = 0; k < 4; ++k) {
    if (!(norm16[4 + k] != 0.f) || !(norm16[12 + k] != 0.f) || !std::isfinite(norm16[4 + k]) ||
        !std::isfinite(norm16[12 + k]))
      return lbm_internal_fail(LBM_E_INVAL, "scales must be finite and non-zero");
    net->norm.in_shift[k] = norm16[k];
    net->norm.in_scale[k] = norm16[4 + k];
    net->norm.out_shift[k] = norm16[8 + k];
    net->norm.out_scale[k] = norm16[12 + k];
  }
  return LBM_OK;
}

int lbm_mlp_get_norm(const lbm_mlp* net, float* norm16) {
  if (!net || !norm16) return lbm_internal_fail(LBM_E_INVAL, "net and norm are required");
  for (int k = 0; k < 4; ++k) {
    norm16[k] = net->norm.in_shift[k];
    norm16[4 + k] = net->norm.in_scale[k];
    norm16[8 + k] = net->norm.out_shift[k];
    norm16[12 + k] = net->norm.out_scale[k];
  }
  return LBM_OK;
}

int lbm_mlp_forward(const lbm_mlp* net, const float* X, int64_t n, float* Y, void* stream) {
  if (!net || !X || !Y || n < 0) return lbm_internal_fail(LBM_E_INVAL, "net, X, Y and n >= 0 are required");
  if (n == 0) return LBM_OK;
  HIPCHK(launch_mlp_forward(net->params, X, n, Y, (hipStream_t)stream));
  return LBM_OK;
}

int lbm_mlp_loss_grad(lbm_mlp* net, const float* X, const float* T, int64_t n, float* grad, float* loss,
                      void* stream) {
  if (!net || !X || !T || !grad || n < 1) return lbm_internal_fail(LBM_E_INVAL, "net, X, T, grad and n >= 1 are required");
  hipStream_t s = (hipStream_t)stream;
  MlpPerm ident{};
  HIPCHK(launch_mlp_grad(net->params, X, T, n, ident, net->partials, s));
  HIPCHK(launch_mlp_reduce(net->partials, mlp_grad_blocks(n), n, grad, loss, s));
  return LBM_OK;
}

int lbm_mlp_adam_step(lbm_mlp* net, const float* grad, double lr, void* stream) {
  if (!net || !grad || !(lr > 0.0)) return lbm_internal_fail(LBM_E_INVAL, "net, grad and lr > 0 are required");
  net->t++;
  HIPCHK(launch_adam(net->params, net->m, net->v, grad, net->t, (float)lr, 0.9f, 0.999f, 1e-8f, (hipStream_t)stream));
  return LBM_OK;
}

int lbm_mlp_train(lbm_mlp* net, const float* X, const float* T, int64_t n, int32_t epochs, int32_t batch,
                  double lr, uint64_t shuffle_seed, float* loss_per_epoch, void* stream) {
  if (!net || !X || !T) return lbm_internal_fail(LBM_E_INVAL, "net, X and T are required");
  if (n < 1 || n >= (int64_t)1 << 31 || epochs < 0 || batch < 1 || batch > n || !(lr > 0.0))
    return lbm_internal_fail(LBM_E_INVAL, "need 1 <= batch <= n < 2^31, epochs >= 0, lr > 0");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nb = n / batch;  // full batches per epoch; the remainder is dropped
  if (net->loss_cap < nb) {
    if (net->loss) HIPCHK(hipFree(net->loss));
    net->loss = nullptr;
    if (hipMalloc((void**)&net->loss, sizeof(float) * (size_t)nb) != hipSuccess)
      return lbm_internal_fail(LBM_E_NOMEM, "loss buffer allocation failed");
    net->loss_cap = nb;
  }
  std::vector<float> lb((size_t)nb);
  int bits = 0;
  while (((int64_t)1 << bits) < n) ++bits;
  MlpPerm perm{};
  perm.on = 1;
  perm.h = (bits + 1) / 2 > 0 ? (bits + 1) / 2 : 1;
  perm.n = (uint32_t)n;
  for (int32_t ep = 0; ep < epochs; ++ep) {
    // a fresh pseudo-random order of the n samples every epoch
    perm.key = splitmix64(shuffle_seed ^ ((uint64_t)(ep + 1) << 32));
    for (int64_t b = 0; b < nb; ++b) {
      perm.offset = (uint32_t)(b * batch);
      HIPCHK(launch_mlp_grad(net->params, X, T, batch, perm, net->partials, s));
      net->t++;
      HIPCHK(launch_mlp_reduce_adam(net->partials, mlp_grad_blocks(batch), batch, net->grad, net->loss + b,
                                    net->params, net->m, net->v, net->t, (float)lr, 0.9f, 0.999f, 1e-8f, s));
    }
    if (loss_per_epoch) {
      HIPCHK(hipMemcpyAsync(lb.data(), net->loss, sizeof(float) * (size_t)nb, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double acc = 0.0;
      for (int64_t b = 0; b < nb; ++b) acc += lb[(size_t)b];
      loss_per_epoch[ep] = (float)(acc / (double)(nb > 0 ? nb : 1));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  return LBM_OK;
}

}  // extern "C"
