// lbm_internal.hpp -- host-side definitions of the opaque handles shared by
// the C-ABI translation units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_fstar.hpp"

// solver workspace (lbm_fstar_*)
struct lbm_fstar {
  int64_t cap = 0;
  hipStream_t stream = nullptr;
  double tol = 1e-10;
  float tol32 = 2e-6f;
  int max32 = 16, max64 = 6;
  uint32_t* ctr = nullptr;
  uint32_t* fail_list = nullptr;
  float* warm = nullptr;
  lbm::FstarStats* stats = nullptr;
};

// warm-start network (lbm_mlp_*)
struct lbm_mlp {
  float* params = nullptr;  // FP32 master weights [4740]
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  float* partials = nullptr;  // [MLP_GRAD_MAX_BLOCKS][4741]
  float* loss = nullptr;      // per-batch losses of the current epoch
  int64_t loss_cap = 0;
  int64_t t = 0;  // Adam step
  lbm::MlpNorm norm{};
};


int lbm_internal_fail(int code, const char* fmt, ...);
