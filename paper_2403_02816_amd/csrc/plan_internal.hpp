// Read access to a plan's shape and stream for other parts of the library
// (the surrogate driver); not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/cgl.h"

namespace cgl {

struct PlanInfo {
  int d = 0;
  int64_t n[3] = {1, 1, 1};
  int precision = 0;
  unsigned flags = 0;
  int batch = 0;
  hipStream_t stream = nullptr;  // the caller's stream given to cgl_plan
};

int plan_info(cgl_plan_t p, PlanInfo* out);

// The Tucker operator of cgl_tucker with its intermediates in tmp0 / tmp1
// (device memory of at least N complex stage elements each) instead of the
// plan's stage buffers; enqueues no tuning and allocates nothing.
int tucker_with_scratch(cgl_plan_t p, int which, const void* in_dev, void* out_dev, void* tmp0,
                        void* tmp1);

// cgl_set_periodic with A_mu = (a1 + i b1) d_mu^2 + adv d_mu + a2/d (the
// first derivative's symbol i k, 0 for the Nyquist mode of an even n).
int set_periodic_adv(cgl_plan_t p, int mu, double a, double b, double adv);

// Split the contraction of a split-form plan's single-action passes when a
// pass has too few tiles to fill the chip (partial products of stage ranges,
// reduced in split order before the epilogue); allocates the plan's two
// workspaces (one per concurrent branch).  No effect on FP64 or batched plans
// or with CGL_KSPLIT=0 in the environment.
int enable_split_contraction(cgl_plan_t p);

}  // namespace cgl
