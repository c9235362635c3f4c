// Launch interface of the coupled system's pointwise kernels
// (kernels_coupled.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cgl {

// the nonlinear coefficients of eq. (coupled)
struct CoupledNl {
  double a3, b3, a4, b4, a5;
};

enum CoupledOp : int {
  CPL_FLOW = 0,  // out0 = phi_t(in0): one RK4 step of (u, v)' = g(u, v) over t
  CPL_G = 1,     // out0 = g(in0)
  CPL_L4R1 = 2,  // (in0, in1) = (P, Q) -> out0 = X, out1 = Y (Lawson4, first round; t = tau)
  CPL_L4R2 = 3,  // (in0, in1) = (HX, HY) -> out0 = HY + t/6 g(HX) (t = tau)
  CPL_L2 = 4,    // (in0, in1) = (P, Q) -> out0 = P + t/2 Q + t/2 g(P + t Q) (t = tau)
  CPL_COMB = 5,  // out0 = s0 in0 + s1 in1
};

struct CoupledArgs {
  const void* in0;
  const void* in1;
  void* out0;
  void* out1;
  int64_t N;       // points per field; a tensor holds u at [0, N), v at [N, 2N)
  int op;
  int f64;         // complex128 elements (else complex64)
  double t, s0, s1;
  CoupledNl c;
  unsigned* flag;  // bit 1: a non-finite result
};

hipError_t launch_coupled(const CoupledArgs& a, hipStream_t s);

}  // namespace cgl
