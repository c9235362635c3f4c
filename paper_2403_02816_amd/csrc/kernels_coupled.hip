// Pointwise kernels of the coupled two-field system (Section 4.4, eq.
// coupled).  A state holds u at [0, N) and v at [N, 2N); the nonlinear part
// couples the two fields at each grid point,
//   g_u = (a3 + i b3)|u|^2 u + (a4 + i b4)|u|^4 u + a5 |v|^2 u,
//   g_v = (a3 + i b3)|v|^2 v + (a4 + i b4)|v|^4 v + a5 |u|^2 v,
// so every kernel here takes the pair (u_i, v_i) of point i.  The
// exponential actions (one per field, the fields' operators differ in the
// sign of the advection term) run on the mu-mode product and Fourier
// kernels between them.  Arithmetic in FP64; elements complex64 (float2) or
// complex128 (double2).
#include <hip/hip_runtime.h>

#include "kernels_coupled.hpp"

namespace cgl {

namespace {

constexpr int NT = 256;
constexpr unsigned FLAG_NONFINITE_C = 1u;  // the plan flag's non-finite bit

struct c2 {
  double re, im;
};

__device__ __forceinline__ c2 operator+(c2 a, c2 b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ c2 operator*(double s, c2 a) { return {s * a.re, s * a.im}; }

template <typename E>
__device__ __forceinline__ c2 ld(const void* p, int64_t i) {
  const E v = static_cast<const E*>(p)[i];
  return {static_cast<double>(v.x), static_cast<double>(v.y)};
}

template <typename E>
__device__ __forceinline__ void st(void* p, int64_t i, c2 v) {
  using S = decltype(E{}.x);
  static_cast<E*>(p)[i] = E{static_cast<S>(v.re), static_cast<S>(v.im)};
}

__device__ __forceinline__ bool finite_c(c2 v) { return isfinite(v.re) && isfinite(v.im); }

// g of the pair (u, v) at one point: each field times its multiplier
// (a3 + i b3)|f|^2 + (a4 + i b4)|f|^4 + a5 |other|^2
__device__ __forceinline__ void g_pair(const CoupledNl& c, c2 u, c2 v, c2& gu, c2& gv) {
  const double ru = u.re * u.re + u.im * u.im;
  const double rv = v.re * v.re + v.im * v.im;
  const double pu = (c.a3 + c.a4 * ru) * ru + c.a5 * rv, qu = (c.b3 + c.b4 * ru) * ru;
  const double pv = (c.a3 + c.a4 * rv) * rv + c.a5 * ru, qv = (c.b3 + c.b4 * rv) * rv;
  gu = {pu * u.re - qu * u.im, pu * u.im + qu * u.re};
  gv = {pv * v.re - qv * v.im, pv * v.im + qv * v.re};
}

// one classical RK4 step (eq. RK4 with K = 0) of (u, v)' = g(u, v) over t
__device__ __forceinline__ void rk4_pair(const CoupledNl& c, double t, c2& u, c2& v) {
  c2 k1u, k1v, k2u, k2v, k3u, k3v, k4u, k4v;
  g_pair(c, u, v, k1u, k1v);
  g_pair(c, u + (0.5 * t) * k1u, v + (0.5 * t) * k1v, k2u, k2v);
  g_pair(c, u + (0.5 * t) * k2u, v + (0.5 * t) * k2v, k3u, k3v);
  g_pair(c, u + t * k3u, v + t * k3v, k4u, k4v);
  u = u + (t / 6.0) * (k1u + 2.0 * k2u + 2.0 * k3u + k4u);
  v = v + (t / 6.0) * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
}

template <typename E>
__global__ void k_cpl(CoupledArgs a) {
  const int64_t N = a.N;
  unsigned flag = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * NT) {
    const int64_t j = i + N;
    const CoupledNl& c = a.c;
    switch (a.op) {
      case CPL_FLOW: {  // out = phi_t(in)
        c2 u = ld<E>(a.in0, i), v = ld<E>(a.in0, j);
        rk4_pair(c, a.t, u, v);
        if (!finite_c(u) || !finite_c(v)) flag |= FLAG_NONFINITE_C;
        st<E>(a.out0, i, u);
        st<E>(a.out0, j, v);
        break;
      }
      case CPL_G: {  // out = g(in)
        c2 gu, gv;
        g_pair(c, ld<E>(a.in0, i), ld<E>(a.in0, j), gu, gv);
        st<E>(a.out0, i, gu);
        st<E>(a.out0, j, gv);
        break;
      }
      case CPL_L4R1: {  // (P, Q) -> X, Y of the regrouped Lawson4 step
        const c2 Pu = ld<E>(a.in0, i), Pv = ld<E>(a.in0, j);
        const c2 Qu = ld<E>(a.in1, i), Qv = ld<E>(a.in1, j);
        const double h = 0.5 * a.t;
        c2 g2u, g2v, g3u, g3v;
        g_pair(c, Pu + h * Qu, Pv + h * Qv, g2u, g2v);                  // g(u2)
        g_pair(c, Pu + h * g2u, Pv + h * g2v, g3u, g3v);                // g(u3)
        st<E>(a.out0, i, Pu + a.t * g3u);
        st<E>(a.out0, j, Pv + a.t * g3v);
        st<E>(a.out1, i, Pu + (a.t / 6.0) * Qu + (a.t / 3.0) * (g2u + g3u));
        st<E>(a.out1, j, Pv + (a.t / 6.0) * Qv + (a.t / 3.0) * (g2v + g3v));
        break;
      }
      case CPL_L4R2: {  // (HX, HY) -> u_{n+1} = HY + tau/6 g(HX)
        const c2 Xu = ld<E>(a.in0, i), Xv = ld<E>(a.in0, j);
        c2 gu, gv;
        g_pair(c, Xu, Xv, gu, gv);
        const c2 u = ld<E>(a.in1, i) + (a.t / 6.0) * gu;
        const c2 v = ld<E>(a.in1, j) + (a.t / 6.0) * gv;
        if (!finite_c(u) || !finite_c(v)) flag |= FLAG_NONFINITE_C;
        st<E>(a.out0, i, u);
        st<E>(a.out0, j, v);
        break;
      }
      case CPL_L2: {  // (P, Q) = (E u, E g(u)) -> P + tau/2 Q + tau/2 g(P + tau Q)
        const c2 Pu = ld<E>(a.in0, i), Pv = ld<E>(a.in0, j);
        const c2 Qu = ld<E>(a.in1, i), Qv = ld<E>(a.in1, j);
        c2 gu, gv;
        g_pair(c, Pu + a.t * Qu, Pv + a.t * Qv, gu, gv);
        const double h = 0.5 * a.t;
        const c2 u = Pu + h * Qu + h * gu, v = Pv + h * Qv + h * gv;
        if (!finite_c(u) || !finite_c(v)) flag |= FLAG_NONFINITE_C;
        st<E>(a.out0, i, u);
        st<E>(a.out0, j, v);
        break;
      }
      default: {  // CPL_COMB: out = s0 in0 + s1 in1 (split4's combination)
        const c2 u = a.s0 * ld<E>(a.in0, i) + a.s1 * ld<E>(a.in1, i);
        const c2 v = a.s0 * ld<E>(a.in0, j) + a.s1 * ld<E>(a.in1, j);
        if (!finite_c(u) || !finite_c(v)) flag |= FLAG_NONFINITE_C;
        st<E>(a.out0, i, u);
        st<E>(a.out0, j, v);
        break;
      }
    }
  }
  if (flag) atomicOr(a.flag, flag);
}

}  // namespace

hipError_t launch_coupled(const CoupledArgs& a, hipStream_t s) {
  if (a.N <= 0 || !a.in0 || !a.out0 || !a.flag || a.op < CPL_FLOW || a.op > CPL_COMB)
    return hipErrorInvalidValue;
  if ((a.op == CPL_L4R1 || a.op == CPL_L4R2 || a.op == CPL_L2 || a.op == CPL_COMB) && !a.in1)
    return hipErrorInvalidValue;
  if (a.op == CPL_L4R1 && !a.out1) return hipErrorInvalidValue;
  int64_t blocks = (a.N + NT - 1) / NT;
  if (blocks > 8192) blocks = 8192;
  if (a.f64)
    hipLaunchKernelGGL(k_cpl<double2>, dim3(static_cast<unsigned>(blocks)), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL(k_cpl<float2>, dim3(static_cast<unsigned>(blocks)), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace cgl
