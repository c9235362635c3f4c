// Pointwise nonlinear terms and flows of the CGL equation, evaluated per grid
// point in FP64 inside the mu-mode kernels' prologues and epilogues.
//
//  g(u)      = (a3 + i b3)|u|^2 u + (a4 + i b4)|u|^4 u        (eq. cqCGL)
//  phi^c_t   = exact flow of u' = (a3 + i b3)|u|^2 u          (eq. exsolcub)
//  phi_t     = one classical RK4 step of u' = g(u) (eq. RK4 with K = 0) when
//              there is no exact flow (cubic-quintic case, Section 4.3)
//  Lawson4 stage combinations of eq. (lawson4), regrouped around four
//  half-step exponential actions.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cgl {

struct cd {
  double re, im;
};

__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd caxpy(double s, cd x, cd y) {  // y + s x
  return {fma(s, x.re, y.re), fma(s, x.im, y.im)};
}

__device__ __forceinline__ cd g_cgl(cd u, const NlParams& p) {
  const double r = u.re * u.re + u.im * u.im;
  const double cr = (p.a3 + p.a4 * r) * r;  // real part of the coefficient of u
  const double ci = (p.b3 + p.b4 * r) * r;  // imaginary part
  return {cr * u.re - ci * u.im, cr * u.im + ci * u.re};
}

// exp(-(a3 + i b3)/(2 a3) log(1 - 2 a3 |u|^2 t)) u; outside the domain
// 1 - 2 a3 |u|^2 t > 0 the flow has blown up: flag it and continue with the
// absolute value as the paper's formula does.
__device__ __forceinline__ cd phi_cubic(cd u, double t, const NlParams& p, unsigned& flag) {
  const double r = u.re * u.re + u.im * u.im;
  double mag = 1.0, ang;
  if (p.a3 == 0.0) {
    ang = p.b3 * r * t;
  } else {
    const double s = -2.0 * p.a3 * r * t;
    double L;
    if (1.0 + s <= 0.0) {
      flag |= FLAG_BLOWUP;
      L = log(fabs(1.0 + s));
    } else {
      L = log1p(s);
    }
    mag = exp(-0.5 * L);
    ang = -p.b3 * L / (2.0 * p.a3);
  }
  double sn, cs;
  sincos(ang, &sn, &cs);
  return {mag * (u.re * cs - u.im * sn), mag * (u.re * sn + u.im * cs)};
}

__device__ __forceinline__ cd rk4_flow(cd u, double t, const NlParams& p) {
  const cd k1 = g_cgl(u, p);
  const cd k2 = g_cgl(caxpy(0.5 * t, k1, u), p);
  const cd k3 = g_cgl(caxpy(0.5 * t, k2, u), p);
  const cd k4 = g_cgl(caxpy(t, k3, u), p);
  cd s = cadd(k1, k4);
  s = caxpy(2.0, cadd(k2, k3), s);
  return caxpy(t / 6.0, s, u);
}

// phi_{tau/2}: the Strang sub-flow
__device__ __forceinline__ cd half_flow(cd u, const NlParams& p, unsigned& flag) {
  const double t = 0.5 * p.tau;
  return p.exact ? phi_cubic(u, t, p, flag) : rk4_flow(u, t, p);
}

__device__ __forceinline__ bool finite2(cd u) { return isfinite(u.re) && isfinite(u.im); }

// Lawson4 round 1 combination: from P = e^{tau K/2} u and Q = e^{tau K/2} g(u)
//   u2 = P + tau/2 Q,  u3 = P + tau/2 g(u2),
//   X = P + tau g(u3),  Y = P + tau/6 Q + tau/3 (g(u2) + g(u3)),
// so that u4 = e^{tau K/2} X and u_{n+1} = e^{tau K/2} Y + tau/6 g(u4).
// The step fractions of tau that the combinations use, formed once per lane
// (an FP64 division has no scalar form) and passed to the per-point code.
struct L4Coef {
  double h, t, t3, t6;  // tau/2, tau, tau/3, tau/6
};
__device__ __forceinline__ L4Coef lawson_coef(double tau) {
  return {0.5 * tau, tau, tau / 3.0, tau / 6.0};
}

__device__ __forceinline__ void lawson_r1(cd P, cd Q, const NlParams& p, const L4Coef& c, cd& X,
                                          cd& Y) {
  const cd u2 = caxpy(c.h, Q, P);
  const cd g2 = g_cgl(u2, p);
  const cd u3 = caxpy(c.h, g2, P);
  const cd g3 = g_cgl(u3, p);
  X = caxpy(c.t, g3, P);
  Y = caxpy(c.t3, cadd(g2, g3), caxpy(c.t6, Q, P));
}
__device__ __forceinline__ void lawson_r1(cd P, cd Q, const NlParams& p, cd& X, cd& Y) {
  lawson_r1(P, Q, p, lawson_coef(p.tau), X, Y);
}

// Lawson4 round 2 combination: u_{n+1} = HY + tau/6 g(HX)
__device__ __forceinline__ cd lawson_r2(cd HX, cd HY, const NlParams& p, double t6) {
  return caxpy(t6, g_cgl(HX, p), HY);
}
__device__ __forceinline__ cd lawson_r2(cd HX, cd HY, const NlParams& p) {
  return lawson_r2(HX, HY, p, p.tau / 6.0);
}

// ---- single-precision versions (prologues of the split-precision passes,
// whose inputs and outputs are complex64 stage tensors)
struct cf {
  float re, im;
};

__device__ __forceinline__ cf cfaxpy(float s, cf x, cf y) {  // y + s x
  return {fmaf(s, x.re, y.re), fmaf(s, x.im, y.im)};
}

__device__ __forceinline__ cf g_cgl_f(cf u, const NlParams& p) {
  const float r = u.re * u.re + u.im * u.im;
  const float cr = (static_cast<float>(p.a3) + static_cast<float>(p.a4) * r) * r;
  const float ci = (static_cast<float>(p.b3) + static_cast<float>(p.b4) * r) * r;
  return {cr * u.re - ci * u.im, cr * u.im + ci * u.re};
}

__device__ __forceinline__ cf half_flow_f(cf u, const NlParams& p, unsigned& flag) {
  const float t = static_cast<float>(0.5 * p.tau);
  if (p.exact) {
    const float r = u.re * u.re + u.im * u.im;
    float mag = 1.0f, ang;
    if (p.a3 == 0.0) {
      ang = static_cast<float>(p.b3) * r * t;
    } else {
      const float s = -2.0f * static_cast<float>(p.a3) * r * t;
      float L;
      if (1.0f + s <= 0.0f) {
        flag |= FLAG_BLOWUP;
        L = logf(fabsf(1.0f + s));
      } else {
        L = log1pf(s);
      }
      mag = expf(-0.5f * L);
      ang = static_cast<float>(-p.b3 / (2.0 * p.a3)) * L;
    }
    float sn, cs;
    sincosf(ang, &sn, &cs);
    return {mag * (u.re * cs - u.im * sn), mag * (u.re * sn + u.im * cs)};
  }
  const cf k1 = g_cgl_f(u, p);
  const cf k2 = g_cgl_f(cfaxpy(0.5f * t, k1, u), p);
  const cf k3 = g_cgl_f(cfaxpy(0.5f * t, k2, u), p);
  const cf k4 = g_cgl_f(cfaxpy(t, k3, u), p);
  const cf s = {k1.re + k4.re + 2.0f * (k2.re + k3.re), k1.im + k4.im + 2.0f * (k2.im + k3.im)};
  return cfaxpy(t / 6.0f, s, u);
}

}  // namespace cgl
