// Pointwise nonlinear terms and flows of the CGL equation, evaluated per grid
// point in FP64 inside the mu-mode kernels' prologues and epilogues.
//
//  g(u)      = (a3 + i b3)|u|^2 u + (a4 + i b4)|u|^4 u        (eq. cqCGL)
//  phi^c_t   = exact flow of u' = (a3 + i b3)|u|^2 u          (eq. exsolcub)
//  phi^q_t   = exact flow of u' = (a4 + i b4)|u|^4 u          (Section 4.3)
//  phi_t     = one classical RK4 step of u' = g(u) (eq. RK4 with K = 0) when
//              there is no exact flow (cubic-quintic case, Section 4.3)
//  The sub-flows of the splitting schemes: entering a step (phi_t, or
//  phi^c_t o phi^q_t for the three-term splitting), leaving it (phi_t, or
//  phi^q_t o phi^c_t), between the two half steps of split4 (eq. Richardson:
//  one phi over 2t; three-term: leaving then entering), and the split4
//  combination 4/3 a - 1/3 b.
//  Lawson4 stage combinations of eq. (lawson4), regrouped around four
//  half-step exponential actions; the Lawson2b combination (eq. lawson2b).
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

// exp(-(a4 + i b4)/(4 a4) log(1 - 4 a4 |u|^4 t)) u, with the same domain
// handling as the cubic flow
__device__ __forceinline__ cd phi_quintic(cd u, double t, const NlParams& p, unsigned& flag) {
  const double r = u.re * u.re + u.im * u.im;
  const double r2 = r * r;
  double mag = 1.0, ang;
  if (p.a4 == 0.0) {
    ang = p.b4 * r2 * t;
  } else {
    const double s = -4.0 * p.a4 * r2 * t;
    double L;
    if (1.0 + s <= 0.0) {
      flag |= FLAG_BLOWUP;
      L = log(fabs(1.0 + s));
    } else {
      L = log1p(s);
    }
    mag = exp(-0.25 * L);
    ang = -p.b4 * L / (4.0 * p.a4);
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

// sub-flow over t entering a splitting step (applied before the linear flow)
__device__ __forceinline__ cd flow_in(cd u, double t, const NlParams& p, unsigned& flag) {
  if (p.flow == FLOW_3T) return phi_cubic(phi_quintic(u, t, p, flag), t, p, flag);
  return p.flow == FLOW_EXACT ? phi_cubic(u, t, p, flag) : rk4_flow(u, t, p);
}

// sub-flow over t leaving a splitting step (applied after the linear flow)
__device__ __forceinline__ cd flow_out(cd u, double t, const NlParams& p, unsigned& flag) {
  if (p.flow == FLOW_3T) return phi_quintic(phi_cubic(u, t, p, flag), t, p, flag);
  return p.flow == FLOW_EXACT ? phi_cubic(u, t, p, flag) : rk4_flow(u, t, p);
}

// between the two half steps of split4 (each with sub-flows over t): the
// printed scheme has one sub-flow over 2t there; the three-term splitting
// composes the flows leaving one half step and entering the next
__device__ __forceinline__ cd flow_mid(cd u, double t, const NlParams& p, unsigned& flag) {
  if (p.flow == FLOW_3T) return flow_in(flow_out(u, t, p, flag), t, p, flag);
  return flow_in(u, 2.0 * t, p, flag);
}

// split4: 4/3 phi_t(y) - 1/3 b, with b the full Strang step of the same point
__device__ __forceinline__ cd richardson(cd y, cd b, const NlParams& p, unsigned& flag) {
  const cd a = flow_out(y, p.tf, p, flag);
  return {(4.0 * a.re - b.re) / 3.0, (4.0 * a.im - b.im) / 3.0};
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

// Lawson2b (eq. lawson2b) from P = e^{tau K} u and Q = e^{tau K} g(u):
//   u_n2 = P + tau Q,  u_{n+1} = P + tau/2 Q + tau/2 g(u_n2)
__device__ __forceinline__ cd lawson2(cd P, cd Q, const NlParams& p, double h) {
  const cd un2 = caxpy(2.0 * h, Q, P);
  return caxpy(h, g_cgl(un2, p), caxpy(h, Q, P));
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

// exact flow of u' = (a + i b)|u|^{2k} u over t in FP32 (k = 1 cubic, 2 quintic)
__device__ __forceinline__ cf phi_power_f(cf u, float t, double a, double b, int k,
                                          unsigned& flag) {
  const float r = u.re * u.re + u.im * u.im;
  const float rk = k == 1 ? r : r * r;
  const float c = static_cast<float>(2 * k);
  float mag = 1.0f, ang;
  if (a == 0.0) {
    ang = static_cast<float>(b) * rk * t;
  } else {
    const float s = -c * static_cast<float>(a) * rk * t;
    float L;
    if (1.0f + s <= 0.0f) {
      flag |= FLAG_BLOWUP;
      L = logf(fabsf(1.0f + s));
    } else {
      L = log1pf(s);
    }
    mag = expf(-L / c);
    ang = static_cast<float>(-b / (2.0 * k * a)) * L;
  }
  float sn, cs;
  sincosf(ang, &sn, &cs);
  return {mag * (u.re * cs - u.im * sn), mag * (u.re * sn + u.im * cs)};
}

// flow_in in FP32 (the prologues of the split-precision passes)
__device__ __forceinline__ cf flow_in_f(cf u, const NlParams& p, unsigned& flag) {
  const float t = static_cast<float>(p.tf);
  if (p.flow == FLOW_3T)
    return phi_power_f(phi_power_f(u, t, p.a4, p.b4, 2, flag), t, p.a3, p.b3, 1, flag);
  if (p.flow == FLOW_EXACT) return phi_power_f(u, t, p.a3, p.b3, 1, flag);
  const cf k1 = g_cgl_f(u, p);
  const cf k2 = g_cgl_f(cfaxpy(0.5f * t, k1, u), p);
  const cf k3 = g_cgl_f(cfaxpy(0.5f * t, k2, u), p);
  const cf k4 = g_cgl_f(cfaxpy(t, k3, u), p);
  const cf s = {k1.re + k4.re + 2.0f * (k2.re + k3.re), k1.im + k4.im + 2.0f * (k2.im + k3.im)};
  return cfaxpy(t / 6.0f, s, u);
}

}  // namespace cgl
