// C ABI of the coupled two-field system (Section 4.4, eq. coupled): two
// plans of one 2-D periodic grid (their operators differ in the sign of the
// advection term a0 d_1), the pointwise kernels that couple the fields, and
// the steppers composed from them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>

#include "../../include/cgl.h"
#include "kernels_coupled.hpp"
#include "plan_internal.hpp"

using namespace cgl;

struct cgl_coupled_s {
  // f[k][j]: field k's plan (u: +a0 d_1, v: -a0 d_1) in slot j; the four run
  // on streams of their own, so that the exponential actions of a step that
  // do not depend on each other (both fields, and P = H w beside Q = H g(w)
  // in the Lawson schemes) run concurrently
  cgl_plan_t f[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipStream_t side[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipEvent_t fork = nullptr;
  hipEvent_t done[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int64_t n[2] = {0, 0};
  int64_t N = 0;
  cgl_coupled_coeffs c{};
  double tau = 0.0;
  int precision = CGL_FP64;
  hipStream_t stream = nullptr;
  void* buf[5] = {};        // stage tensors of 2N elements
  unsigned* dflag = nullptr;
  unsigned* hflag = nullptr;
  bool periodic[2] = {false, false};
};

namespace {

int dev(hipError_t e) { return e == hipSuccess ? CGL_OK : CGL_EDEVICE; }

size_t esz(const cgl_coupled_s* p) { return p->precision == CGL_FP64 ? 16 : 8; }

void* field(void* t, const cgl_coupled_s* p, int k) {
  return static_cast<char*>(t) + static_cast<size_t>(k) * p->N * esz(p);
}

// the exponential action of e^{t K} (which = CGL_E: t = tau, CGL_H: tau/2)
// on both fields of in0 (-> out0) and, if in1 is given, of in1 (-> out1):
// up to four independent actions forked from the plan's stream and joined
// back into it; inputs and outputs must not overlap
int act(cgl_coupled_s* p, int which, const void* in0, void* out0, const void* in1 = nullptr,
        void* out1 = nullptr) {
  const void* in[2] = {in0, in1};
  void* out[2] = {out0, out1};
  const int slots = in1 ? 2 : 1;
  int r = dev(hipEventRecord(p->fork, p->stream));
  for (int j = 0; j < slots && r == CGL_OK; ++j)
    for (int k = 0; k < 2 && r == CGL_OK; ++k) {
      r = dev(hipStreamWaitEvent(p->side[k][j], p->fork, 0));
      if (r == CGL_OK)
        r = cgl_tucker(p->f[k][j], which, field(const_cast<void*>(in[j]), p, k), field(out[j], p, k));
      if (r == CGL_OK) r = dev(hipEventRecord(p->done[k][j], p->side[k][j]));
      if (r == CGL_OK) r = dev(hipStreamWaitEvent(p->stream, p->done[k][j], 0));
    }
  return r;
}

int pw(cgl_coupled_s* p, int op, const void* in0, const void* in1, void* out0, void* out1,
       double t, double s0 = 0.0, double s1 = 0.0) {
  CoupledArgs a{};
  a.in0 = in0;
  a.in1 = in1;
  a.out0 = out0;
  a.out1 = out1;
  a.N = p->N;
  a.op = op;
  a.f64 = p->precision == CGL_FP64 ? 1 : 0;
  a.t = t;
  a.s0 = s0;
  a.s1 = s1;
  a.c = CoupledNl{p->c.a3, p->c.b3, p->c.a4, p->c.b4, p->c.a5};
  a.flag = p->dflag;
  return dev(launch_coupled(a, p->stream));
}

// Strang (eq. Strang): phi_{tau/2}, e^{tau K}, phi_{tau/2}; ex is the
// exponential of the step (CGL_E for a step tau, CGL_H for a half step)
int strang(cgl_coupled_s* p, int ex, double h, const void* in, void* out) {
  void *A = p->buf[0], *B = p->buf[1];
  int r = pw(p, CPL_FLOW, in, nullptr, A, nullptr, 0.5 * h);
  if (r == CGL_OK) r = act(p, ex, A, B);
  if (r == CGL_OK) r = pw(p, CPL_FLOW, B, nullptr, out, nullptr, 0.5 * h);
  return r;
}

// Lawson4 (eq. lawson4) with four actions of e^{tau K/2}:
// P = H w, Q = H g(w); X, Y from P, Q; w <- H Y + tau/6 g(H X)
int lawson4(cgl_coupled_s* p, void* w) {
  void *P = p->buf[0], *Q = p->buf[1], *G = p->buf[2], *X = p->buf[3], *Y = p->buf[4];
  int r = pw(p, CPL_G, w, nullptr, G, nullptr, 0.0);
  if (r == CGL_OK) r = act(p, CGL_H, w, P, G, Q);
  if (r == CGL_OK) r = pw(p, CPL_L4R1, P, Q, X, Y, p->tau);
  if (r == CGL_OK) r = act(p, CGL_H, X, P, Y, Q);
  if (r == CGL_OK) r = pw(p, CPL_L4R2, P, Q, w, nullptr, p->tau);
  return r;
}

// Lawson2b (eq. lawson2b): P = E w, Q = E g(w); w <- P + tau/2 Q + tau/2 g(P + tau Q)
int lawson2(cgl_coupled_s* p, void* w) {
  void *P = p->buf[0], *Q = p->buf[1], *G = p->buf[2];
  int r = pw(p, CPL_G, w, nullptr, G, nullptr, 0.0);
  if (r == CGL_OK) r = act(p, CGL_E, w, P, G, Q);
  if (r == CGL_OK) r = pw(p, CPL_L2, P, Q, w, nullptr, p->tau);
  return r;
}

// split4 (eq. Richardson): 4/3 S_{tau/2}(S_{tau/2}(w)) - 1/3 S_tau(w), the two
// half steps joined by one sub-flow over tau/2 as the equation writes them:
// phi_{tau/4} e^{tau K/2} phi_{tau/2} e^{tau K/2} phi_{tau/4}
int split4(cgl_coupled_s* p, void* w) {
  void *A = p->buf[0], *B = p->buf[1], *S = p->buf[2];
  const double q = 0.25 * p->tau;
  int r = strang(p, CGL_E, p->tau, w, S);
  if (r == CGL_OK) r = pw(p, CPL_FLOW, w, nullptr, A, nullptr, q);
  if (r == CGL_OK) r = act(p, CGL_H, A, B);
  if (r == CGL_OK) r = pw(p, CPL_FLOW, B, nullptr, A, nullptr, 2.0 * q);
  if (r == CGL_OK) r = act(p, CGL_H, A, B);
  if (r == CGL_OK) r = pw(p, CPL_FLOW, B, nullptr, A, nullptr, q);
  if (r == CGL_OK) r = pw(p, CPL_COMB, A, S, w, nullptr, 0.0, 4.0 / 3.0, -1.0 / 3.0);
  return r;
}

void release(cgl_coupled_s* p) {
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 2; ++j) {
      cgl_destroy(p->f[k][j]);
      p->f[k][j] = nullptr;
      if (p->done[k][j]) (void)hipEventDestroy(p->done[k][j]);
      p->done[k][j] = nullptr;
      if (p->side[k][j]) (void)hipStreamDestroy(p->side[k][j]);
      p->side[k][j] = nullptr;
    }
  if (p->fork) (void)hipEventDestroy(p->fork);
  p->fork = nullptr;
  for (auto& b : p->buf) {
    if (b) (void)hipFree(b);
    b = nullptr;
  }
  if (p->dflag) (void)hipFree(p->dflag);
  if (p->hflag) (void)hipHostFree(p->hflag);
  p->dflag = nullptr;
  p->hflag = nullptr;
}

}  // namespace

extern "C" {

int cgl_coupled_plan(cgl_coupled_t* out, const int64_t* n, const cgl_coupled_coeffs* c,
                     double tau, int precision, void* hip_stream) {
  if (!out) return CGL_EINVAL;
  *out = nullptr;
  if (!n || !c || !(tau > 0.0) || !std::isfinite(tau) ||
      (precision != CGL_FP64 && precision != CGL_SPLIT_BF16))
    return CGL_EINVAL;
  const double vals[9] = {c->a0, c->a1, c->b1, c->a2, c->a3, c->b3, c->a4, c->b4, c->a5};
  for (double v : vals)
    if (!std::isfinite(v)) return CGL_EINVAL;
  cgl_coupled_s* p = new (std::nothrow) cgl_coupled_s();
  if (!p) return CGL_ENOMEM;
  p->n[0] = n[0];
  p->n[1] = n[1];
  p->N = n[0] * n[1];
  p->c = *c;
  p->tau = tau;
  p->precision = precision;
  p->stream = static_cast<hipStream_t>(hip_stream);
  // each field's plan: its linear part (the nonlinear coefficients are unused:
  // the coupled kernels evaluate g)
  const cgl_coeffs cf{c->a1, c->b1, c->a2, c->a3, c->b3, c->a4, c->b4};
  int r = dev(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 2 && r == CGL_OK; ++j) {
      // default-priority streams, synchronised with the plan's stream by events
      r = dev(hipStreamCreateWithFlags(&p->side[k][j], hipStreamNonBlocking));
      if (r == CGL_OK) r = dev(hipEventCreateWithFlags(&p->done[k][j], hipEventDisableTiming));
      if (r == CGL_OK) r = cgl_plan(&p->f[k][j], 2, n, &cf, tau, precision, 0, p->side[k][j]);
      // a field's pass has few tiles (245 000-point fields at the paper's size)
      if (r == CGL_OK) r = enable_split_contraction(p->f[k][j]);
    }
  for (int b = 0; b < 5 && r == CGL_OK; ++b)
    if (hipMalloc(&p->buf[b], 2 * static_cast<size_t>(p->N) * esz(p)) != hipSuccess) r = CGL_ENOMEM;
  if (r == CGL_OK && hipMalloc(reinterpret_cast<void**>(&p->dflag), sizeof(unsigned)) != hipSuccess)
    r = CGL_ENOMEM;
  if (r == CGL_OK &&
      hipHostMalloc(reinterpret_cast<void**>(&p->hflag), sizeof(unsigned)) != hipSuccess)
    r = CGL_ENOMEM;
  if (r == CGL_OK) r = dev(hipMemsetAsync(p->dflag, 0, sizeof(unsigned), p->stream));
  if (r == CGL_OK) r = dev(hipStreamSynchronize(p->stream));
  if (r != CGL_OK) {
    release(p);
    delete p;
    return r;
  }
  *out = p;
  return CGL_OK;
}

int cgl_coupled_set_periodic(cgl_coupled_t p, int mu, double a, double b) {
  if (!p || mu < 0 || mu > 1) return CGL_EINVAL;
  // direction 1 carries +a0 d_1 for u and -a0 d_1 for v
  for (int k = 0; k < 2; ++k) {
    const double adv = mu == 0 ? (k == 0 ? p->c.a0 : -p->c.a0) : 0.0;
    for (int j = 0; j < 2; ++j) {
      const int r = set_periodic_adv(p->f[k][j], mu, a, b, adv);
      if (r != CGL_OK) return r;
    }
  }
  p->periodic[mu] = true;
  return CGL_OK;
}

int cgl_coupled_get_factor(cgl_coupled_t p, int field, int mu, int which, double* out_host) {
  if (!p || field < 0 || field > 1) return CGL_EINVAL;
  return cgl_get_periodic_factor(p->f[field][0], mu, which, out_host);
}

int cgl_coupled_step(cgl_coupled_t p, int method, void* w_dev, int64_t nsteps) {
  if (!p || !w_dev || nsteps < 0) return CGL_EINVAL;
  if (!p->periodic[0] || !p->periodic[1]) return CGL_ENOTREADY;
  int r = CGL_OK;
  for (int64_t s = 0; s < nsteps && r == CGL_OK; ++s) {
    switch (method) {
      case CGL_STRANG: r = strang(p, CGL_E, p->tau, w_dev, w_dev); break;
      case CGL_LAWSON4: r = lawson4(p, w_dev); break;
      case CGL_SPLIT4: r = split4(p, w_dev); break;
      case CGL_LAWSON2: r = lawson2(p, w_dev); break;
      default: return CGL_EINVAL;
    }
  }
  return r;
}

int cgl_coupled_status(cgl_coupled_t p) {
  if (!p) return CGL_EINVAL;
  int r = dev(hipMemcpyAsync(p->hflag, p->dflag, sizeof(unsigned), hipMemcpyDeviceToHost,
                             p->stream));
  if (r == CGL_OK) r = dev(hipStreamSynchronize(p->stream));
  if (r != CGL_OK) return r;
  const unsigned f = *p->hflag;
  r = dev(hipMemsetAsync(p->dflag, 0, sizeof(unsigned), p->stream));
  if (r == CGL_OK) r = dev(hipStreamSynchronize(p->stream));
  if (r != CGL_OK) return r;
  return f ? CGL_ENONFINITE : CGL_OK;
}

void cgl_coupled_destroy(cgl_coupled_t p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  for (auto& row : p->side)
    for (auto s : row)
      if (s) (void)hipStreamSynchronize(s);
  release(p);
  delete p;
}

}  // extern "C"
