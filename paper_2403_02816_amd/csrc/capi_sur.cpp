// C ABI of the learned surrogate: network state, training on the device,
// inference, and the gated run in which the plain stepper checks the jumps
// and takes over when a check fails.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>

#include "../../include/cgl.h"
#include "plan_internal.hpp"
#include "surrogate.hpp"

using namespace cgl;

namespace {

// conv_in (7 -> 48), four residual convs (48 -> 48), conv_out (48 -> 2)
struct Layer {
  int cout, cin;
  int cout_pad, cin_pad;    // forward weight layout
  int coutT_pad, cinT_pad;  // transposed layout (0: not needed)
  int64_t off;              // offset of W in the packed parameters (b follows)
};

constexpr int NL = SUR_LAYERS;
constexpr double ADAM_B1 = 0.9, ADAM_B2 = 0.999, ADAM_EPS = 1e-8;

}  // namespace

struct cgl_sur_s {
  int n1 = 0, n2 = 0;
  int64_t P = 0;
  int maxS = 0;
  hipStream_t stream = nullptr;
  Layer L[NL];
  int64_t count = 0;
  float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* wf[NL] = {};
  uint16_t* wt[NL] = {};
  float* x = nullptr;  // [maxS][7][P]
  float* xb = nullptr; // [maxS][2][P] base planes when a base state is given
  float* a[SUR_BLOCKS + 1] = {};
  float* h[SUR_BLOCKS + 1] = {};
  float *y = nullptr, *dy = nullptr, *dh = nullptr, *da[2] = {};
  float* part = nullptr;
  double* dacc = nullptr;   // [0] loss sum, [2..3] difference norms
  double* hacc = nullptr;   // pinned copy
  float* cstd1 = nullptr;   // [5] coefficients of a gated run
  void *ver = nullptr, *prev = nullptr;  // complex64 [P]
  void* base1 = nullptr;                 // complex64 [P]: the base of a gated jump
  bool have_params = false;
  int64_t t = 0;            // Adam steps taken
  int64_t loss_steps = 0;   // train steps since the last cgl_sur_take_loss
  int loss_kind = CGL_SUR_LOSS_MSE;
  float oscale = 1.0f;      // scale of the network's correction (cgl_sur_set_output_scale)
  double* wsamp = nullptr;  // [maxS] per-sample weights of the relative loss
};

namespace {

int dev(hipError_t e) { return e == hipSuccess ? CGL_OK : CGL_EDEVICE; }

template <class T>
int alloc(T** p, int64_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, static_cast<size_t>(count) * sizeof(T)) != hipSuccess) return CGL_ENOMEM;
  *p = static_cast<T*>(q);
  return CGL_OK;
}

void layers(Layer* L) {
  int64_t off = 0;
  for (int k = 0; k < NL; ++k) {
    Layer& l = L[k];
    if (k == 0) {
      l = Layer{SUR_C, SUR_CIN, 48, 8, 0, 0, 0};
    } else if (k < NL - 1) {
      l = Layer{SUR_C, SUR_C, 48, 48, 48, 48, 0};
    } else {
      l = Layer{2, SUR_C, 16, 48, 48, 8, 0};
    }
    l.off = off;
    off += static_cast<int64_t>(l.cout) * l.cin * 9 + l.cout;
  }
}

int64_t count_params() {
  Layer L[NL];
  layers(L);
  return L[NL - 1].off + 2LL * SUR_C * 9 + 2;
}

const float* W(const cgl_sur_s* s, int k) { return s->params + s->L[k].off; }
const float* B(const cgl_sur_s* s, int k) {
  return s->params + s->L[k].off + static_cast<int64_t>(s->L[k].cout) * s->L[k].cin * 9;
}

int pack_weights(cgl_sur_s* s, hipStream_t st) {
  for (int k = 0; k < NL; ++k) {
    const Layer& l = s->L[k];
    if (launch_pack_weights(W(s, k), l.cout, l.cin, s->wf[k], l.cout_pad, l.cin_pad, s->wt[k],
                            l.cinT_pad, l.coutT_pad, st) != hipSuccess)
      return CGL_EDEVICE;
  }
  return CGL_OK;
}

ConvArgs conv_args(const cgl_sur_s* s, int S, const float* x, const uint16_t* w, const float* b,
                   float* out0, float* out1, const float* aux, const float* aux2, int cin, int cout,
                   int epi, int aux_ch) {
  ConvArgs c{};
  c.x = x;
  c.w = w;
  c.bias = b;
  c.out0 = out0;
  c.out1 = out1;
  c.aux = aux;
  c.aux2 = aux2;
  c.cin = cin;
  c.cout = cout;
  c.n1 = s->n1;
  c.n2 = s->n2;
  c.S = S;
  c.epi = epi;
  c.aux_ch = aux_ch;
  c.oscale = s->oscale;
  return c;
}

int conv(const ConvArgs& c, int cin_pad, int cout_pad, hipStream_t st) {
  return dev(launch_conv(c, cin_pad, cout_pad, st));
}

// x -> y.  keep: store every pre-activation a_k and h_k for backward;
// otherwise the hidden state ping-pongs between h[0] and h[1].  based: the
// output adds the correction to the planes in xb instead of the input's.
int forward(cgl_sur_s* s, int S, bool keep, bool based, hipStream_t st) {
  const Layer* L = s->L;
  int r = conv(conv_args(s, S, s->x, s->wf[0], B(s, 0), keep ? s->a[0] : nullptr, s->h[0],
                         nullptr, nullptr, L[0].cin, L[0].cout, CEPI_SILU, 0),
               L[0].cin_pad, L[0].cout_pad, st);
  const float* hin = s->h[0];
  for (int k = 1; k <= SUR_BLOCKS && r == CGL_OK; ++k) {
    float* hout = keep ? s->h[k] : s->h[k % 2];
    r = conv(conv_args(s, S, hin, s->wf[k], B(s, k), keep ? s->a[k] : nullptr, hout, hin, nullptr,
                       L[k].cin, L[k].cout, CEPI_RES, 0),
             L[k].cin_pad, L[k].cout_pad, st);
    hin = hout;
  }
  if (r != CGL_OK) return r;
  const int k = NL - 1;
  return conv(conv_args(s, S, hin, s->wf[k], B(s, k), s->y, nullptr, based ? s->xb : s->x,
                        nullptr, L[k].cin, L[k].cout, CEPI_OUT, based ? 2 : SUR_CIN),
              L[k].cin_pad, L[k].cout_pad, st);
}

// gradients of the loss whose dy is in s->dy, after forward(keep = true)
int backward(cgl_sur_s* s, int S, hipStream_t st) {
  const Layer* L = s->L;
  auto wgrad = [&](int k, const float* X, const float* dout) {
    WgradArgs w{X, dout, L[k].cin, L[k].cout, s->n1, s->n2, S};
    return dev(launch_wgrad(w, s->part, s->grad + L[k].off, st));
  };
  const int ko = NL - 1;
  int r = wgrad(ko, s->h[SUR_BLOCKS], s->dy);
  // dh_4 = conv_out^T dy, da_4 = dh_4 silu'(a_4)
  if (r == CGL_OK)
    r = conv(conv_args(s, S, s->dy, s->wt[ko], nullptr, s->dh, s->da[0], nullptr, s->a[SUR_BLOCKS],
                       L[ko].cout, L[ko].cin, CEPI_BWD, 0),
             L[ko].cinT_pad, L[ko].coutT_pad, st);
  int cur = 0;
  for (int k = SUR_BLOCKS; k >= 1 && r == CGL_OK; --k) {
    r = wgrad(k, s->h[k - 1], s->da[cur]);
    // dh_{k-1} = dh_k + conv_k^T da_k, da_{k-1} = dh_{k-1} silu'(a_{k-1})
    if (r == CGL_OK)
      r = conv(conv_args(s, S, s->da[cur], s->wt[k], nullptr, k > 1 ? s->dh : nullptr, s->da[1 - cur],
                         s->dh, s->a[k - 1], L[k].cout, L[k].cin, CEPI_BWD, 0),
               L[k].cinT_pad, L[k].coutT_pad, st);
    cur = 1 - cur;
  }
  if (r == CGL_OK) r = wgrad(0, s->x, s->da[cur]);
  return r;
}

int check_batch(const cgl_sur_s* s, int S) { return (S >= 1 && S <= s->maxS) ? CGL_OK : CGL_EINVAL; }

int loss_and_grad(cgl_sur_s* s, int S, const void* src, const float* cstd, const int32_t* idx,
                  int64_t toff, const void* base, hipStream_t st) {
  if (!s->have_params) return CGL_ENOTREADY;
  int r = dev(launch_sur_pack(src, idx, cstd, s->x, S, s->P, st));
  if (r == CGL_OK && base) r = dev(launch_sur_pack_base(base, idx, s->xb, S, s->P, st));
  if (r == CGL_OK) r = forward(s, S, true, base != nullptr, st);
  if (r == CGL_OK)
    r = dev(launch_mse(s->y, src, idx, toff, s->loss_kind == CGL_SUR_LOSS_REL ? s->wsamp : nullptr,
                       s->oscale, s->dy, s->dacc, S, s->P, st));
  if (r == CGL_OK) r = backward(s, S, st);
  return r;
}

int infer(cgl_sur_s* s, int S, const void* u, const float* cstd, const void* base, void* out,
          hipStream_t st) {
  if (!s->have_params) return CGL_ENOTREADY;
  int r = dev(launch_sur_pack(u, nullptr, cstd, s->x, S, s->P, st));
  if (r == CGL_OK && base) r = dev(launch_sur_pack_base(base, nullptr, s->xb, S, s->P, st));
  if (r == CGL_OK) r = forward(s, S, false, base != nullptr, st);
  if (r == CGL_OK) r = dev(launch_sur_unpack(s->y, out, S, s->P, st));
  return r;
}

void release(cgl_sur_s* s) {
  auto f = [](auto*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
  };
  f(s->params); f(s->grad); f(s->m); f(s->v);
  for (int k = 0; k < NL; ++k) { f(s->wf[k]); f(s->wt[k]); }
  f(s->x); f(s->xb); f(s->base1);
  for (int k = 0; k <= SUR_BLOCKS; ++k) { f(s->a[k]); f(s->h[k]); }
  f(s->y); f(s->dy); f(s->dh); f(s->da[0]); f(s->da[1]); f(s->part);
  f(s->dacc); f(s->cstd1); f(s->ver); f(s->prev); f(s->wsamp);
  if (s->hacc) (void)hipHostFree(s->hacc);
  s->hacc = nullptr;
}

}  // namespace

extern "C" {

int cgl_sur_param_count(int64_t* count) {
  if (!count) return CGL_EINVAL;
  *count = count_params();
  return CGL_OK;
}

int cgl_sur_create(cgl_sur_t* out, int64_t n1, int64_t n2, int max_batch, void* hip_stream) {
  if (!out) return CGL_EINVAL;
  *out = nullptr;
  if (n1 < 64 || n1 % 64 != 0 || n1 > 4096 || n2 < 1 || n2 > 4096 || max_batch < 1)
    return CGL_EINVAL;
  const int64_t P = n1 * n2;
  if (P * max_batch > (int64_t{1} << 31) / SUR_C) return CGL_EINVAL;  // activations addressable
  cgl_sur_s* s = new (std::nothrow) cgl_sur_s();
  if (!s) return CGL_ENOMEM;
  s->n1 = static_cast<int>(n1);
  s->n2 = static_cast<int>(n2);
  s->P = P;
  s->maxS = max_batch;
  s->stream = static_cast<hipStream_t>(hip_stream);
  layers(s->L);
  s->count = count_params();
  const int64_t S = max_batch;
  int r = CGL_OK;
  auto need = [&](int rr) { if (r == CGL_OK) r = rr; };
  need(alloc(&s->params, s->count));
  need(alloc(&s->grad, s->count));
  need(alloc(&s->m, s->count));
  need(alloc(&s->v, s->count));
  for (int k = 0; k < NL && r == CGL_OK; ++k) {
    const Layer& l = s->L[k];
    need(alloc(&s->wf[k], static_cast<int64_t>(l.cout_pad) * conv_kpad(l.cin_pad)));
    if (l.coutT_pad) need(alloc(&s->wt[k], static_cast<int64_t>(l.coutT_pad) * conv_kpad(l.cinT_pad)));
  }
  need(alloc(&s->x, S * SUR_CIN * P));
  need(alloc(&s->xb, S * 2 * P));
  for (int k = 0; k <= SUR_BLOCKS; ++k) {
    need(alloc(&s->a[k], S * SUR_C * P));
    need(alloc(&s->h[k], S * SUR_C * P));
  }
  need(alloc(&s->y, S * 2 * P));
  need(alloc(&s->dy, S * 2 * P));
  need(alloc(&s->dh, S * SUR_C * P));
  need(alloc(&s->da[0], S * SUR_C * P));
  need(alloc(&s->da[1], S * SUR_C * P));
  need(alloc(&s->part, static_cast<int64_t>(wgrad_grid(max_batch, s->n1, s->n2)) *
                           (SUR_C * SUR_C * 9 + SUR_C)));
  need(alloc(&s->dacc, 4));
  need(alloc(&s->wsamp, S));
  need(alloc(&s->cstd1, 8));
  need(alloc(reinterpret_cast<float**>(&s->ver), 2 * P));
  need(alloc(reinterpret_cast<float**>(&s->prev), 2 * P));
  need(alloc(reinterpret_cast<float**>(&s->base1), 2 * P));
  if (r == CGL_OK && hipHostMalloc(reinterpret_cast<void**>(&s->hacc), 4 * sizeof(double)) != hipSuccess)
    r = CGL_ENOMEM;
  if (r == CGL_OK) r = dev(launch_zero(reinterpret_cast<float*>(s->dacc), 8, s->stream));
  if (r != CGL_OK) {
    release(s);
    delete s;
    return r;
  }
  *out = s;
  return CGL_OK;
}

int cgl_sur_set_params(cgl_sur_t s, const float* params_host) {
  if (!s || !params_host) return CGL_EINVAL;
  for (int64_t i = 0; i < s->count; ++i)
    if (!std::isfinite(params_host[i])) return CGL_EINVAL;
  const size_t bytes = static_cast<size_t>(s->count) * sizeof(float);
  int r = dev(hipMemcpyAsync(s->params, params_host, bytes, hipMemcpyHostToDevice, s->stream));
  if (r == CGL_OK) r = dev(hipStreamSynchronize(s->stream));
  if (r == CGL_OK) r = dev(launch_zero(s->m, s->count, s->stream));
  if (r == CGL_OK) r = dev(launch_zero(s->v, s->count, s->stream));
  if (r == CGL_OK) r = pack_weights(s, s->stream);
  if (r == CGL_OK) {
    s->t = 0;
    s->have_params = true;
  }
  return r;
}

int cgl_sur_set_loss(cgl_sur_t s, int kind) {
  if (!s || (kind != CGL_SUR_LOSS_MSE && kind != CGL_SUR_LOSS_REL)) return CGL_EINVAL;
  s->loss_kind = kind;
  return CGL_OK;
}

int cgl_sur_set_output_scale(cgl_sur_t s, float scale) {
  if (!s || !std::isfinite(scale) || !(scale > 0.0f)) return CGL_EINVAL;
  s->oscale = scale;
  return CGL_OK;
}

int cgl_sur_get_params(cgl_sur_t s, float* params_host) {
  if (!s || !params_host) return CGL_EINVAL;
  if (!s->have_params) return CGL_ENOTREADY;
  int r = dev(hipMemcpyAsync(params_host, s->params, static_cast<size_t>(s->count) * sizeof(float),
                             hipMemcpyDeviceToHost, s->stream));
  if (r == CGL_OK) r = dev(hipStreamSynchronize(s->stream));
  return r;
}

int cgl_sur_forward(cgl_sur_t s, int batch, const void* u_dev, const float* cstd_dev,
                    const void* base_dev, void* out_dev) {
  if (!s || !u_dev || !cstd_dev || !out_dev) return CGL_EINVAL;
  int r = check_batch(s, batch);
  if (r != CGL_OK) return r;
  return infer(s, batch, u_dev, cstd_dev, base_dev, out_dev, s->stream);
}

int cgl_sur_grad(cgl_sur_t s, int batch, const void* src_dev, const float* cstd_dev,
                 const int32_t* idx_dev, int64_t target_offset, const void* base_dev,
                 float* grad_host, double* loss_host) {
  if (!s || !src_dev || !cstd_dev || !grad_host) return CGL_EINVAL;
  int r = check_batch(s, batch);
  if (r != CGL_OK) return r;
  r = dev(launch_zero(reinterpret_cast<float*>(s->dacc), 2, s->stream));
  if (r == CGL_OK)
    r = loss_and_grad(s, batch, src_dev, cstd_dev, idx_dev, target_offset, base_dev, s->stream);
  if (r == CGL_OK)
    r = dev(hipMemcpyAsync(grad_host, s->grad, static_cast<size_t>(s->count) * sizeof(float),
                           hipMemcpyDeviceToHost, s->stream));
  if (r == CGL_OK)
    r = dev(hipMemcpyAsync(s->hacc, s->dacc, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  if (r == CGL_OK) r = dev(hipStreamSynchronize(s->stream));
  if (r == CGL_OK && loss_host) *loss_host = s->hacc[0];
  s->loss_steps = 0;
  if (r == CGL_OK) r = dev(launch_zero(reinterpret_cast<float*>(s->dacc), 2, s->stream));
  return r;
}

int cgl_sur_train_step(cgl_sur_t s, int batch, const void* src_dev, const float* cstd_dev,
                       const int32_t* idx_dev, int64_t target_offset, const void* base_dev,
                       float lr) {
  if (!s || !src_dev || !cstd_dev || !(lr >= 0.0f)) return CGL_EINVAL;
  int r = check_batch(s, batch);
  if (r != CGL_OK) return r;
  r = loss_and_grad(s, batch, src_dev, cstd_dev, idx_dev, target_offset, base_dev, s->stream);
  if (r != CGL_OK) return r;
  s->t += 1;
  const double c1 = 1.0 / (1.0 - std::pow(ADAM_B1, static_cast<double>(s->t)));
  const double c2 = 1.0 / (1.0 - std::pow(ADAM_B2, static_cast<double>(s->t)));
  r = dev(launch_adam(s->params, s->grad, s->m, s->v, static_cast<int>(s->count), lr,
                      static_cast<float>(ADAM_B1), static_cast<float>(ADAM_B2),
                      static_cast<float>(ADAM_EPS), static_cast<float>(c1), static_cast<float>(c2),
                      s->stream));
  if (r == CGL_OK) r = pack_weights(s, s->stream);
  if (r == CGL_OK) s->loss_steps += 1;
  return r;
}

int cgl_sur_take_loss(cgl_sur_t s, double* mean_loss) {
  if (!s || !mean_loss) return CGL_EINVAL;
  int r = dev(hipMemcpyAsync(s->hacc, s->dacc, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  if (r == CGL_OK) r = dev(hipStreamSynchronize(s->stream));
  if (r != CGL_OK) return r;
  *mean_loss = s->loss_steps > 0 ? s->hacc[0] / static_cast<double>(s->loss_steps) : 0.0;
  s->loss_steps = 0;
  return dev(launch_zero(reinterpret_cast<float*>(s->dacc), 2, s->stream));
}

void cgl_sur_destroy(cgl_sur_t s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  release(s);
  delete s;
}

int cgl_run_surrogate(cgl_plan_t p, cgl_sur_t s, void* u_dev, const double* cstd,
                      int64_t njumps, int64_t steps_per_jump, int64_t check_every, double tol,
                      cgl_plan_t coarse, int base, int64_t* stats) {
  if (!p || !s || !u_dev || !cstd || njumps < 0 || steps_per_jump < 1 || check_every < 1 ||
      !(tol > 0.0) || base < CGL_SUR_BASE_INPUT || base > CGL_SUR_BASE_STRANG ||
      (base != CGL_SUR_BASE_INPUT && !coarse))
    return CGL_EINVAL;
  PlanInfo pi;
  int r = plan_info(p, &pi);
  if (r != CGL_OK) return r;
  // complex64 state of one 2-D instance of the network's grid
  auto fits = [&](const PlanInfo& q) {
    return q.batch == 0 && q.d == 2 && q.n[0] == s->n1 && q.n[1] == s->n2 &&
           q.precision == CGL_SPLIT_BF16 && !(q.flags & CGL_FLAG_FP64_MASTER);
  };
  if (!fits(pi)) return CGL_EINVAL;
  if (base != CGL_SUR_BASE_INPUT) {
    PlanInfo ci;
    r = plan_info(coarse, &ci);
    if (r != CGL_OK) return r;
    if (!fits(ci) || ci.stream != pi.stream) return CGL_EINVAL;
  }
  if (!s->have_params) return CGL_ENOTREADY;
  int64_t st[4] = {0, 0, 0, 0};  // accepted jumps, rejected jumps, checks, plain steps
  const hipStream_t q = pi.stream;
  const size_t bytes = static_cast<size_t>(s->P) * 8;
  float c5[5];
  for (int k = 0; k < 5; ++k) c5[k] = static_cast<float>(cstd[k]);
  r = dev(hipMemcpyAsync(s->cstd1, c5, sizeof(c5), hipMemcpyHostToDevice, q));
  if (r == CGL_OK) r = dev(hipStreamSynchronize(q));
  if (r == CGL_OK) r = dev(hipMemcpyAsync(s->ver, u_dev, bytes, hipMemcpyDeviceToDevice, q));
  int64_t since = 0;  // provisional jumps since the last verified state
  for (int64_t j = 1; j <= njumps && r == CGL_OK; ++j) {
    const bool check = (j % check_every == 0) || j == njumps;
    if (check) r = dev(hipMemcpyAsync(s->prev, u_dev, bytes, hipMemcpyDeviceToDevice, q));
    // the base of the jump: the input itself, the coarse plan's exponential
    // (e^{M tau K} u when its step is M tau) or one Strang step of the coarse plan
    if (r == CGL_OK && base == CGL_SUR_BASE_LINEAR) r = cgl_tucker(coarse, CGL_E, u_dev, s->base1);
    if (r == CGL_OK && base == CGL_SUR_BASE_STRANG) {
      r = dev(hipMemcpyAsync(s->base1, u_dev, bytes, hipMemcpyDeviceToDevice, q));
      if (r == CGL_OK) r = cgl_step(coarse, CGL_STRANG, s->base1, 1);
    }
    if (r == CGL_OK)
      r = infer(s, 1, u_dev, s->cstd1, base == CGL_SUR_BASE_INPUT ? nullptr : s->base1, u_dev, q);
    if (r != CGL_OK) break;
    since += 1;
    if (!check) continue;
    // a-posteriori check: the plain stepper from the same start (which is
    // provisional: a non-finite or blown-up check run is a failed check)
    r = cgl_run(p, CGL_LAWSON4, s->prev, steps_per_jump, 0);
    st[2] += 1;
    st[3] += steps_per_jump;
    double rel = HUGE_VAL;
    if (r == CGL_OK) {
      r = dev(launch_zero(reinterpret_cast<float*>(s->dacc + 2), 4, q));
      if (r == CGL_OK) r = dev(launch_diff_norms(u_dev, s->prev, s->P, s->dacc + 2, q));
      if (r == CGL_OK)
        r = dev(hipMemcpyAsync(s->hacc + 2, s->dacc + 2, 2 * sizeof(double),
                               hipMemcpyDeviceToHost, q));
      if (r == CGL_OK) r = dev(hipStreamSynchronize(q));
      if (r != CGL_OK) break;
      rel = std::sqrt(s->hacc[2] / s->hacc[3]);
    } else if (r == CGL_ENONFINITE || r == CGL_EBLOWUP) {
      r = CGL_OK;
    } else {
      break;
    }
    if (std::isfinite(rel) && rel <= tol) {
      // accepted: continue from the plain result of the checked span
      st[0] += since;
      r = dev(hipMemcpyAsync(u_dev, s->prev, bytes, hipMemcpyDeviceToDevice, q));
    } else {
      // rejected: roll back to the verified state and redo the span plainly
      st[1] += since;
      r = dev(hipMemcpyAsync(u_dev, s->ver, bytes, hipMemcpyDeviceToDevice, q));
      if (r == CGL_OK) r = cgl_run(p, CGL_LAWSON4, u_dev, since * steps_per_jump, 0);
      if (r == CGL_OK) st[3] += since * steps_per_jump;
    }
    if (r == CGL_OK) r = dev(hipMemcpyAsync(s->ver, u_dev, bytes, hipMemcpyDeviceToDevice, q));
    since = 0;
  }
  if (r == CGL_OK) r = dev(hipStreamSynchronize(q));
  if (stats)
    for (int k = 0; k < 4; ++k) stats[k] = st[k];
  return r;
}

}  // extern "C"
