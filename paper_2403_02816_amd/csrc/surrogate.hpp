// Residual CNN surrogate of the stepper (device side).
//
// Network (C = 48 channels, 3x3 kernels, zero padding, pixel p = i1 + n1 i2,
// activations FP32 [sample][channel][pixel]):
//   x = [Re u, Im u, 5 standardised coefficient planes]            (7 channels)
//   h0 = silu(conv_in x);  h_k = h_{k-1} + silu(conv_k h_{k-1}), k = 1..4
//   y  = (Re u, Im u) + conv_out h_4                               (2 channels)
// Convolutions run on BF16 MFMA (weights and activations rounded to bf16,
// FP32 accumulation) as implicit GEMMs: out[co, p] = sum_k W[co, k] X[k, p]
// with k = tap * cin_pad + ci.  The transposed convolution of the backward
// pass is the same kernel with transposed, tap-flipped weights.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cgl {

constexpr int SUR_C = 48;
constexpr int SUR_BLOCKS = 4;
constexpr int SUR_CIN = 7;
constexpr int SUR_LAYERS = SUR_BLOCKS + 2;

enum ConvEpi : int {
  CEPI_SILU = 1,  // out0 = a = conv + b, out1 = silu(a)
  CEPI_RES = 2,   // out0 = a = conv + b, out1 = aux + silu(a)      (aux = h_prev)
  CEPI_OUT = 3,   // out0 = aux[channels 0,1] + oscale (conv + b)    (aux = base planes)
  CEPI_BWD = 4,   // out0 = conv (+ aux), out1 = out0 * silu'(aux2)  (transposed conv)
};

struct ConvArgs {
  const float* x;     // [S][cin][P]
  const uint16_t* w;  // bf16 [cout_pad][kpad], k = tap * cin_pad + ci, tap = 3 ky + kx
  const float* bias;  // [cout] (may be null)
  float* out0;        // [S][cout][P]
  float* out1;        // [S][cout][P] (may be null for CEPI_OUT / CEPI_BWD without aux2)
  const float* aux;   // see ConvEpi
  const float* aux2;
  int cin, cout, n1, n2, S;
  int epi;
  int aux_ch;  // channel count of aux's samples (CEPI_OUT: network input channels)
  float oscale;  // CEPI_OUT: scale of the network's correction
};

// cin_pad in {8, 48}, cout_pad in {16, 48}; requires n1 % 64 == 0
hipError_t launch_conv(const ConvArgs& a, int cin_pad, int cout_pad, hipStream_t s);
int conv_kpad(int cin_pad);

struct WgradArgs {
  const float* x;     // layer input [S][cin][P]
  const float* dout;  // gradient of the layer's pre-activation output [S][cout][P]
  int cin, cout, n1, n2, S;
};
// Workgroups of the weight-gradient kernel; part holds wgrad_grid(...) * L
// floats, L = cout * cin * 9 + cout.  grad (L floats, parameter order
// W[co][ci][ky][kx] then b[co]) is overwritten.
int wgrad_grid(int S, int n1, int n2);
hipError_t launch_wgrad(const WgradArgs& a, float* part, float* grad, hipStream_t s);

// x[s] = [Re u, Im u, cstd planes] of source sample idx[s] (idx null: s);
// u complex64 [*][P], cstd [*][5]
hipError_t launch_sur_pack(const void* u, const int* idx, const float* cstd, float* x, int S,
                           int64_t P, hipStream_t s);
// xb[s] = [Re b, Im b] of base sample idx[s] (idx null: s); b complex64 [*][P]
hipError_t launch_sur_pack_base(const void* b, const int* idx, float* xb, int S, int64_t P,
                                hipStream_t s);
// out complex64 [S][P] from y [S][2][P]
hipError_t launch_sur_unpack(const float* y, void* out, int S, int64_t P, hipStream_t s);
// target of sample s: complex64 sample (idx[s] or s) + toff.  wbuf null: the
// mean square error; otherwise ([S] doubles of scratch) the mean over samples
// of the squared relative L2 error.  dy = dscale * d loss / dy (the gradient
// with respect to the unscaled correction when y = base + dscale * d),
// *loss += loss (FP64).
hipError_t launch_mse(const float* y, const void* target, const int* idx, int64_t toff,
                      double* wbuf, float dscale, float* dy, double* loss, int S, int64_t P,
                      hipStream_t s);
// Adam on FP32 parameters; c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t)
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int count, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s);
// bf16 forward and transposed, tap-flipped weight layouts of one layer from
// FP32 W[cout][cin][3][3] (wt may be null)
hipError_t launch_pack_weights(const float* W, int cout, int cin, uint16_t* wf, int cout_pad,
                               int cin_pad, uint16_t* wt, int cinT_pad, int coutT_pad,
                               hipStream_t s);
// acc[0] += sum |a - b|^2, acc[1] += sum |b|^2 over n complex64 values
hipError_t launch_diff_norms(const void* a, const void* b, int64_t n, double* acc, hipStream_t s);
hipError_t launch_zero(float* p, int64_t count, hipStream_t s);

}  // namespace cgl
