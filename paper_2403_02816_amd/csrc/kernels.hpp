// Device-side interfaces of the mu-mode product kernels (internal to libcgl).
//
// One pass computes out = in x_mu M for one direction mu of a column-major
// (index 1 fastest) complex tensor.  With R = n_1...n_{mu-1} and n = n_mu,
// fibre f = (r, b) (r = f mod R, b = f div R) starts at complex offset
// r + b R n and steps by R; F = N / n fibres.  Input and output may use
// different R: the exponential actions of the time steppers run every pass
// on a tensor whose contraction axis is the fastest one (R_in = 1) and write
// its result with that axis moved to the slowest position (R_out = F), so
// after d passes the axis order is the original one again.  The complex product is run as
// the real product of the 2n x 2n block embedding
//   [[Re M, -Im M], [Im M, Re M]]
// with real rows/columns interleaved (2m + c, c = 0 real, 1 imaginary), so that
// a complex number's two parts sit in adjacent rows of the MFMA accumulators.
//
// Pointwise work of the time steppers is fused into the first pass (prologue,
// applied to the input as it is staged) and the last pass (epilogue, applied
// to the accumulators before the store).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cgl {

// prologue codes (first pass of an exponential action); t = NlParams::tf
enum Prologue : int {
  PRO_NONE = 0,
  PRO_FLOW = 1,  // x <- phi_t(x) (the sub-flow entering a splitting step)
  PRO_G = 2,     // x <- g(x)                                    (Lawson: Q = e^{s K} g(u))
};

// epilogue codes (last pass of an exponential action); "aux" is a second
// tensor read at the same grid point; t = NlParams::tf
enum Epilogue : int {
  EPI_NONE = 0,
  EPI_FLOW = 1,   // y <- phi_t(y) (the sub-flow leaving a splitting step), check finite
  EPI_L4_R1 = 2,  // acc = Q, aux = P:  out0 <- X, out1 <- Y        (Lawson4 round 1)
  EPI_L4_R2 = 3,  // acc = H Y, aux = H X:  out0 <- H Y + tau/6 g(H X), check finite
  EPI_MID = 4,    // y <- the sub-flow between the two half steps of split4, check finite
  EPI_RICH = 5,   // out0 <- 4/3 phi_t(y) - 1/3 aux (split4), check finite
  EPI_L2 = 6,     // acc = Q = E g(u), aux = P = E u:  out0 <- P + tau/2 Q + tau/2 g(P + tau Q)
};

// sub-flow of the splitting schemes
enum FlowKind : int {
  FLOW_RK4 = 0,    // one classical RK4 step of u' = g(u)
  FLOW_EXACT = 1,  // the exact cubic flow (eq. exsolcub), a4 = b4 = 0
  FLOW_3T = 2,     // exact cubic and exact quintic flows in sequence (three-term splitting)
};

// latched device conditions
enum : unsigned { FLAG_NONFINITE = 1u, FLAG_BLOWUP = 2u };

struct NlParams {
  double tau;  // full step
  double tf;   // time of the sub-flows of this pass (PRO_FLOW, EPI_FLOW, EPI_MID, EPI_RICH)
  double a3, b3, a4, b4;
  int flow;    // FlowKind
};

// FP64 pass: complex128 tensors, FP64 operator embedding.
struct PassF64 {
  const double* in0;
  const double* aux;
  double* out0;
  double* out1;
  const double* op;  // embedding, rows k' (Kp of them), p' fastest (Pp per row)
  int64_t R;
  int64_t F;
  int n;
  int Pp;
  int Kp;
  int pro;
  int epi;
  NlParams nl;
  unsigned* flag;
};

// FP64 kernel tiling (see kernels_f64.hip)
constexpr int F64_PT = 64;  // real output rows per workgroup
constexpr int F64_FT = 64;  // fibres per workgroup
constexpr int F64_KC = 16;  // real contraction rows per LDS stage

hipError_t launch_pass_f64(const PassF64& a, hipStream_t s);
hipError_t launch_clear_flag(unsigned* flag, hipStream_t s);

// Split-precision pass: complex64 stage tensors (optionally complex128 master
// state at the pass ends), bf16 operator terms, FP32 accumulation.
struct PassSplit {
  const void* in0;
  const void* in1;  // paired pass: the second action's input (see launch_pass_split_pair)
  const void* aux;  // complex64 stage tensor, in the output's layout
  void* out0;
  void* out1;
  const uint16_t* op;  // bf16 terms of the embedding, see kernels_split.hip
  int64_t R;       // input: contraction stride
  int64_t R_out;   // output: contraction stride
  int64_t F;
  int n;
  int Pp;
  int Kp;
  int pro;
  int epi;
  int in_f64;   // in0 is complex128 (master state) instead of complex64
  int out_f64;  // out0/out1 are complex128
  int aux_f64;  // aux is complex128 (EPI_RICH of a master-state plan)
  int tile;     // index into SPLIT_TILES (the operator planes must match it)
  NlParams nl;
  unsigned* flag;
  // split contraction (direct-to-LDS shapes; ksplit <= 1: off): ksplit <= 4
  // workgroups per tile, kchunk stages each (every split gets at least one
  // stage), partial accumulators in ws (ws_floats floats: at least
  // ksplit x tiles x PT / 64 x 8192)
  int ksplit;
  int kchunk;
  float* ws;
  int64_t ws_floats;
};

constexpr int SP_FT = 64;    // fibres per workgroup (rows/stage sizes: split_layout.hpp)
constexpr int SPLIT_MAX_TILES = 4;
constexpr int SP_TERMS = 3;  // bf16 terms per operand

hipError_t launch_pass_split(const PassSplit& a, hipStream_t s);
// One direction of both actions of a Lawson4 round (64 x 16 direct-to-LDS
// operator planes): out0 <- M in0, out1 <- M in1, or with pro == PRO_G out1
// <- M g(in0); epi EPI_NONE, EPI_L4_R1 (out0 = X, out1 = Y) or EPI_L4_R2
// (out0 = u_{n+1}).
hipError_t launch_pass_split_pair(const PassSplit& a, hipStream_t s);

// ---- batched split-precision passes (many independent instances)
struct BatchInstance {
  int64_t off;  // complex offset of the instance in every batched tensor
  int n;        // contraction length of this pass
  int F;        // fibres of this pass
  int Pp[SPLIT_MAX_TILES];
  int Kp[SPLIT_MAX_TILES];
  const uint16_t* opE[SPLIT_MAX_TILES];  // bf16 planes of exp(tau A) per tile shape
  const uint16_t* opH[SPLIT_MAX_TILES];  // and of exp(tau A / 2)
  NlParams nl;
};

struct BatchTile {
  int inst, pt, ft;  // inst < 0: a padding entry (no work)
};

struct PassBatch {
  const void* in0;
  const void* in1;  // paired pass: the second action's input
  const void* aux;
  void* out0;
  void* out1;
  const BatchInstance* inst;  // device table for this pass direction
  const BatchTile* tiles;     // device list, largest instances first
  int ntiles;
  int which;  // 0: E, 1: H
  int pro;
  int epi;
  int in_f64;
  int out_f64;
  int aux_f64;
  int tile;  // tile shape (index into SPLIT_TILES)
  double tf;  // sub-flow time of this pass (every instance shares tau)
  unsigned* flag;
};

// ---- Fourier pass of a periodic direction (kernels_fft.hip): every fibre
// goes through F^{-1} diag(fac) F (lengths n = 2^k, 8 <= n <= 1024), with the
// same prologue / epilogue codes and layouts as the mu-mode products.
struct PassFFT {
  const void* in0;
  const void* aux;
  void* out0;
  void* out1;
  const void* fac;   // n complex factors: double2 (fp64 passes) or float2
  const double* tw;  // n complex128 twiddles exp(-2 pi i q / n)
  int64_t R;         // input: fibre stride
  int64_t R_out;     // output: fibre stride
  int64_t F;
  int n;
  int pro;
  int epi;
  int in_f64;
  int out_f64;
  int aux_f64;
  int fp64;          // arithmetic and stage tensors in FP64 (else FP32 / complex64)
  NlParams nl;
  unsigned* flag;
};
bool fft_length_supported(int64_t n);
hipError_t launch_pass_fft(const PassFFT& a, hipStream_t s);

// launches a persistent grid of at most nwg workgroups over b.tiles
hipError_t launch_pass_split_batched(const PassBatch& b, int nwg, hipStream_t s);
// the paired pass (see launch_pass_split_pair) over every instance: b.tile
// must be the 64 x 16 direct-to-LDS shape, b.pro PRO_G (the second product
// reads g(in0)) or PRO_NONE (in0 and in1)
hipError_t launch_pass_split_batched_pair(const PassBatch& b, int nwg, hipStream_t s);

}  // namespace cgl
