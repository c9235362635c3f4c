// Host-side FP64 numerics of the plan: finite-difference operators, the
// matrix exponential of the small 1-D operators, bf16 term splitting and the
// real block embedding of complex operators used by the device kernels.
#pragma once

#include <cstdint>
#include <vector>

namespace cgl {

// Complex n x n matrix, column-major, stored as separate real and imaginary
// planes (element (i, j) at i + n*j).
struct CMat {
  int64_t n = 0;
  std::vector<double> re, im;
  CMat() = default;
  explicit CMat(int64_t n_) : n(n_), re(n_ * n_, 0.0), im(n_ * n_, 0.0) {}
  static CMat identity(int64_t n);
  static CMat from_interleaved(int64_t n, const double* z);  // complex128 col-major
  void to_interleaved(double* z) const;
  double norm1() const;  // max column sum of |a_ij|
};

void cmat_mul(const CMat& A, const CMat& B, CMat& C);  // C = A B (C must not alias)

// exp(t A) by the [13/13] Pade approximant with scaling and squaring
// (Higham, SIAM J. Matrix Anal. Appl. 26 (2005); the Pade route the paper cites
// for its small exponentials).  Returns false on a singular denominator.
bool expm_pade13(const CMat& A, double t, CMat& out);

// 2nd-order central FD operator A = (a1 + i b1) D2 + (a2/d) I (see cgl.h).
CMat fd_operator_2nd(int64_t n, double a, double b, int bc, double a1, double b1, double a2,
                     int d);

// FD operator of order 2 or 4 with a Dirichlet (0) or Neumann (1) condition at
// each end (see cgl_fd_operator_ex in cgl.h).  Returns false for an order or
// size it does not support.
bool fd_operator(int64_t n, double a, double b, int bc_lo, int bc_hi, int order, double a1,
                 double b1, double a2, int d, CMat& A);

// Periodic direction on (a, b) with n equispaced nodes (Section 3.2): the
// diagonal of exp(t A_mu), A_mu = (a1 + i b1)(-k^2) + adv (i k') + a2/d over
// the wave numbers k = 2 pi q / (b - a), q = 0, 1, .., n/2, -n/2 + 1, .., -1
// in the transform's coefficient order; k' = k except k' = 0 for the Nyquist
// mode of an even n (the first derivative of the coupled system's advection
// term, Section 4.4); interleaved complex128 (2n doubles).
void fourier_factors(int64_t n, double a, double b, double a1, double b1, double a2, int d,
                     double t, std::vector<double>& fac, double adv = 0.0);
// The same exponential as a dense circulant matrix on grid values,
// F^{-1} diag(fac) F.
CMat circulant_from_factors(int64_t n, const std::vector<double>& fac);
// exp(-2 pi i q / n), q < n, interleaved complex128.
void fft_twiddles(int64_t n, std::vector<double>& tw);

// Round-to-nearest-even float -> bf16 bits and back.
uint16_t f32_to_bf16_rne(float x);
float bf16_to_f32(uint16_t h);

// Split a double into k bf16 terms t_0 + t_1 + ... (each term is the bf16
// rounding of what the previous terms left over).
void split_bf16(double x, int k, uint16_t* terms);

}  // namespace cgl
