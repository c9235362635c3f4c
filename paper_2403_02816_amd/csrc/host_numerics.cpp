// Host FP64 numerics: FD operators, Pade-13 matrix exponential, bf16 splitting.
#include "host_numerics.hpp"

#include <cmath>
#include <cstring>
#include <limits>

namespace cgl {

CMat CMat::identity(int64_t n) {
  CMat I(n);
  for (int64_t i = 0; i < n; ++i) I.re[i + n * i] = 1.0;
  return I;
}

CMat CMat::from_interleaved(int64_t n, const double* z) {
  CMat M(n);
  for (int64_t k = 0; k < n * n; ++k) {
    M.re[k] = z[2 * k];
    M.im[k] = z[2 * k + 1];
  }
  return M;
}

void CMat::to_interleaved(double* z) const {
  for (int64_t k = 0; k < n * n; ++k) {
    z[2 * k] = re[k];
    z[2 * k + 1] = im[k];
  }
}

double CMat::norm1() const {
  double best = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += std::hypot(re[i + n * j], im[i + n * j]);
    if (s > best) best = s;
  }
  return best;
}

// C = A B, column by column: C(:, j) = sum_k A(:, k) B(k, j).  The inner loop
// runs down a column of A, which is contiguous.
void cmat_mul(const CMat& A, const CMat& B, CMat& C) {
  const int64_t n = A.n;
  C = CMat(n);
  for (int64_t j = 0; j < n; ++j) {
    double* cr = &C.re[n * j];
    double* ci = &C.im[n * j];
    for (int64_t k = 0; k < n; ++k) {
      const double br = B.re[k + n * j], bi = B.im[k + n * j];
      if (br == 0.0 && bi == 0.0) continue;
      const double* ar = &A.re[n * k];
      const double* ai = &A.im[n * k];
      for (int64_t i = 0; i < n; ++i) {
        cr[i] += ar[i] * br - ai[i] * bi;
        ci[i] += ar[i] * bi + ai[i] * br;
      }
    }
  }
}

static void axpy_into(CMat& Y, double s, const CMat& X) {  // Y += s X
  for (size_t k = 0; k < Y.re.size(); ++k) {
    Y.re[k] += s * X.re[k];
    Y.im[k] += s * X.im[k];
  }
}

// Solve P X = Q for X (P, Q complex n x n) by Gaussian elimination with
// partial pivoting.  Overwrites P and Q; X is returned in Q.
static bool solve_inplace(CMat& P, CMat& Q) {
  const int64_t n = P.n;
  std::vector<double>& pr = P.re;
  std::vector<double>& pi = P.im;
  for (int64_t c = 0; c < n; ++c) {
    int64_t piv = c;
    double best = -1.0;
    for (int64_t r = c; r < n; ++r) {
      const double m = std::hypot(pr[r + n * c], pi[r + n * c]);
      if (m > best) {
        best = m;
        piv = r;
      }
    }
    if (!(best > 0.0)) return false;
    if (piv != c) {
      for (int64_t j = 0; j < n; ++j) {
        std::swap(pr[c + n * j], pr[piv + n * j]);
        std::swap(pi[c + n * j], pi[piv + n * j]);
        std::swap(Q.re[c + n * j], Q.re[piv + n * j]);
        std::swap(Q.im[c + n * j], Q.im[piv + n * j]);
      }
    }
    const double dr = pr[c + n * c], di = pi[c + n * c];
    const double dd = dr * dr + di * di;
    const double ir = dr / dd, ii = -di / dd;  // 1 / pivot
    for (int64_t r = c + 1; r < n; ++r) {
      const double xr = pr[r + n * c], xi = pi[r + n * c];
      const double fr = xr * ir - xi * ii, fi = xr * ii + xi * ir;  // multiplier
      if (fr == 0.0 && fi == 0.0) continue;
      for (int64_t j = c; j < n; ++j) {
        const double ar = pr[c + n * j], ai = pi[c + n * j];
        pr[r + n * j] -= fr * ar - fi * ai;
        pi[r + n * j] -= fr * ai + fi * ar;
      }
      for (int64_t j = 0; j < n; ++j) {
        const double ar = Q.re[c + n * j], ai = Q.im[c + n * j];
        Q.re[r + n * j] -= fr * ar - fi * ai;
        Q.im[r + n * j] -= fr * ai + fi * ar;
      }
    }
  }
  // back substitution, one right-hand-side column at a time
  for (int64_t j = 0; j < n; ++j) {
    for (int64_t r = n - 1; r >= 0; --r) {
      double sr = Q.re[r + n * j], si = Q.im[r + n * j];
      for (int64_t k = r + 1; k < n; ++k) {
        const double ar = pr[r + n * k], ai = pi[r + n * k];
        const double xr = Q.re[k + n * j], xi = Q.im[k + n * j];
        sr -= ar * xr - ai * xi;
        si -= ar * xi + ai * xr;
      }
      const double dr = pr[r + n * r], di = pi[r + n * r];
      const double dd = dr * dr + di * di;
      Q.re[r + n * j] = (sr * dr + si * di) / dd;
      Q.im[r + n * j] = (si * dr - sr * di) / dd;
    }
  }
  return true;
}

// Coefficients of the [m/m] Pade approximant of exp, normalised so b_m = 1:
// b_j = (2m - j)! / (j! (m - j)!), from p_j = (2m-j)! m! / ((2m)! j! (m-j)!).
static void pade_coeffs(int m, double* b) {
  for (int j = 0; j <= m; ++j) {
    long double v = 1.0L;
    for (int q = m - j + 1; q <= 2 * m - j; ++q) v *= q;  // (2m-j)!/(m-j)!
    for (int q = 2; q <= j; ++q) v /= q;                  // / j!
    b[j] = static_cast<double>(v);
  }
}

bool expm_pade13(const CMat& A0, double t, CMat& out) {
  const int64_t n = A0.n;
  CMat A = A0;
  for (size_t k = 0; k < A.re.size(); ++k) {
    A.re[k] *= t;
    A.im[k] *= t;
  }
  // theta_13: largest 1-norm for which the degree-13 approximant meets unit
  // roundoff in backward error (Higham 2005, Table 2.3).
  const double theta13 = 5.371920351148152;
  const double nrm = A.norm1();
  if (!std::isfinite(nrm)) return false;
  int s = 0;
  if (nrm > theta13) s = static_cast<int>(std::ceil(std::log2(nrm / theta13)));
  if (s > 0) {
    const double sc = std::ldexp(1.0, -s);
    for (size_t k = 0; k < A.re.size(); ++k) {
      A.re[k] *= sc;
      A.im[k] *= sc;
    }
  }
  double b[14];
  pade_coeffs(13, b);
  CMat A2, A4, A6;
  cmat_mul(A, A, A2);
  cmat_mul(A2, A2, A4);
  cmat_mul(A4, A2, A6);
  const CMat I = CMat::identity(n);
  // U = A [A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I]
  CMat T1(n);
  axpy_into(T1, b[13], A6);
  axpy_into(T1, b[11], A4);
  axpy_into(T1, b[9], A2);
  CMat W;
  cmat_mul(A6, T1, W);
  axpy_into(W, b[7], A6);
  axpy_into(W, b[5], A4);
  axpy_into(W, b[3], A2);
  axpy_into(W, b[1], I);
  CMat U;
  cmat_mul(A, W, U);
  // V = A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I
  CMat T2(n);
  axpy_into(T2, b[12], A6);
  axpy_into(T2, b[10], A4);
  axpy_into(T2, b[8], A2);
  CMat V;
  cmat_mul(A6, T2, V);
  axpy_into(V, b[6], A6);
  axpy_into(V, b[4], A4);
  axpy_into(V, b[2], A2);
  axpy_into(V, b[0], I);
  // (V - U) R = (V + U)
  CMat P = V, Q = V;
  axpy_into(P, -1.0, U);
  axpy_into(Q, 1.0, U);
  if (!solve_inplace(P, Q)) return false;
  // undo the scaling: R <- R^(2^s)
  CMat R = Q, tmp;
  for (int k = 0; k < s; ++k) {
    cmat_mul(R, R, tmp);
    R.re.swap(tmp.re);
    R.im.swap(tmp.im);
  }
  out = R;
  for (size_t k = 0; k < out.re.size(); ++k)
    if (!std::isfinite(out.re[k]) || !std::isfinite(out.im[k])) return false;
  return true;
}

CMat fd_operator_2nd(int64_t n, double a, double b, int bc, double a1, double b1, double a2,
                     int d) {
  const double h = (bc == 0) ? (b - a) / double(n + 1) : (b - a) / double(n - 1);
  const double ih2 = 1.0 / (h * h);
  CMat A(n);
  auto set = [&](int64_t i, int64_t j, double v) {
    A.re[i + n * j] += a1 * v * ih2;
    A.im[i + n * j] += b1 * v * ih2;
  };
  for (int64_t i = 0; i < n; ++i) {
    set(i, i, -2.0);
    if (i > 0) set(i, i - 1, 1.0);
    if (i < n - 1) set(i, i + 1, 1.0);
  }
  if (bc == 1) {  // Neumann: ghost value from the centred u' = 0 doubles the inner neighbour
    set(0, 1, 1.0);
    set(n - 1, n - 2, 1.0);
  }
  for (int64_t i = 0; i < n; ++i) A.re[i + n * i] += a2 / double(d);
  return A;
}

bool fd_operator(int64_t n, double a, double b, int bc_lo, int bc_hi, int order, double a1,
                 double b1, double a2, int d, CMat& A) {
  if ((bc_lo != 0 && bc_lo != 1) || (bc_hi != 0 && bc_hi != 1)) return false;
  if (order != 2 && order != 4) return false;
  if (n < (order == 4 ? 6 : 3)) return false;
  // a Dirichlet end is not a node, a Neumann end is the first / last node
  const int ends = (bc_lo == 1) + (bc_hi == 1);
  const double h = (b - a) / double(n + 1 - ends);
  std::vector<double> D(static_cast<size_t>(n * n), 0.0);  // column-major
  auto at = [&](int64_t i, int64_t j) -> double& { return D[static_cast<size_t>(i + n * j)]; };
  double scale;
  if (order == 2) {
    for (int64_t i = 0; i < n; ++i) {
      at(i, i) = -2.0;
      if (i > 0) at(i, i - 1) = 1.0;
      if (i < n - 1) at(i, i + 1) = 1.0;
    }
    // Neumann end: the ghost value of the centred u' = 0 doubles the inner neighbour
    if (bc_lo == 1) at(0, 1) = 2.0;
    if (bc_hi == 1) at(n - 1, n - 2) = 2.0;
    scale = 1.0 / (h * h);
  } else {
    // Sections 4.1.1 and 4.2: centred five-point rows (a Dirichlet boundary
    // value, 0, drops out); next to a Dirichlet end the one-sided six-point
    // row whose boundary weight multiplies that zero; at a Neumann end the
    // two modified rows of the semi-internal grid.  The left end mirrors the
    // right one (column order reversed).
    static const double kCentre[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};
    static const double kNextToDirichlet[5] = {-15.0, -4.0, 14.0, -6.0, 1.0};  // from the end inwards
    static const double kBeforeNeumannEnd[6] = {10.0, -15.0, -4.0, 14.0, -6.0, 1.0};
    static const double kNeumannEnd[5] = {-145.0 / 3.0, 56.0, -6.0, -8.0 / 3.0, 1.0};
    for (int64_t i = 0; i < n; ++i)
      for (int k = -2; k <= 2; ++k)
        if (i + k >= 0 && i + k < n) at(i, i + k) = kCentre[k + 2];
    auto clear_row = [&](int64_t i) {
      for (int64_t j = 0; j < n; ++j) at(i, j) = 0.0;
    };
    // right end: column n-1-k takes entry k of a table written from the end inwards
    if (bc_hi == 0) {
      clear_row(n - 1);
      for (int k = 0; k < 5; ++k) at(n - 1, n - 1 - k) = kNextToDirichlet[k];
    } else {
      clear_row(n - 2);
      clear_row(n - 1);
      for (int k = 0; k < 6; ++k) at(n - 2, n - 1 - k) = kBeforeNeumannEnd[k];
      for (int k = 0; k < 5; ++k) at(n - 1, n - 1 - k) = kNeumannEnd[k];
    }
    // left end: column k
    if (bc_lo == 0) {
      clear_row(0);
      for (int k = 0; k < 5; ++k) at(0, k) = kNextToDirichlet[k];
    } else {
      clear_row(1);
      clear_row(0);
      for (int k = 0; k < 6; ++k) at(1, k) = kBeforeNeumannEnd[k];
      for (int k = 0; k < 5; ++k) at(0, k) = kNeumannEnd[k];
    }
    scale = 1.0 / (12.0 * h * h);
  }
  A = CMat(n);
  for (size_t q = 0; q < D.size(); ++q) {
    A.re[q] = a1 * (D[q] * scale);
    A.im[q] = b1 * (D[q] * scale);
  }
  for (int64_t i = 0; i < n; ++i) A.re[i + n * i] += a2 / double(d);
  return true;
}

void fourier_factors(int64_t n, double a, double b, double a1, double b1, double a2, int d,
                     double t, std::vector<double>& fac, double adv) {
  const double two_pi = 6.283185307179586476925286766559;
  fac.assign(static_cast<size_t>(2 * n), 0.0);
  for (int64_t q = 0; q < n; ++q) {
    const double wave = two_pi * static_cast<double>(q <= n / 2 ? q : q - n) / (b - a);
    const double k2 = wave * wave;
    const double k1 = (n % 2 == 0 && q == n / 2) ? 0.0 : wave;
    // t ((a1 + i b1)(-k^2) + adv i k' + a2/d)
    const double re = t * (-a1 * k2 + a2 / d), im = t * (-b1 * k2 + adv * k1);
    const double m = std::exp(re);
    fac[2 * q] = m * std::cos(im);
    fac[2 * q + 1] = m * std::sin(im);
  }
}

// angle 2 pi r / n for an integer r reduced modulo n
static void unit_root(int64_t r, int64_t n, double& c, double& s) {
  const double two_pi = 6.283185307179586476925286766559;
  const int64_t q = ((r % n) + n) % n;
  const double th = two_pi * static_cast<double>(q) / static_cast<double>(n);
  c = std::cos(th);
  s = std::sin(th);
}

CMat circulant_from_factors(int64_t n, const std::vector<double>& fac) {
  // C[j, l] = c[(j - l) mod n], c[r] = (1/n) sum_q fac_q exp(2 pi i q r / n)
  std::vector<double> cr(static_cast<size_t>(n)), ci(static_cast<size_t>(n));
  for (int64_t r = 0; r < n; ++r) {
    double sr = 0.0, si = 0.0;
    for (int64_t q = 0; q < n; ++q) {
      double co, so;
      unit_root(q * r, n, co, so);
      sr += fac[2 * q] * co - fac[2 * q + 1] * so;
      si += fac[2 * q] * so + fac[2 * q + 1] * co;
    }
    cr[r] = sr / static_cast<double>(n);
    ci[r] = si / static_cast<double>(n);
  }
  CMat C(n);
  for (int64_t l = 0; l < n; ++l)
    for (int64_t j = 0; j < n; ++j) {
      const int64_t r = ((j - l) % n + n) % n;
      C.re[j + n * l] = cr[r];
      C.im[j + n * l] = ci[r];
    }
  return C;
}

void fft_twiddles(int64_t n, std::vector<double>& tw) {
  tw.assign(static_cast<size_t>(2 * n), 0.0);
  for (int64_t q = 0; q < n; ++q) {
    double c, s;
    unit_root(q, n, c, s);
    tw[2 * q] = c;
    tw[2 * q + 1] = -s;
  }
}

uint16_t f32_to_bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) {  // Inf / NaN: truncate, keep NaN quiet
    uint16_t h = static_cast<uint16_t>(u >> 16);
    if (u & 0x007fffffu) h |= 0x0040;
    return h;
  }
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return static_cast<uint16_t>(u >> 16);
}

float bf16_to_f32(uint16_t h) {
  const uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

void split_bf16(double x, int k, uint16_t* terms) {
  double r = x;
  for (int i = 0; i < k; ++i) {
    // round the remainder to float first (exact for the bf16 range of
    // interest), then to bf16; the remainder update is exact in double
    const uint16_t h = f32_to_bf16_rne(static_cast<float>(r));
    terms[i] = h;
    r -= static_cast<double>(bf16_to_f32(h));
  }
}

}  // namespace cgl
