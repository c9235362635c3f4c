// Runs libcgl's host code and kernels on the CPU through the HIP emulation
// in this directory (built with AddressSanitizer by test_cpu_emulation.py).
// Checks every entry point for out-of-bounds accesses and checks the mode
// products / Tucker operator against a naive triple loop.
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <cmath>
#include <random>
#include <string>
#include <vector>

#include "../../include/cgl.h"

using cd = std::complex<double>;
static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL: %s\n", what);
    ++failures;
  }
}

static std::vector<cd> rnd(size_t n, unsigned seed, double scale = 1.0) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> d(0.0, 1.0);
  std::vector<cd> v(n);
  for (auto& x : v) x = cd(d(g), d(g)) * scale;
  return v;
}

// naive mode product, column-major tensor of shape n[0..d-1]
static std::vector<cd> mode_ref(const std::vector<cd>& U, const std::vector<int64_t>& n, int mu,
                                const std::vector<cd>& M) {
  int64_t R = 1, B = 1;
  for (int i = 0; i < mu; ++i) R *= n[i];
  for (size_t i = mu + 1; i < n.size(); ++i) B *= n[i];
  const int64_t nm = n[mu];
  std::vector<cd> Y(U.size());
  for (int64_t b = 0; b < B; ++b)
    for (int64_t i = 0; i < nm; ++i)
      for (int64_t r = 0; r < R; ++r) {
        cd s = 0.0;
        for (int64_t j = 0; j < nm; ++j) s += M[i + nm * j] * U[r + R * (j + nm * b)];
        Y[r + R * (i + nm * b)] = s;
      }
  return Y;
}

static double rel(const std::vector<cd>& a, const std::vector<cd>& b) {
  double num = 0, den = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    num += std::norm(a[i] - b[i]);
    den += std::norm(b[i]);
  }
  return std::sqrt(num / den);
}

template <class T>
static std::vector<std::complex<T>> cast(const std::vector<cd>& v) {
  std::vector<std::complex<T>> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = std::complex<T>(v[i]);
  return o;
}
template <class T>
static std::vector<cd> back(const std::vector<std::complex<T>>& v) {
  std::vector<cd> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = cd(v[i]);
  return o;
}

static void kernel_parity(std::vector<int64_t> n, int precision, unsigned seed) {
  const int d = static_cast<int>(n.size());
  int64_t N = 1;
  for (auto v : n) N *= v;
  cgl_coeffs c{1.0, 1.5, 0.5, -1.0, 1.0, 0.0, 0.0};
  cgl_plan_t p = nullptr;
  expect(cgl_plan(&p, d, n.data(), &c, 0.01, precision, 0, nullptr) == CGL_OK, "plan");
  std::vector<std::vector<cd>> Es, Hs;
  for (int mu = 0; mu < d; ++mu) {
    auto E = rnd(n[mu] * n[mu], seed + 10 * mu, 1.0 / std::sqrt(double(n[mu])));
    auto H = rnd(n[mu] * n[mu], seed + 10 * mu + 1, 1.0 / std::sqrt(double(n[mu])));
    expect(cgl_set_exponentials(p, mu, reinterpret_cast<double*>(E.data()),
                                reinterpret_cast<double*>(H.data())) == CGL_OK, "set_exponentials");
    Es.push_back(E);
    Hs.push_back(H);
  }
  auto U = rnd(N, seed + 99);
  const double tol = precision == CGL_FP64 ? 1e-13 : 1e-6;
  if (precision == CGL_SPLIT_BF16) U = back(cast<float>(U));
  for (int mu = 0; mu < d; ++mu) {
    std::vector<cd> out;
    if (precision == CGL_FP64) {
      std::vector<cd> y(N);
      expect(cgl_mode_product(p, mu, CGL_H, U.data(), y.data()) == CGL_OK, "mode_product");
      out = y;
    } else {
      auto u32 = cast<float>(U);
      std::vector<std::complex<float>> y(N);
      expect(cgl_mode_product(p, mu, CGL_H, u32.data(), y.data()) == CGL_OK, "mode_product");
      out = back(y);
    }
    const double e = rel(out, mode_ref(U, n, mu, Hs[mu]));
    std::printf("  mode_product prec=%d d=%d mu=%d rel=%.2e\n", precision, d, mu, e);
    expect(e < tol, "mode product parity");
  }
  // Tucker in place
  std::vector<cd> ref = U;
  for (int mu = 0; mu < d; ++mu) ref = mode_ref(ref, n, mu, Es[mu]);
  std::vector<cd> out;
  if (precision == CGL_FP64) {
    std::vector<cd> y = U;
    expect(cgl_tucker(p, CGL_E, y.data(), y.data()) == CGL_OK, "tucker");
    out = y;
  } else {
    auto y = cast<float>(U);
    expect(cgl_tucker(p, CGL_E, y.data(), y.data()) == CGL_OK, "tucker");
    out = back(y);
  }
  const double e = rel(out, ref);
  std::printf("  tucker prec=%d d=%d rel=%.2e\n", precision, d, e);
  expect(e < 4 * tol, "tucker parity");
  // the allocation-free variant (intermediates in the library's fixed
  // scratch) gives the same bits, out of place and in place
  if (precision == CGL_FP64) {
    std::vector<cd> y = U, z(U.size());
    expect(cgl_tucker_noalloc(p, CGL_E, y.data(), z.data()) == CGL_OK, "tucker noalloc");
    expect(std::memcmp(z.data(), out.data(), z.size() * sizeof(cd)) == 0, "noalloc == tucker");
    expect(cgl_tucker_noalloc(p, CGL_E, y.data(), y.data()) == CGL_OK, "tucker noalloc in place");
    expect(std::memcmp(y.data(), out.data(), y.size() * sizeof(cd)) == 0, "noalloc in place");
  } else {
    auto y = cast<float>(U);
    std::vector<std::complex<float>> z(U.size());
    expect(cgl_tucker_noalloc(p, CGL_E, y.data(), z.data()) == CGL_OK, "tucker noalloc");
    expect(back(z) == out, "noalloc == tucker");
  }
  cgl_destroy(p);
}

// Periodic directions (Fourier pass for power-of-two n, the dense circulant
// exponential otherwise): the Tucker operator against naive mode products
// with the plan's dense exponentials, then every stepper.
static void fourier_parity(std::vector<int64_t> n, int precision, unsigned seed,
                           unsigned flags = 0) {
  const int d = static_cast<int>(n.size());
  int64_t N = 1;
  for (auto v : n) N *= v;
  cgl_coeffs c{1.0, 0.6, -0.2, -1.0, 0.8, -0.1, -0.3};
  cgl_plan_t p = nullptr;
  expect(cgl_plan(&p, d, n.data(), &c, 0.01, precision, flags, nullptr) == CGL_OK, "plan");
  std::vector<std::vector<cd>> Es(d);
  for (int mu = 0; mu < d; ++mu) {
    expect(cgl_set_periodic(p, mu, -3.0, 4.0) == CGL_OK, "set_periodic");
    Es[mu].resize(n[mu] * n[mu]);
    expect(cgl_get_operator(p, mu, CGL_E, reinterpret_cast<double*>(Es[mu].data())) == CGL_OK, "get");
  }
  auto U = rnd(N, seed);
  std::vector<cd> ref = U;
  for (int mu = 0; mu < d; ++mu) ref = mode_ref(ref, n, mu, Es[mu]);
  std::vector<cd> out;
  if (precision == CGL_FP64) {
    std::vector<cd> y(U.size());
    expect(cgl_tucker(p, CGL_E, U.data(), y.data()) == CGL_OK, "tucker");
    out = y;
  } else {
    auto x = cast<float>(U);
    std::vector<std::complex<float>> y(U.size());
    expect(cgl_tucker(p, CGL_E, x.data(), y.data()) == CGL_OK, "tucker");
    out = back(y);
  }
  const double e = rel(out, ref), tol = precision == CGL_FP64 ? 1e-12 : 2e-6;
  std::printf("  fourier tucker prec=%d d=%d rel=%.2e\n", precision, d, e);
  expect(e < tol, "fourier tucker parity");
  auto V = rnd(N, seed + 1, 0.3);
  std::vector<cd> v64 = V;
  std::vector<std::complex<float>> v32 = cast<float>(V);
  const bool wide = precision == CGL_FP64 || (flags & CGL_FLAG_FP64_MASTER);
  void* u = wide ? static_cast<void*>(v64.data()) : static_cast<void*>(v32.data());
  for (int m : {CGL_STRANG, CGL_LAWSON4, CGL_SPLIT4, CGL_LAWSON2})
    expect(cgl_step(p, m, u, 1) == CGL_OK, "fourier step");
  expect(cgl_run(p, CGL_LAWSON4, u, 2, 1) == CGL_OK, "fourier run");
  expect(cgl_status(p) == CGL_OK, "fourier status");
  cgl_destroy(p);
}

// The coupled two-field system: every method on Fourier and dense-circulant
// directions; checks that the state stays finite and that with a0 = a5 = 0
// that mirrored fields stay each other's mirror image (the system is
// symmetric under x1 -> L - x1 with u and v swapped), which checks the
// per-field indexing (u at [0, N), v at [N, 2N)) and the advection signs.
static void coupled(std::vector<int64_t> n, int precision, unsigned seed) {
  const int64_t N = n[0] * n[1];
  cgl_coupled_coeffs c{-0.4, 0.125, 0.5, -0.9, 1.0, 0.8, -0.1, -0.6, 0.5};
  cgl_coupled_t p = nullptr;
  expect(cgl_coupled_plan(&p, n.data(), &c, 0.01, precision, nullptr) == CGL_OK, "coupled plan");
  std::vector<double> fac(2 * n[0]);
  expect(cgl_coupled_get_factor(p, 0, 0, CGL_E, fac.data()) == CGL_ENOTREADY ||
             cgl_coupled_step(p, CGL_STRANG, fac.data(), 1) == CGL_ENOTREADY,
         "coupled not ready");
  for (int mu = 0; mu < 2; ++mu)
    expect(cgl_coupled_set_periodic(p, mu, 0.0, 7.0 * (2 - mu)) == CGL_OK, "coupled periodic");
  expect(cgl_coupled_get_factor(p, 1, 0, CGL_H, fac.data()) == CGL_OK, "coupled factor");
  // u and its mirror image x1 -> L - x1 (node j -> -j mod n1) as v
  auto U = rnd(N, seed, 0.5);
  std::vector<cd> W(2 * N);
  for (int64_t j2 = 0; j2 < n[1]; ++j2)
    for (int64_t j1 = 0; j1 < n[0]; ++j1) {
      W[j1 + n[0] * j2] = U[j1 + n[0] * j2];
      W[N + j1 + n[0] * j2] = U[(n[0] - j1) % n[0] + n[0] * j2];
    }
  std::vector<std::complex<float>> W32 = cast<float>(W);
  void* w = precision == CGL_FP64 ? static_cast<void*>(W.data()) : static_cast<void*>(W32.data());
  for (int m : {CGL_STRANG, CGL_LAWSON4, CGL_SPLIT4, CGL_LAWSON2})
    expect(cgl_coupled_step(p, m, w, 1) == CGL_OK, "coupled step");
  expect(cgl_coupled_status(p) == CGL_OK, "coupled status");
  expect(cgl_coupled_step(p, 7, w, 1) == CGL_EINVAL, "coupled bad method");
  std::vector<cd> out = precision == CGL_FP64 ? W : back(W32);
  double worst = 0.0, mx = 0.0;
  for (int64_t j2 = 0; j2 < n[1]; ++j2)
    for (int64_t j1 = 0; j1 < n[0]; ++j1) {
      const cd u = out[j1 + n[0] * j2], v = out[N + (n[0] - j1) % n[0] + n[0] * j2];
      worst = std::max(worst, std::abs(u - v));
      mx = std::max(mx, std::abs(u));
    }
  std::printf("  coupled prec=%d n=%lldx%lld mirror %.2e (max %.2e)\n", precision,
              static_cast<long long>(n[0]), static_cast<long long>(n[1]), worst, mx);
  expect(std::isfinite(mx) && mx > 0.0, "coupled finite");
  expect(worst < (precision == CGL_FP64 ? 1e-12 : 1e-5) * mx, "coupled mirror symmetry");
  cgl_coupled_destroy(p);
}

// The coupled split form with its long dense directions' contractions split
// over workgroups (partial products reduced in split order) against the
// same steps with the split turned off (CGL_KSPLIT=0 at plan creation), for
// both direct-to-LDS tile shapes (the only ones that split).
static void coupled_ksplit(std::vector<int64_t> n, unsigned seed, bool full = true) {
  const int64_t N = n[0] * n[1];
  cgl_coupled_coeffs c{-0.4, 0.125, 0.5, -0.9, 1.0, 0.8, -0.1, -0.6, 0.5};
  auto U = rnd(2 * N, seed, 0.5);
  const char* tile0 = std::getenv("CGL_SPLIT_TILE");
  const std::string saved = tile0 ? tile0 : "";
  for (const char* tile : {"2", "3"}) {
    if (!full && tile[0] == '3') break;  // smoke mode: the 64-row shape only
    setenv("CGL_SPLIT_TILE", tile, 1);
    std::vector<std::complex<float>> res[2];
    for (int off = 0; off < 2; ++off) {
      if (off) setenv("CGL_KSPLIT", "0", 1);
      cgl_coupled_t p = nullptr;
      expect(cgl_coupled_plan(&p, n.data(), &c, 0.01, CGL_SPLIT_BF16, nullptr) == CGL_OK,
             "ksplit plan");
      if (off) unsetenv("CGL_KSPLIT");
      for (int mu = 0; mu < 2; ++mu)
        expect(cgl_coupled_set_periodic(p, mu, 0.0, 7.0 * (2 - mu)) == CGL_OK, "ksplit periodic");
      res[off] = cast<float>(U);
      for (int m : {CGL_LAWSON4, CGL_STRANG}) {
        if (!full && m == CGL_STRANG) break;  // smoke mode: one Lawson4 step
        expect(cgl_coupled_step(p, m, res[off].data(), 1) == CGL_OK, "ksplit step");
      }
      expect(cgl_coupled_status(p) == CGL_OK, "ksplit status");
      cgl_coupled_destroy(p);
    }
    double worst = 0.0, mx = 0.0;
    for (int64_t i = 0; i < 2 * N; ++i) {
      worst = std::max(worst, static_cast<double>(std::abs(res[0][i] - res[1][i])));
      mx = std::max(mx, static_cast<double>(std::abs(res[1][i])));
    }
    std::printf("  coupled split contraction n=%lldx%lld tile %s: max diff %.2e (max %.2e)\n",
                static_cast<long long>(n[0]), static_cast<long long>(n[1]), tile, worst, mx);
    // the split sums the stages in another order: FP32 rounding, not bits
    expect(std::isfinite(mx) && mx > 0.0 && worst < 1e-5 * mx, "split contraction = unsplit");
    expect(worst > 0.0, "the contraction was split");
  }
  if (tile0)
    setenv("CGL_SPLIT_TILE", saved.c_str(), 1);
  else
    unsetenv("CGL_SPLIT_TILE");
}

static void steppers(std::vector<int64_t> n, int precision, unsigned flags, cgl_coeffs c,
                     double a, double b, int bc) {
  const int d = static_cast<int>(n.size());
  int64_t N = 1;
  for (auto v : n) N *= v;
  cgl_plan_t p = nullptr;
  expect(cgl_plan(&p, d, n.data(), &c, 0.005, precision, flags, nullptr) == CGL_OK, "plan");
  for (int mu = 0; mu < d; ++mu) {
    std::vector<cd> A(n[mu] * n[mu]);
    expect(cgl_fd_operator(n[mu], a, b, bc, &c, d, reinterpret_cast<double*>(A.data())) == CGL_OK,
           "fd");
    expect(cgl_set_operators(p, mu, reinterpret_cast<double*>(A.data())) == CGL_OK, "set_operators");
  }
  auto U = rnd(N, 7, 0.3);
  const bool c128 = precision == CGL_FP64 || (flags & CGL_FLAG_FP64_MASTER);
  std::vector<cd> u64 = U;
  std::vector<std::complex<float>> u32 = cast<float>(U);
  void* u = c128 ? static_cast<void*>(u64.data()) : static_cast<void*>(u32.data());
  expect(cgl_step_strang(p, u, 2) == CGL_OK, "strang");
  expect(cgl_step_lawson4(p, u, 2) == CGL_OK, "lawson4");
  expect(cgl_run(p, CGL_LAWSON4, u, 3, 2) == CGL_OK, "run lawson4");
  expect(cgl_run(p, CGL_STRANG, u, 3, 0) == CGL_OK, "run strang");
  expect(cgl_step(p, CGL_SPLIT4, u, 1) == CGL_OK, "split4");
  expect(cgl_step(p, CGL_LAWSON2, u, 1) == CGL_OK, "lawson2");
  expect(cgl_run(p, CGL_SPLIT4, u, 2, 1) == CGL_OK, "run split4");
  expect(cgl_run(p, CGL_LAWSON2, u, 2, 0) == CGL_OK, "run lawson2");
  expect(cgl_status(p) == CGL_OK, "status");
  std::printf("  steppers prec=%d flags=%u d=%d ok\n", precision, flags, d);
  cgl_destroy(p);
}

// The direct-to-LDS tile shapes (2: 64 x 16, 3: 128 x 16) against the
// register-staged ones with the same row count and 16-deep steps (0: 64 x 32,
// 1: 128 x 16): the same products in the same order, so Strang and Lawson4
// steps must agree bit for bit.
static void dma_tiles_bitwise(std::vector<int64_t> n, unsigned flags, cgl_coeffs c, double a,
                              double b, int bc) {
  const int d = static_cast<int>(n.size());
  int64_t N = 1;
  for (auto v : n) N *= v;
  const bool c128 = (flags & CGL_FLAG_FP64_MASTER) != 0;
  const size_t bytes = static_cast<size_t>(N) * (c128 ? 16 : 8);
  std::vector<std::vector<unsigned char>> res;
  for (const char* t : {"0", "2", "1", "3"}) {
    setenv("CGL_SPLIT_TILE", t, 1);
    cgl_plan_t p = nullptr;
    expect(cgl_plan(&p, d, n.data(), &c, 0.005, CGL_SPLIT_BF16, flags, nullptr) == CGL_OK, "plan");
    for (int mu = 0; mu < d; ++mu) {
      std::vector<cd> A(n[mu] * n[mu]);
      expect(cgl_fd_operator(n[mu], a, b, bc, &c, d, reinterpret_cast<double*>(A.data())) == CGL_OK,
             "fd");
      expect(cgl_set_operators(p, mu, reinterpret_cast<double*>(A.data())) == CGL_OK, "set");
    }
    auto U = rnd(N, 11, 0.3);
    std::vector<cd> u64 = U;
    std::vector<std::complex<float>> u32 = cast<float>(U);
    void* u = c128 ? static_cast<void*>(u64.data()) : static_cast<void*>(u32.data());
    expect(cgl_step_lawson4(p, u, 2) == CGL_OK, "lawson4");
    expect(cgl_step_strang(p, u, 1) == CGL_OK, "strang");
    expect(cgl_status(p) == CGL_OK, "status");
    const unsigned char* q = static_cast<const unsigned char*>(u);
    res.emplace_back(q, q + bytes);
    cgl_destroy(p);
  }
  expect(res[0] == res[1], "64-row tiles: direct-to-LDS == register staged");
  expect(res[2] == res[3], "128-row tiles: direct-to-LDS == register staged");
  std::printf("  dma tiles bitwise d=%d flags=%u ok\n", d, flags);
}

// Lawson4 with both actions of a round in one paired pass per direction
// (CGL_LAWSON_PAIRED=1) against the two concurrent actions: the same
// products and combinations, so the steps must agree bit for bit.
static void paired_bitwise(std::vector<int64_t> n, unsigned flags, cgl_coeffs c, double a,
                           double b, int bc) {
  const int d = static_cast<int>(n.size());
  int64_t N = 1;
  for (auto v : n) N *= v;
  const bool c128 = (flags & CGL_FLAG_FP64_MASTER) != 0;
  const size_t bytes = static_cast<size_t>(N) * (c128 ? 16 : 8);
  std::vector<std::vector<unsigned char>> res;
  for (const char* pv : {"0", "1"}) {
    setenv("CGL_LAWSON_PAIRED", pv, 1);
    cgl_plan_t p = nullptr;
    expect(cgl_plan(&p, d, n.data(), &c, 0.005, CGL_SPLIT_BF16, flags, nullptr) == CGL_OK, "plan");
    for (int mu = 0; mu < d; ++mu) {
      std::vector<cd> A(n[mu] * n[mu]);
      expect(cgl_fd_operator(n[mu], a, b, bc, &c, d, reinterpret_cast<double*>(A.data())) == CGL_OK,
             "fd");
      expect(cgl_set_operators(p, mu, reinterpret_cast<double*>(A.data())) == CGL_OK, "set");
    }
    auto U = rnd(N, 13, 0.3);
    std::vector<cd> u64 = U;
    std::vector<std::complex<float>> u32 = cast<float>(U);
    void* u = c128 ? static_cast<void*>(u64.data()) : static_cast<void*>(u32.data());
    expect(cgl_step_lawson4(p, u, 2) == CGL_OK, "lawson4");
    expect(cgl_run(p, CGL_LAWSON4, u, 2, 2) == CGL_OK, "run lawson4");
    expect(cgl_step(p, CGL_LAWSON2, u, 2) == CGL_OK, "lawson2");
    expect(cgl_status(p) == CGL_OK, "status");
    const unsigned char* q = static_cast<const unsigned char*>(u);
    res.emplace_back(q, q + bytes);
    cgl_destroy(p);
  }
  unsetenv("CGL_LAWSON_PAIRED");
  expect(res[0] == res[1], "paired Lawson4 / Lawson2b == two concurrent actions");
  std::printf("  paired lawson4 bitwise d=%d flags=%u ok\n", d, flags);
}

static void run_steps(std::vector<int64_t> n, int precision, unsigned flags, cgl_coeffs c,
                      double a, double b, int bc, double tau, int method, int m) {
  const int d = static_cast<int>(n.size());
  int64_t N = 1;
  for (auto v : n) N *= v;
  cgl_plan_t p = nullptr;
  expect(cgl_plan(&p, d, n.data(), &c, tau, precision, flags, nullptr) == CGL_OK, "plan");
  for (int mu = 0; mu < d; ++mu) {
    std::vector<cd> A(n[mu] * n[mu]);
    expect(cgl_fd_operator(n[mu], a, b, bc, &c, d, reinterpret_cast<double*>(A.data())) == CGL_OK,
           "fd");
    expect(cgl_set_operators(p, mu, reinterpret_cast<double*>(A.data())) == CGL_OK, "set_operators");
  }
  auto U = rnd(N, 11, 0.3);
  std::vector<std::complex<float>> u32 = cast<float>(U);
  const bool c128 = precision == CGL_FP64 || (flags & CGL_FLAG_FP64_MASTER);
  void* u = c128 ? static_cast<void*>(U.data()) : static_cast<void*>(u32.data());
  if (method == CGL_STRANG)
    expect(cgl_step_strang(p, u, m) == CGL_OK, "strang");
  else
    expect(cgl_step_lawson4(p, u, m) == CGL_OK, "lawson4");
  expect(cgl_status(p) == CGL_OK, "status");
  std::printf("  run_steps prec=%d d=%d method=%d m=%d ok\n", precision, d, method, m);
  cgl_destroy(p);
}

// Batched plan vs one plain plan per instance with the same exponentials:
// the same kernels run on the same data, so the states must agree bitwise.
static void batched_vs_single(int precision,
                              const std::vector<std::vector<int64_t>>& grids = {
                                  {32, 48}, {20, 33}, {64, 32}, {9, 7}}) {
  const int B = static_cast<int>(grids.size()), d = 2;
  std::vector<int64_t> flat;
  std::vector<cgl_coeffs> cs;
  for (int j = 0; j < B; ++j) {
    flat.insert(flat.end(), grids[j].begin(), grids[j].end());
    cs.push_back(cgl_coeffs{1.0 + 0.2 * j, -0.5 + 0.3 * j, 0.1 * j, -1.0 - 0.1 * j, 0.5 + 0.2 * j, 0, 0});
  }
  cgl_plan_t bp = nullptr;
  expect(cgl_plan_batched(&bp, B, d, flat.data(), cs.data(), 0.01, precision, 0, nullptr) == CGL_OK,
         "plan_batched");
  std::vector<std::vector<cd>> As;
  std::vector<const double*> ptrs;
  for (int j = 0; j < B; ++j)
    for (int mu = 0; mu < d; ++mu) {
      As.emplace_back(grids[j][mu] * grids[j][mu]);
      expect(cgl_fd_operator(grids[j][mu], -10, 10, CGL_DIRICHLET, &cs[j], d,
                             reinterpret_cast<double*>(As.back().data())) == CGL_OK, "fd");
    }
  for (auto& A : As) ptrs.push_back(reinterpret_cast<const double*>(A.data()));
  expect(cgl_set_operators_all(bp, ptrs.data()) == CGL_OK, "set_operators_all");
  int64_t N = 0;
  std::vector<int64_t> offs(B);
  for (int j = 0; j < B; ++j) {
    expect(cgl_instance_offset(bp, j, &offs[j]) == CGL_OK, "offset");
    N += grids[j][0] * grids[j][1];
  }
  auto U = rnd(N, 21, 0.4);
  std::vector<cd> u64 = U;
  std::vector<std::complex<float>> u32 = cast<float>(U);
  const bool c128 = precision == CGL_FP64;
  void* u = c128 ? static_cast<void*>(u64.data()) : static_cast<void*>(u32.data());
  expect(cgl_step_lawson4(bp, u, 2) == CGL_OK, "batched lawson4");
  expect(cgl_run(bp, CGL_STRANG, u, 2, 1) == CGL_OK, "batched run strang");
  expect(cgl_step(bp, CGL_SPLIT4, u, 1) == CGL_OK, "batched split4");
  expect(cgl_step(bp, CGL_LAWSON2, u, 1) == CGL_OK, "batched lawson2");
  expect(cgl_status(bp) == CGL_OK, "batched status");
  int mism = 0;
  for (int j = 0; j < B; ++j) {
    cgl_plan_t sp = nullptr;
    expect(cgl_plan(&sp, d, grids[j].data(), &cs[j], 0.01, precision, 0, nullptr) == CGL_OK, "plan");
    for (int mu = 0; mu < d; ++mu) {
      std::vector<cd> E(grids[j][mu] * grids[j][mu]), H(E.size());
      expect(cgl_get_instance_operator(bp, j, mu, CGL_E, reinterpret_cast<double*>(E.data())) ==
                 CGL_OK, "get E");
      expect(cgl_get_instance_operator(bp, j, mu, CGL_H, reinterpret_cast<double*>(H.data())) ==
                 CGL_OK, "get H");
      expect(cgl_set_exponentials(sp, mu, reinterpret_cast<double*>(E.data()),
                                  reinterpret_cast<double*>(H.data())) == CGL_OK, "set exps");
    }
    const int64_t Nj = grids[j][0] * grids[j][1];
    std::vector<cd> v64(U.begin() + offs[j], U.begin() + offs[j] + Nj);
    std::vector<std::complex<float>> v32 = cast<float>(v64);
    void* v = c128 ? static_cast<void*>(v64.data()) : static_cast<void*>(v32.data());
    expect(cgl_step_lawson4(sp, v, 2) == CGL_OK, "single lawson4");
    expect(cgl_run(sp, CGL_STRANG, v, 2, 1) == CGL_OK, "single run strang");
    expect(cgl_step(sp, CGL_SPLIT4, v, 1) == CGL_OK, "single split4");
    expect(cgl_step(sp, CGL_LAWSON2, v, 1) == CGL_OK, "single lawson2");
    for (int64_t i = 0; i < Nj; ++i) {
      const bool same = c128 ? (v64[i] == u64[offs[j] + i]) : (v32[i] == u32[offs[j] + i]);
      if (!same) ++mism;
    }
    cgl_destroy(sp);
  }
  std::printf("  batched vs single prec=%d mismatches=%d\n", precision, mism);
  expect(mism == 0, "batched == single");
  cgl_destroy(bp);
}

template <class T>
static std::vector<T> read_file(const std::string& path, size_t n) {
  std::vector<T> v(n);
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f || std::fread(v.data(), sizeof(T), n, f) != n) {
    std::printf("FAIL: cannot read %s\n", path.c_str());
    std::exit(2);
  }
  std::fclose(f);
  return v;
}

template <class T>
static void write_file(const std::string& path, const std::vector<T>& v) {
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f || std::fwrite(v.data(), sizeof(T), v.size(), f) != v.size()) {
    std::printf("FAIL: cannot write %s\n", path.c_str());
    std::exit(2);
  }
  std::fclose(f);
}

// Surrogate entry points on inputs written by the test (dir/params.f32,
// dir/src.c64 with 2S samples: inputs then targets, dir/cstd.f32 [2S][5]);
// writes the forward result, the gradient, the loss and the parameters
// after one Adam step, for comparison with the oracle.  Then checks that a
// gated run whose checks fail reproduces the plain stepper exactly.
static void surrogate(const std::string& dir, int64_t n1, int64_t n2, int S, float lr) {
  const int64_t P = n1 * n2;
  int64_t count = 0;
  expect(cgl_sur_param_count(&count) == CGL_OK && count == 87074, "param count");
  auto params = read_file<float>(dir + "/params.f32", count);
  auto src = read_file<std::complex<float>>(dir + "/src.c64", 2 * S * P);
  auto cstd = read_file<float>(dir + "/cstd.f32", 2 * S * 5);
  cgl_sur_t s = nullptr;
  expect(cgl_sur_create(&s, n1, n2, S, nullptr) == CGL_OK, "sur create");
  std::vector<std::complex<float>> out(S * P);
  expect(cgl_sur_forward(s, S, src.data(), cstd.data(), nullptr, out.data()) == CGL_ENOTREADY,
         "not ready");
  expect(cgl_sur_set_params(s, params.data()) == CGL_OK, "set params");
  expect(cgl_sur_forward(s, S, src.data(), cstd.data(), nullptr, out.data()) == CGL_OK, "forward");
  write_file(dir + "/fwd.c64", out);
  // an explicit base equal to the input gives the same bits; a base shifted
  // by a constant shifts the output by it (up to FP32 rounding)
  std::vector<std::complex<float>> outb(S * P), based(src.begin(), src.begin() + S * P);
  expect(cgl_sur_forward(s, S, src.data(), cstd.data(), based.data(), outb.data()) == CGL_OK,
         "forward base");
  expect(std::memcmp(out.data(), outb.data(), out.size() * sizeof(out[0])) == 0, "base = input");
  const std::complex<float> shift(0.25f, -0.5f);
  for (auto& v : based) v += shift;
  expect(cgl_sur_forward(s, S, src.data(), cstd.data(), based.data(), outb.data()) == CGL_OK,
         "forward shifted base");
  double worst = 0.0;
  for (int64_t i = 0; i < S * P; ++i)
    worst = std::max(worst, static_cast<double>(std::abs(outb[i] - out[i] - shift)));
  expect(worst < 1e-5, "shifted base");
  // the output scale multiplies the correction
  expect(cgl_sur_set_output_scale(s, 0.0f) == CGL_EINVAL && cgl_sur_set_output_scale(s, NAN) ==
                                                                  CGL_EINVAL,
         "bad output scale");
  expect(cgl_sur_set_output_scale(s, 0.5f) == CGL_OK, "output scale");
  expect(cgl_sur_forward(s, S, src.data(), cstd.data(), nullptr, outb.data()) == CGL_OK,
         "forward scaled");
  worst = 0.0;
  for (int64_t i = 0; i < S * P; ++i)
    worst = std::max(worst, static_cast<double>(std::abs((outb[i] - src[i]) -
                                                         0.5f * (out[i] - src[i]))));
  expect(worst < 1e-5, "scaled correction");
  expect(cgl_sur_set_output_scale(s, 1.0f) == CGL_OK, "unit output scale");
  std::vector<float> grad(count);
  double loss = 0.0;
  expect(cgl_sur_grad(s, S, src.data(), cstd.data(), nullptr, S, nullptr, grad.data(), &loss) ==
             CGL_OK,
         "grad");
  write_file(dir + "/grad.f32", grad);
  write_file(dir + "/loss.f64", std::vector<double>{loss});
  expect(cgl_sur_train_step(s, S, src.data(), cstd.data(), nullptr, S, nullptr, lr) == CGL_OK,
         "train");
  double mean = 0.0;
  expect(cgl_sur_take_loss(s, &mean) == CGL_OK && std::fabs(mean - loss) <= 1e-6 * loss,
         "take loss");
  std::vector<float> after(count);
  expect(cgl_sur_get_params(s, after.data()) == CGL_OK, "get params");
  write_file(dir + "/params_after.f32", after);
  // an index array: sample 1 then 0
  std::vector<int32_t> idx = {1, 0};
  if (S >= 2) {
    std::vector<float> g2(count);
    double l2 = 0.0;
    expect(cgl_sur_set_params(s, params.data()) == CGL_OK, "reset params");
    expect(cgl_sur_grad(s, 2, src.data(), cstd.data(), idx.data(), S, nullptr, g2.data(), &l2) ==
               CGL_OK,
           "grad idx");
    double num = 0, den = 0;
    for (int64_t i = 0; i < count; ++i) {
      num += (g2[i] - grad[i]) * (g2[i] - grad[i]);
      den += grad[i] * grad[i];
    }
    // the same two pairs in the other order: equal up to summation order
    expect(std::sqrt(num / den) < 1e-5 && std::fabs(l2 - loss) < 1e-9 * loss, "idx permutation");
    // the base indexed like the source: the input itself as an explicit base
    std::vector<float> g3(count);
    double l3 = 0.0;
    expect(cgl_sur_grad(s, 2, src.data(), cstd.data(), idx.data(), S, src.data(), g3.data(), &l3) ==
               CGL_OK,
           "grad base");
    expect(std::memcmp(g2.data(), g3.data(), count * sizeof(float)) == 0 && l2 == l3,
           "grad base = input");
  }

  // gated run with checks that fail: equals the plain stepper bit for bit
  cgl_coeffs c{1.0, 0.5, 0.2, -1.0, 1.0, 0.0, 0.0};
  const int64_t n[2] = {n1, n2};
  cgl_plan_t p = nullptr;
  expect(cgl_plan(&p, 2, n, &c, 0.01, CGL_SPLIT_BF16, 0, nullptr) == CGL_OK, "plan");
  for (int mu = 0; mu < 2; ++mu) {
    std::vector<double> A(2 * n[mu] * n[mu]);
    expect(cgl_fd_operator(n[mu], -10, 10, CGL_DIRICHLET, &c, 2, A.data()) == CGL_OK, "fd");
    expect(cgl_set_operators(p, mu, A.data()) == CGL_OK, "ops");
  }
  std::vector<std::complex<float>> ua(src.begin(), src.begin() + P), ub = ua;
  const double cs[5] = {0.1, -0.2, 0.3, 0.0, 0.5};
  int64_t stats[4] = {};
  std::vector<float> bad(count, 0.0f);
  bad[count - 2] = 50.0f;  // output bias: a jump far from the stepper
  bad[count - 1] = 50.0f;
  expect(cgl_sur_set_params(s, bad.data()) == CGL_OK, "bad params");
  // 3 jumps of 1 step, checks at jumps 2 and 3: check 1, redo 2, check 1, redo 1
  const int gst = cgl_run_surrogate(p, s, ua.data(), cs, 3, 1, 2, 1e-3, nullptr,
                                    CGL_SUR_BASE_INPUT, stats);
  if (gst != CGL_OK) std::printf("gated run status %d\n", gst);
  expect(gst == CGL_OK, "gated run");
  expect(stats[0] == 0 && stats[1] == 3 && stats[2] == 2 && stats[3] == 1 + 2 + 1 + 1,
         "gated stats");
  expect(cgl_run(p, CGL_LAWSON4, ub.data(), 3, 0) == CGL_OK, "plain run");
  expect(std::memcmp(ua.data(), ub.data(), ua.size() * sizeof(ua[0])) == 0, "rollback exact");
  double rs[5] = {0, 0, 0, 0, 0};
  expect(cgl_run_surrogate(p, s, ua.data(), rs, 1, 0, 1, 1e-3, nullptr, CGL_SUR_BASE_INPUT,
                           stats) == CGL_EINVAL,
         "bad M");
  expect(cgl_run_surrogate(p, s, ua.data(), rs, 1, 1, 1, 1e-3, nullptr, CGL_SUR_BASE_LINEAR,
                           stats) == CGL_EINVAL,
         "base without a coarse plan");
  // a zero network about the linear base, with a loose tolerance: every jump
  // is the coarse plan's exponential, and the checked spans continue from
  // the plain result
  cgl_plan_t q = nullptr;
  expect(cgl_plan(&q, 2, n, &c, 0.02, CGL_SPLIT_BF16, 0, nullptr) == CGL_OK, "coarse plan");
  for (int mu = 0; mu < 2; ++mu) {
    std::vector<double> A(2 * n[mu] * n[mu]);
    expect(cgl_fd_operator(n[mu], -10, 10, CGL_DIRICHLET, &c, 2, A.data()) == CGL_OK, "fd");
    expect(cgl_set_operators(q, mu, A.data()) == CGL_OK, "coarse ops");
  }
  expect(cgl_sur_set_params(s, std::vector<float>(count, 0.0f).data()) == CGL_OK, "zero params");
  std::vector<std::complex<float>> uc(src.begin(), src.begin() + P), ud = uc, ue(P);
  expect(cgl_run_surrogate(p, s, uc.data(), cs, 1, 2, 2, 1e3, q, CGL_SUR_BASE_LINEAR, stats) ==
             CGL_OK,
         "gated linear");
  expect(stats[0] == 1 && stats[2] == 1, "linear accepted");
  expect(cgl_run(p, CGL_LAWSON4, ud.data(), 2, 0) == CGL_OK, "plain 2");
  expect(std::memcmp(uc.data(), ud.data(), uc.size() * sizeof(uc[0])) == 0, "continues plain");
  // two jumps, only the last checked (and accepted): the first jump's result
  // is the coarse exponential of u (a zero network adds nothing), the
  // second continues from the plain stepper's span after it
  for (int base : {CGL_SUR_BASE_LINEAR, CGL_SUR_BASE_STRANG}) {
    uc.assign(src.begin(), src.begin() + P);
    ue = uc;
    if (base == CGL_SUR_BASE_LINEAR) {
      expect(cgl_tucker(q, CGL_E, uc.data(), ue.data()) == CGL_OK, "coarse tucker");
    } else {
      expect(cgl_step(q, CGL_STRANG, ue.data(), 1) == CGL_OK, "coarse strang");
    }
    expect(cgl_run(p, CGL_LAWSON4, ue.data(), 2, 0) == CGL_OK, "plain after base");
    expect(cgl_run_surrogate(p, s, uc.data(), cs, 2, 2, 5, 1e3, q, base, stats) == CGL_OK,
           "gated two jumps");
    expect(stats[0] == 2 && stats[2] == 1, "two accepted");
    expect(std::memcmp(uc.data(), ue.data(), uc.size() * sizeof(uc[0])) == 0, "base jump exact");
  }
  expect(cgl_run_surrogate(p, s, uc.data(), cs, 1, 2, 1, 1e3, q, 3, stats) == CGL_EINVAL,
         "bad base");
  cgl_destroy(q);
  cgl_destroy(p);
  cgl_sur_destroy(s);
}

int main(int argc, char** argv) {
  if (argc > 1 && std::string(argv[1]) == "gpu-sequence") {
    // the GPU FP64 test file's order: mode products, Tuckers, C0 Strang, C0 Lawson4
    const std::vector<std::vector<int64_t>> shapes = {{150}, {64, 45}, {130, 70},
                                                      {20, 33, 17}, {64, 64, 40}, {3, 5, 4}};
    unsigned seed = 100;
    for (auto& s : shapes) kernel_parity(s, CGL_FP64, seed++);
    cgl_coeffs c0{1.0, 1.5, 0.5, -1.0, 1.0, 0.0, 0.0};
    run_steps({64, 64}, CGL_FP64, 0, c0, -10, 10, CGL_DIRICHLET, 0.01, CGL_STRANG, 100);
    run_steps({64, 64}, CGL_FP64, 0, c0, -10, 10, CGL_DIRICHLET, 0.01, CGL_LAWSON4, 50);
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "PASSED", failures);
    return failures ? 1 : 0;
  }
  if (argc > 1 && std::string(argv[1]) == "smoke") {
    // one case of every kernel family (the default of the CPU suite; the
    // quick, split and fft modes are the full sweep)
    const cgl_coeffs cub{1.0, 1.5, 0.5, -1.0, 1.0, 0.0, 0.0};
    const cgl_coeffs cq{1.0, 0.8, -0.1, 1.2, 1.0, -0.1, -0.5};
    auto t0 = std::chrono::steady_clock::now();
    auto lap = [&](const char* what) {
      const auto t1 = std::chrono::steady_clock::now();
      std::printf("  [%s: %.1f s]\n", what, std::chrono::duration<double>(t1 - t0).count());
      std::fflush(stdout);
      t0 = t1;
    };
    for (int prec : {CGL_FP64, CGL_SPLIT_BF16}) kernel_parity({20, 9, 7}, prec, 3);
    lap("kernel parity");
    steppers({12, 10, 6}, CGL_FP64, 0, cq, -15, 15, CGL_NEUMANN);
    lap("fp64 steppers");
    steppers({16, 12}, CGL_SPLIT_BF16, 0, cub, -10, 10, CGL_DIRICHLET);
    lap("split steppers");
    steppers({7, 6, 5}, CGL_SPLIT_BF16, CGL_FLAG_FP64_MASTER, cq, -15, 15, CGL_NEUMANN);
    lap("master steppers");
    paired_bitwise({7, 6, 5}, 0, cq, -15, 15, CGL_NEUMANN);
    lap("paired 64");
    setenv("CGL_PAIR_TILE", "3", 1);
    paired_bitwise({7, 6, 5}, CGL_FLAG_FP64_MASTER, cq, -15, 15, CGL_NEUMANN);
    unsetenv("CGL_PAIR_TILE");
    lap("paired 128");
    batched_vs_single(CGL_SPLIT_BF16, {{16, 24}, {9, 7}});
    lap("batched");
    fourier_parity({16, 8, 32}, CGL_SPLIT_BF16, 21);
    lap("fourier");
    coupled({16, 8}, CGL_FP64, 28);
    lap("coupled");
    coupled_ksplit({144, 6}, 32, false);
    lap("split contraction");
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "PASSED", failures);
    return failures ? 1 : 0;
  }
  if (argc > 1 && std::string(argv[1]) == "fft") {
    // the Fourier pass alone: every transform length's staging shape, both
    // precisions, a complex128 state entering a complex64 plan
    for (int prec : {CGL_FP64, CGL_SPLIT_BF16}) {
      fourier_parity({16, 8, 32}, prec, 21);
      fourier_parity({128, 4}, prec, 24);
      fourier_parity({256, 4}, prec, 25);
      fourier_parity({512, 3}, prec, 30);    // fewer than 16 fibres per workgroup:
      fourier_parity({1024, 3}, prec, 31);   // padded rows, spread fibres
    }
    fourier_parity({32, 16}, CGL_SPLIT_BF16, 26, CGL_FLAG_FP64_MASTER);
    fourier_parity({64, 12}, CGL_SPLIT_BF16, 27, CGL_FLAG_FP64_MASTER);
    for (int prec : {CGL_FP64, CGL_SPLIT_BF16}) {
      coupled({16, 8}, prec, 28);   // Fourier passes
      coupled({12, 6}, prec, 29);   // dense circulant exponentials
    }
    coupled_ksplit({144, 6}, 32);   // 9 stages: 2 splits of 5 and 4
    coupled_ksplit({208, 6}, 33);   // 13 stages: 3 splits of 5, 5 and 3
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "PASSED", failures);
    return failures ? 1 : 0;
  }
  if (argc > 1 && std::string(argv[1]) == "sur") {
    if (argc < 7) return 2;
    surrogate(argv[2], std::atoll(argv[3]), std::atoll(argv[4]), std::atoi(argv[5]),
              static_cast<float>(std::atof(argv[6])));
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "PASSED", failures);
    return failures ? 1 : 0;
  }
  cgl_coeffs cub{1.0, 1.5, 0.5, -1.0, 1.0, 0.0, 0.0};
  cgl_coeffs cq{1.0, 0.8, -0.1, 1.2, 1.0, -0.1, -0.5};
  if (argc > 1 && std::string(argv[1]) == "full") {
    for (int prec : {CGL_FP64, CGL_SPLIT_BF16}) {
      kernel_parity({150}, prec, 1);
      kernel_parity({64, 45}, prec, 2);
      kernel_parity({20, 33, 17}, prec, 3);
      kernel_parity({3, 5, 4}, prec, 4);
      kernel_parity({130, 7}, prec, 5);
    }
    steppers({64, 64}, CGL_FP64, 0, cub, -10, 10, CGL_DIRICHLET);
    steppers({12, 10, 14}, CGL_FP64, 0, cq, -15, 15, CGL_NEUMANN);
    steppers({37}, CGL_FP64, 0, cub, -10, 10, CGL_DIRICHLET);
    steppers({64, 64}, CGL_SPLIT_BF16, 0, cub, -10, 10, CGL_DIRICHLET);
    steppers({12, 10, 14}, CGL_SPLIT_BF16, 0, cq, -15, 15, CGL_NEUMANN);
    steppers({12, 10, 14}, CGL_SPLIT_BF16, CGL_FLAG_FP64_MASTER, cq, -15, 15, CGL_NEUMANN);
    steppers({37}, CGL_SPLIT_BF16, CGL_FLAG_FP64_MASTER, cub, -10, 10, CGL_DIRICHLET);
  } else if (argc > 1 && std::string(argv[1]) == "split") {
    batched_vs_single(CGL_SPLIT_BF16);
    kernel_parity({20, 9, 7}, CGL_SPLIT_BF16, 3);
    kernel_parity({32, 64, 3}, CGL_SPLIT_BF16, 6);
    steppers({32, 64}, CGL_SPLIT_BF16, 0, cub, -10, 10, CGL_DIRICHLET);
    steppers({7, 6, 5}, CGL_SPLIT_BF16, CGL_FLAG_FP64_MASTER, cq, -15, 15, CGL_NEUMANN);
    const char* keep = std::getenv("CGL_SPLIT_TILE");
    const std::string saved = keep ? keep : "";
    dma_tiles_bitwise({32, 64}, 0, cub, -10, 10, CGL_DIRICHLET);     // full tiles
    dma_tiles_bitwise({20, 9, 7}, 0, cq, -15, 15, CGL_NEUMANN);      // ragged: n % 16, F % 64
    dma_tiles_bitwise({37}, CGL_FLAG_FP64_MASTER, cub, -10, 10, CGL_DIRICHLET);
    dma_tiles_bitwise({7, 6, 5}, CGL_FLAG_FP64_MASTER, cq, -15, 15, CGL_NEUMANN);
    paired_bitwise({32, 64}, 0, cub, -10, 10, CGL_DIRICHLET);
    paired_bitwise({20, 9, 7}, 0, cq, -15, 15, CGL_NEUMANN);
    paired_bitwise({37}, CGL_FLAG_FP64_MASTER, cub, -10, 10, CGL_DIRICHLET);
    paired_bitwise({7, 6, 5}, CGL_FLAG_FP64_MASTER, cq, -15, 15, CGL_NEUMANN);
    for (const char* t : {"2", "3"}) {  // the batched pass on the direct-to-LDS shapes
      setenv("CGL_SPLIT_TILE", t, 1);
      batched_vs_single(CGL_SPLIT_BF16);
    }
    // the 128-row paired pass (8 waves) against the two-action form and in
    // the batched persistent pass
    setenv("CGL_PAIR_TILE", "3", 1);
    paired_bitwise({20, 9, 7}, 0, cq, -15, 15, CGL_NEUMANN);
    paired_bitwise({7, 6, 5}, CGL_FLAG_FP64_MASTER, cq, -15, 15, CGL_NEUMANN);
    batched_vs_single(CGL_SPLIT_BF16);
    unsetenv("CGL_PAIR_TILE");
    if (keep) setenv("CGL_SPLIT_TILE", saved.c_str(), 1); else unsetenv("CGL_SPLIT_TILE");
  } else {
    // quick: every kernel variant (mu = 1 contiguous, mu > 1 strided, ragged
    // tiles, both precisions) and every stepper path, on small grids
    for (int prec : {CGL_FP64, CGL_SPLIT_BF16}) {
      kernel_parity({37}, prec, 1);
      kernel_parity({20, 9, 7}, prec, 3);
      kernel_parity({3, 5, 4}, prec, 4);
      kernel_parity({32, 64, 3}, prec, 6);  // full tiles: unmasked fast path
    }
    steppers({12, 10, 6}, CGL_FP64, 0, cq, -15, 15, CGL_NEUMANN);
    steppers({9}, CGL_FP64, 0, cub, -10, 10, CGL_DIRICHLET);
    steppers({16, 12}, CGL_SPLIT_BF16, 0, cub, -10, 10, CGL_DIRICHLET);
    steppers({32, 64}, CGL_SPLIT_BF16, 0, cub, -10, 10, CGL_DIRICHLET);
    steppers({64, 32}, CGL_SPLIT_BF16, CGL_FLAG_FP64_MASTER, cub, -10, 10, CGL_DIRICHLET);
    steppers({7, 6, 5}, CGL_SPLIT_BF16, CGL_FLAG_FP64_MASTER, cq, -15, 15, CGL_NEUMANN);
    steppers({9}, CGL_SPLIT_BF16, CGL_FLAG_FP64_MASTER, cub, -10, 10, CGL_DIRICHLET);
    steppers({12, 10, 6}, CGL_FP64, CGL_FLAG_THREE_TERM, cq, -15, 15, CGL_NEUMANN);
    for (int prec : {CGL_FP64, CGL_SPLIT_BF16}) {
      fourier_parity({16, 8, 32}, prec, 21);   // every direction a Fourier pass (strided in FP64)
      fourier_parity({64, 12}, prec, 22);      // n = 12: the dense circulant on MFMA
      fourier_parity({8}, prec, 23);
    }
    steppers({16, 12}, CGL_SPLIT_BF16, CGL_FLAG_THREE_TERM, cq, -10, 10, CGL_DIRICHLET);
    batched_vs_single(CGL_FP64);
    batched_vs_single(CGL_SPLIT_BF16);
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "PASSED", failures);
  return failures ? 1 : 0;
}
