// Runs libcgl's host code and kernels on the CPU through the HIP emulation
// in this directory (built with AddressSanitizer by test_cpu_emulation.py).
// Checks every entry point for out-of-bounds accesses and checks the mode
// products / Tucker operator against a naive triple loop.
#include <complex>
#include <cstdio>
#include <cstdlib>
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
  cgl_destroy(p);
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
  expect(cgl_status(p) == CGL_OK, "status");
  std::printf("  steppers prec=%d flags=%u d=%d ok\n", precision, flags, d);
  cgl_destroy(p);
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
static void batched_vs_single(int precision) {
  const std::vector<std::vector<int64_t>> grids = {{32, 48}, {20, 33}, {64, 32}, {9, 7}};
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
    batched_vs_single(CGL_FP64);
    batched_vs_single(CGL_SPLIT_BF16);
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "PASSED", failures);
  return failures ? 1 : 0;
}
