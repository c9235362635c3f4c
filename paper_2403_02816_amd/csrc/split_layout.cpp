#include "split_layout.hpp"

namespace cgl {

void build_split_operator(const CMat& M, std::vector<uint16_t>& out, int& Pp, int& Kp) {
  const int64_t n = M.n;
  Pp = static_cast<int>((n + SPK_P - 1) / SPK_P * SPK_P);
  Kp = static_cast<int>((n + SPK_K - 1) / SPK_K * SPK_K);
  const int nPT = Pp / SPK_P, nKS = Kp / SPK_K;
  const size_t block = static_cast<size_t>(SPK_Q) * SPK_P * SPK_K;
  out.assign(block * nPT * nKS, 0);
  for (int64_t k = 0; k < n; ++k) {
    for (int64_t m = 0; m < n; ++m) {
      uint16_t tr[3], ti[3];
      split_bf16(M.re[m + n * k], 3, tr);
      split_bf16(M.im[m + n * k], 3, ti);
      const int pt = static_cast<int>(m / SPK_P), row = static_cast<int>(m % SPK_P);
      const int ks = static_cast<int>(k / SPK_K), kk = static_cast<int>(k % SPK_K);
      uint16_t* b = out.data() + (static_cast<size_t>(pt) * nKS + ks) * block;
      for (int t = 0; t < 3; ++t) {
        b[(static_cast<size_t>(t) * SPK_P + row) * SPK_K + kk] = tr[t];
        b[(static_cast<size_t>(3 + t) * SPK_P + row) * SPK_K + kk] = ti[t];
      }
    }
  }
}

}  // namespace cgl
