#include "split_layout.hpp"

namespace cgl {

void build_split_operator(const CMat& M, const SplitTile& tile, std::vector<uint16_t>& out,
                          int& Pp, int& Kp) {
  const int PT = tile.PT, KS = tile.KS;  // KS == 16 when tile.dma
  const int64_t n = M.n;
  Pp = static_cast<int>((n + PT - 1) / PT * PT);
  Kp = static_cast<int>((n + KS - 1) / KS * KS);
  const int nPT = Pp / PT, nKS = Kp / KS;
  const size_t block = static_cast<size_t>(SPK_Q) * PT * KS;
  out.assign(block * nPT * nKS, 0);
  for (int64_t k = 0; k < n; ++k) {
    for (int64_t m = 0; m < n; ++m) {
      uint16_t tr[3], ti[3];
      split_bf16(M.re[m + n * k], 3, tr);
      split_bf16(M.im[m + n * k], 3, ti);
      const int pt = static_cast<int>(m / PT), row = static_cast<int>(m % PT);
      const int ks = static_cast<int>(k / KS), kk = static_cast<int>(k % KS);
      uint16_t* b = out.data() + (static_cast<size_t>(pt) * nKS + ks) * block;
      // within a plane: 16-byte chunk (kk / 8, row) at chunk index (kk / 8) * PT + row,
      // or, for the LDS-image layout, row * KS / 8 + (kk / 8 swizzled by row)
      const size_t c = tile.dma ? static_cast<size_t>(row) * (KS / 8) + dma_chunk(row, kk / 8)
                                : static_cast<size_t>(kk / 8) * PT + row;
      for (int t = 0; t < 3; ++t) {
        b[(static_cast<size_t>(t) * PT * KS) + c * 8 + kk % 8] = tr[t];
        b[(static_cast<size_t>(3 + t) * PT * KS) + c * 8 + kk % 8] = ti[t];
      }
    }
  }
}

}  // namespace cgl
