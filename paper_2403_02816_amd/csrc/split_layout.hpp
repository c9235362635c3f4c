// Device layout of the bf16 term planes of one complex exponential M (n x n)
// for the split-precision mu-mode kernel.
//
// The complex product y = M x is evaluated as four real products
//   Re y = Re M Re x - Im M Im x,   Im y = Im M Re x + Re M Im x,
// each operand given as a sum of three bf16 terms.  Layout, in bf16 units:
//   [p-tile pt < Pp/PT][k-stage ks < Kp/KS][plane q < 6][k/8 < KS/8][row < PT][k%8 < 8]
// with planes q = 0,1,2: terms of Re M; q = 3,4,5: terms of Im M, row = output
// index m (within the p-tile), k = contraction index j (within the stage);
// entries beyond n are zero.  One (pt, ks) block is contiguous, so a
// workgroup copies one stage of its p-tile with plain 16-byte loads, and
// consecutive 16-byte chunks belong to consecutive rows (consecutive lanes
// write distinct LDS banks).
#pragma once

#include <cstdint>
#include <vector>

#include "host_numerics.hpp"

namespace cgl {

constexpr int SPK_Q = 6;  // planes per stage block

// Tile shapes of the split kernel: (rows per workgroup, stage depth, layout).
// dma = 0: the chunk layout above, staged through registers; dma = 1 (KS =
// 16 only): each (pt, ks) block is the image of its LDS tile (planes of PT
// rows x 16, rows unpadded, 16-byte chunk c of row r at position
// dma_chunk(r, c)), copied by direct-to-LDS loads (contiguous contraction
// axis only).
struct SplitTile {
  int PT, KS, dma;
};
constexpr SplitTile SPLIT_TILES[4] = {{64, 32, 0}, {128, 16, 0}, {64, 16, 1}, {128, 16, 1}};
constexpr int SPLIT_NTILES = 4;

// Position of 16-byte chunk c (0 or 1) of row r in a 32-byte row of the
// direct-to-LDS layout.  Rows r and r + 4 (128 bytes apart) and rows r and
// r + 8 (256 bytes apart) take opposite positions, so the 16-byte reads of 8
// or 16 consecutive lanes (consecutive rows, one chunk) hit distinct banks.
constexpr int dma_chunk(int r, int c) { return c ^ (((r >> 2) ^ (r >> 3)) & 1); }
constexpr int SPLIT_NTILES_BATCHED = SPLIT_NTILES;  // every shape has a batched form

// Builds the planes of M (3 bf16 terms of Re and Im of every entry) for tile
// shape t; Pp, Kp receive the padded row / contraction counts.
void build_split_operator(const CMat& M, const SplitTile& t, std::vector<uint16_t>& out, int& Pp,
                          int& Kp);

}  // namespace cgl
