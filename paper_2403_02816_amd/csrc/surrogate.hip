// Residual CNN surrogate: 3x3 convolutions on CDNA4 BF16 MFMA
// (v_mfma_f32_16x16x32_bf16), their weight gradients, the MSE loss, Adam and
// the packing kernels.
//
// MFMA 16x16x32 bf16 lane layout (lane l, g = l / 16): A[l % 16][8g + e],
// B[8g + e][l % 16] for e = 0..7, accumulator register r holds
// D[4g + r][l % 16].
//
// Convolution (implicit GEMM): out[co][p] = sum_k W[co][k] X[k][p] with
// k = tap * CIN_PAD + ci, tap = 3 ky + kx, X[k][p] = x[ci][p shifted by
// (ky - 1, kx - 1)].  A workgroup keeps the layer's bf16 weights in LDS and
// loops over output tiles of TR rows x TW columns; a tile's input halo is
// staged channels-last (8 consecutive k of one tap are 16 contiguous bytes).
//
// Weight gradient: dW[co][(tap, ci)] = sum_p dout[co][p] X[(tap, ci)][p], a GEMM
// whose contraction runs over pixels.  The shifted operand is built in
// registers from aligned LDS reads (two bf16 of a dword shifted by 16 bits),
// and a constant-one column yields the bias gradient.  Each workgroup writes
// its partial sums; a reduction kernel adds them in FP64.
#include "surrogate.hpp"

namespace cgl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;  // threads per workgroup (4 waves)
constexpr int TW = 64;   // tile width (pixels along i1)
constexpr int TR = 2;    // tile height (rows along i2)

constexpr int kpad_of(int cin_pad) { return (9 * cin_pad + 31) / 32 * 32; }

// two FP32 values as packed bf16 (round to nearest even), a in the low half
__device__ __forceinline__ unsigned pack_bf16(float a, float b) {
  const f32x2 v = {a, b};
  const bf16x2 h = __builtin_convertvector(v, bf16x2);
  return __builtin_bit_cast(unsigned, h);
}

__device__ __forceinline__ float sigmoid_f(float a) { return 1.0f / (1.0f + expf(-a)); }

template <int CIN_PAD, int COUT_PAD, int EPI>
__global__ __launch_bounds__(NT) void k_conv(ConvArgs a, int ntiles) {
  constexpr int KP = kpad_of(CIN_PAD);
  constexpr int KSTEPS = KP / 32;
  constexpr int WS = KP + 8;                            // weight row pitch (bf16)
  constexpr int XS = CIN_PAD == 8 ? 8 : CIN_PAD + 8;    // halo position pitch (bf16)
  constexpr int XPOS = TW + 2, XROWS = TR + 2;
  constexpr int ZSLOT = XROWS * XPOS * XS;              // 8 zero bf16 for padded k
  constexpr int MB = COUT_PAD / 16;
  constexpr int NG = CIN_PAD / 8;
  static_assert(CIN_PAD % 8 == 0 && COUT_PAD % 16 == 0, "padding");
  __shared__ __attribute__((aligned(16))) uint16_t sW[COUT_PAD * WS];
  __shared__ __attribute__((aligned(16))) uint16_t sX[ZSLOT + 8];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, lc = lane & 15;
  for (int i = tid; i < COUT_PAD * (KP / 8); i += NT) {
    const int r = i / (KP / 8), c = i % (KP / 8);
    *reinterpret_cast<u32x4*>(&sW[r * WS + c * 8]) =
        *reinterpret_cast<const u32x4*>(a.w + static_cast<size_t>(r) * KP + c * 8);
  }
  if (tid < 4) reinterpret_cast<unsigned*>(&sX[ZSLOT])[tid] = 0u;

  const int n1 = a.n1, n2 = a.n2;
  const int64_t P = static_cast<int64_t>(n1) * n2;
  const int ncb = n1 / TW, nrb = (n2 + TR - 1) / TR;
  // this wave's two 16-pixel column blocks: tile row prow, columns pcol[j]
  const int nb0 = 2 * wave;
  const int prow = nb0 / (TW / 16);
  const int pcol[2] = {(nb0 % (TW / 16)) * 16 + lc, ((nb0 + 1) % (TW / 16)) * 16 + lc};

  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int cb = t % ncb, rb = (t / ncb) % nrb, s = t / (ncb * nrb);
    const int c0 = cb * TW, r0 = rb * TR;
    __syncthreads();  // weights staged / previous tile's halo no longer read
    // the halo in items of two adjacent image columns (starting at an even
    // column: one 8-byte load per channel, the pair entirely inside or
    // outside the image) x 8 channels; all loads of a thread are issued
    // before its LDS stores
    {
      constexpr int NPAIR = TW / 2 + 2;  // columns c0 - 2 .. c0 + TW + 1
      constexpr int ITEMS = NPAIR * XROWS * NG;
      constexpr int IT = (ITEMS + NT - 1) / NT;
      f32x2 v[IT][8];
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = tid + it * NT;
        const int pr = i % NPAIR, rr = (i / NPAIR) % XROWS, grp = i / (NPAIR * XROWS);
        const int gi1 = c0 + 2 * pr - 2, gi2 = r0 + rr - 1;
        const bool in = i < ITEMS && gi1 >= 0 && gi1 < n1 && gi2 >= 0 && gi2 < n2;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int ci = grp * 8 + e;
          v[it][e] = f32x2{0.0f, 0.0f};
          if (in && ci < a.cin)
            v[it][e] = *reinterpret_cast<const f32x2*>(
                a.x + (static_cast<int64_t>(s) * a.cin + ci) * P + static_cast<int64_t>(gi2) * n1 + gi1);
        }
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = tid + it * NT;
        if (i >= ITEMS) continue;
        const int pr = i % NPAIR, rr = (i / NPAIR) % XROWS, grp = i / (NPAIR * XROWS);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int pos = 2 * pr - 1 + h;  // LDS position of image column c0 + pos - 1
          if (pos < 0 || pos >= XPOS) continue;
          const u32x4 pk = {pack_bf16(v[it][0][h], v[it][1][h]), pack_bf16(v[it][2][h], v[it][3][h]),
                            pack_bf16(v[it][4][h], v[it][5][h]), pack_bf16(v[it][6][h], v[it][7][h])};
          *reinterpret_cast<u32x4*>(&sX[(rr * XPOS + pos) * XS + grp * 8]) = pk;
        }
      }
    }
    __syncthreads();

    f32x4 acc[MB][2];
#pragma unroll
    for (int m = 0; m < MB; ++m) acc[m][0] = acc[m][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int ks = 0; ks < KSTEPS; ++ks) {
      const int k0 = ks * 32 + g * 8;
      const int tap = k0 / CIN_PAD, ci0 = k0 - tap * CIN_PAD;
      const int ky = tap / 3, kx = tap - 3 * ky;
      bf16x8 bfr[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int off = tap < 9 ? ((prow + ky) * XPOS + pcol[j] + kx) * XS + ci0 : ZSLOT;
        bfr[j] = *reinterpret_cast<const bf16x8*>(&sX[off]);
      }
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        const bf16x8 afr = *reinterpret_cast<const bf16x8*>(&sW[(m * 16 + lc) * WS + k0]);
        acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[0], acc[m][0], 0, 0, 0);
        acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[1], acc[m][1], 0, 0, 0);
      }
    }

    const int gi2 = r0 + prow;
    if (gi2 >= n2) continue;
    // auxiliary inputs of all of this lane's outputs are loaded before the
    // first store (the stores may alias them, so interleaved they would wait
    // out one memory latency each)
    float xa[MB][2][4], xb[MB][2][4];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int co = m * 16 + g * 4 + r;
          const int64_t p = static_cast<int64_t>(gi2) * n1 + c0 + pcol[j];
          const int64_t o = (static_cast<int64_t>(s) * a.cout + co) * P + p;
          xa[m][j][r] = 0.0f;
          xb[m][j][r] = 0.0f;
          if (co >= a.cout) continue;
          if constexpr (EPI == CEPI_RES) {
            xa[m][j][r] = a.aux[o];
          } else if constexpr (EPI == CEPI_OUT) {
            xa[m][j][r] = a.aux[(static_cast<int64_t>(s) * a.aux_ch + co) * P + p];
          } else if constexpr (EPI == CEPI_BWD) {
            if (a.aux) xa[m][j][r] = a.aux[o];
            if (a.out1) xb[m][j][r] = a.aux2[o];
          }
        }
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int co = m * 16 + g * 4 + r;
          if (co >= a.cout) continue;
          const int64_t p = static_cast<int64_t>(gi2) * n1 + c0 + pcol[j];
          const int64_t o = (static_cast<int64_t>(s) * a.cout + co) * P + p;
          const float v = acc[m][j][r];
          if constexpr (EPI == CEPI_SILU) {
            const float av = v + a.bias[co];
            if (a.out0) a.out0[o] = av;
            a.out1[o] = av * sigmoid_f(av);
          } else if constexpr (EPI == CEPI_RES) {
            const float av = v + a.bias[co];
            if (a.out0) a.out0[o] = av;
            a.out1[o] = xa[m][j][r] + av * sigmoid_f(av);
          } else if constexpr (EPI == CEPI_OUT) {
            a.out0[o] = fmaf(a.oscale, v + a.bias[co], xa[m][j][r]);
          } else {
            const float tot = v + xa[m][j][r];
            if (a.out0) a.out0[o] = tot;
            if (a.out1) {
              const float z = xb[m][j][r];
              const float sg = sigmoid_f(z);
              a.out1[o] = tot * (sg * (1.0f + z * (1.0f - sg)));
            }
          }
        }
  }
}

template <int CIN_PAD, int MB>
__global__ __launch_bounds__(NT) void k_wgrad(WgradArgs a, float* part, int ntiles) {
  constexpr int NCOL = 9 * CIN_PAD;
  constexpr int NBM = (NCOL + 15) / 16;  // column blocks of dW
  constexpr int NBT = NBM + 1;           // + the bias block
  constexpr int NBW = (NBT + 3) / 4;     // column blocks per wave
  constexpr int XW = TW + 16;            // halo row pitch: image column j at index 8 + j
  constexpr int XR = TR + 2;
  constexpr int DS = TR * TW + 8;        // dout row pitch
  __shared__ __attribute__((aligned(16))) uint16_t sX[CIN_PAD * XR * XW];
  __shared__ __attribute__((aligned(16))) uint16_t sD[MB * 16 * DS];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, lc = lane & 15;
  const int n1 = a.n1, n2 = a.n2;
  const int64_t P = static_cast<int64_t>(n1) * n2;
  const int ncb = n1 / TW, nrb = (n2 + TR - 1) / TR;
  const int L = a.cout * a.cin * 9 + a.cout;

  for (int i = tid; i < CIN_PAD * XR * XW / 2; i += NT) reinterpret_cast<unsigned*>(sX)[i] = 0u;

  // this lane's column of each of its blocks: kind 0 = weight (ci, ky, kx), 1 = bias, 2 = none
  int xoff[NBW], kxs[NBW], kind[NBW];
#pragma unroll
  for (int i = 0; i < NBW; ++i) {
    const int nb = wave * NBW + i;
    const int n = nb * 16 + lc;
    xoff[i] = 0;
    kxs[i] = 1;
    if (nb < NBM && n < NCOL) {
      const int tap = n / CIN_PAD, ci = n - tap * CIN_PAD;
      const int ky = tap / 3;
      kind[i] = 0;
      kxs[i] = tap - 3 * ky;
      xoff[i] = (ci * XR + ky) * XW + 8;
    } else {
      kind[i] = (nb == NBM && lc == 0) ? 1 : 2;
    }
  }

  f32x4 acc[MB][NBW];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int i = 0; i < NBW; ++i) acc[m][i] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int t0 = static_cast<int>(static_cast<int64_t>(blockIdx.x) * ntiles / gridDim.x);
  const int t1 = static_cast<int>(static_cast<int64_t>(blockIdx.x + 1) * ntiles / gridDim.x);
  for (int t = t0; t < t1; ++t) {
    const int cb = t % ncb, rb = (t / ncb) % nrb, s = t / (ncb * nrb);
    const int c0 = cb * TW, r0 = rb * TR;
    __syncthreads();
    // dout tile [co][TR * TW], 8 pixels per item; all loads of a thread are
    // issued before its LDS stores
    {
      constexpr int ITEMS = MB * 16 * TR * (TW / 8);
      constexpr int IT = (ITEMS + NT - 1) / NT;
      f32x4 lo[IT], hi[IT];
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = tid + it * NT;
        const int c8 = i % (TW / 8), rr = (i / (TW / 8)) % TR, co = i / (TR * (TW / 8));
        const int gi2 = r0 + rr;
        lo[it] = hi[it] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (i < ITEMS && co < a.cout && gi2 < n2) {
          const float* src = a.dout + (static_cast<int64_t>(s) * a.cout + co) * P +
                             static_cast<int64_t>(gi2) * n1 + c0 + c8 * 8;
          lo[it] = *reinterpret_cast<const f32x4*>(src);
          hi[it] = *reinterpret_cast<const f32x4*>(src + 4);
        }
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = tid + it * NT;
        if (i >= ITEMS) continue;
        const int c8 = i % (TW / 8), rr = (i / (TW / 8)) % TR, co = i / (TR * (TW / 8));
        const u32x4 pk = {pack_bf16(lo[it][0], lo[it][1]), pack_bf16(lo[it][2], lo[it][3]),
                          pack_bf16(hi[it][0], hi[it][1]), pack_bf16(hi[it][2], hi[it][3])};
        *reinterpret_cast<u32x4*>(&sD[co * DS + rr * TW + c8 * 8]) = pk;
      }
    }
    // input halo [ci][XR rows][image columns c0 - 2 .. c0 + TW + 1] in pairs
    // starting at even columns (one 8-byte load each; a pair is either inside
    // the image or outside it, as n1 is a multiple of TW), in chunks of CH
    // pairs per thread whose loads are issued before their stores
    {
      constexpr int NPAIR = TW / 2 + 2;
      constexpr int ITEMS = CIN_PAD * XR * NPAIR;
      constexpr int CH = 8;
      for (int base = 0; base < ITEMS; base += CH * NT) {
        f32x2 v[CH];
#pragma unroll
        for (int it = 0; it < CH; ++it) {
          const int i = base + tid + it * NT;
          const int pr = i % NPAIR, rr = (i / NPAIR) % XR, ci = i / (NPAIR * XR);
          const int gi1 = c0 + 2 * pr - 2, gi2 = r0 + rr - 1;
          v[it] = f32x2{0.f, 0.f};
          if (i < ITEMS && ci < a.cin && gi2 >= 0 && gi2 < n2 && gi1 >= 0 && gi1 < n1)
            v[it] = *reinterpret_cast<const f32x2*>(
                a.x + (static_cast<int64_t>(s) * a.cin + ci) * P + static_cast<int64_t>(gi2) * n1 + gi1);
        }
#pragma unroll
        for (int it = 0; it < CH; ++it) {
          const int i = base + tid + it * NT;
          if (i >= ITEMS) continue;
          const int pr = i % NPAIR, rr = (i / NPAIR) % XR, ci = i / (NPAIR * XR);
          reinterpret_cast<unsigned*>(sX)[((ci * XR + rr) * XW + 8 + 2 * pr - 2) / 2] =
              pack_bf16(v[it][0], v[it][1]);
        }
      }
    }
    __syncthreads();

#pragma unroll
    for (int q = 0; q < TR * TW / 32; ++q) {
      const int qr = q / (TW / 32), qc = (q % (TW / 32)) * 32 + g * 8;
      bf16x8 afr[MB];
#pragma unroll
      for (int m = 0; m < MB; ++m)
        afr[m] = *reinterpret_cast<const bf16x8*>(&sD[(m * 16 + lc) * DS + qr * TW + qc]);
#pragma unroll
      for (int i = 0; i < NBW; ++i) {
        u32x4 b = {0u, 0u, 0u, 0u};
        if (kind[i] == 0) {
          const uint16_t* base = &sX[xoff[i] + qr * XW + qc];
          const u32x4 c = *reinterpret_cast<const u32x4*>(base);
          if (kxs[i] == 1) {
            b = c;
          } else if (kxs[i] == 0) {  // columns qc - 1 .. qc + 6
            const unsigned e = *reinterpret_cast<const unsigned*>(base - 2);
            b = u32x4{(e >> 16) | (c[0] << 16), (c[0] >> 16) | (c[1] << 16),
                      (c[1] >> 16) | (c[2] << 16), (c[2] >> 16) | (c[3] << 16)};
          } else {  // columns qc + 1 .. qc + 8
            const unsigned e = *reinterpret_cast<const unsigned*>(base + 8);
            b = u32x4{(c[0] >> 16) | (c[1] << 16), (c[1] >> 16) | (c[2] << 16),
                      (c[2] >> 16) | (c[3] << 16), (c[3] >> 16) | (e << 16)};
          }
        } else if (kind[i] == 1) {
          b = u32x4{0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u};  // bf16 ones
        }
        const bf16x8 bfr = __builtin_bit_cast(bf16x8, b);
#pragma unroll
        for (int m = 0; m < MB; ++m)
          acc[m][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[m], bfr, acc[m][i], 0, 0, 0);
      }
    }
  }

  // partial sums in parameter order: W[co][ci][tap], then b[co]
  float* out = part + static_cast<int64_t>(blockIdx.x) * L;
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = m * 16 + g * 4 + r;
        if (co >= a.cout) continue;
        const int nb = wave * NBW + i;
        const int n = nb * 16 + lc;
        if (kind[i] == 0) {
          const int tap = n / CIN_PAD, ci = n - tap * CIN_PAD;
          if (ci < a.cin) out[(co * a.cin + ci) * 9 + tap] = acc[m][i][r];
        } else if (kind[i] == 1) {
          out[a.cout * a.cin * 9 + co] = acc[m][i][r];
        }
      }
}

// grad[j] = sum over the G partial rows of part[b][j]: a workgroup takes 32
// consecutive j, its 8 thread rows take every 8th partial row, and the 8
// FP64 sums are combined in LDS
constexpr int RJ = 32, RB = NT / RJ;
__global__ void k_reduce_parts(const float* part, int G, int L, float* grad) {
  __shared__ double red[RB][RJ];
  const int jj = threadIdx.x % RJ, bg = threadIdx.x / RJ;
  const int j = blockIdx.x * RJ + jj;
  double s = 0.0;
  if (j < L)
    for (int b = bg; b < G; b += RB) s += part[static_cast<int64_t>(b) * L + j];
  red[bg][jj] = s;
  __syncthreads();
  if (bg == 0 && j < L) {
    double t = 0.0;
    for (int k = 0; k < RB; ++k) t += red[k][jj];
    grad[j] = static_cast<float>(t);
  }
}

__global__ void k_pack_input(const float2* u, const int* idx, const float* cstd, float* x, int S,
                             int64_t P) {
  const int64_t total = static_cast<int64_t>(S) * P;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * NT) {
    const int s = static_cast<int>(i / P);
    const int64_t p = i - s * P;
    const int64_t src = idx ? idx[s] : s;
    const float2 v = u[src * P + p];
    float* xs = x + static_cast<int64_t>(s) * SUR_CIN * P + p;
    xs[0] = v.x;
    xs[P] = v.y;
#pragma unroll
    for (int k = 0; k < 5; ++k) xs[(2 + k) * P] = cstd[src * 5 + k];
  }
}

// base states (complex64 [*][P], sample idx[s] or s) -> planes xb[s][2][P]
__global__ void k_pack_base(const float2* b, const int* idx, float* xb, int S, int64_t P) {
  const int64_t total = static_cast<int64_t>(S) * P;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * NT) {
    const int s = static_cast<int>(i / P);
    const int64_t p = i - s * P;
    const int64_t src = idx ? idx[s] : s;
    const float2 v = b[src * P + p];
    float* xs = xb + 2 * static_cast<int64_t>(s) * P + p;
    xs[0] = v.x;
    xs[P] = v.y;
  }
}

__global__ void k_unpack(const float* y, float2* out, int S, int64_t P) {
  const int64_t total = static_cast<int64_t>(S) * P;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * NT) {
    const int s = static_cast<int>(i / P);
    const int64_t p = i - s * P;
    out[i] = float2{y[(2 * static_cast<int64_t>(s)) * P + p], y[(2 * static_cast<int64_t>(s) + 1) * P + p]};
  }
}

// per-sample loss weights of the relative loss: w[s] = 1 / sum |t_s|^2 (0 for
// a zero target); one workgroup per sample
__global__ void k_rel_weights(const float2* tgt, const int* idx, int64_t toff, double* w, int64_t P) {
  __shared__ double red[NT];
  const int s = blockIdx.x;
  const int64_t src = (idx ? idx[s] : s) + toff;
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < P; p += NT) {
    const float2 t = tgt[src * P + p];
    acc += static_cast<double>(t.x) * t.x + static_cast<double>(t.y) * t.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = NT / 2; k > 0; k >>= 1) {
    if (static_cast<int>(threadIdx.x) < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) w[s] = red[0] > 0.0 ? 1.0 / red[0] : 0.0;
}

// loss = (1/S) sum_s w_s sum_{c,p} (y - t)^2 with w_s = w[s], or 1 / (2P)
// when w is null (the mean square); dy = d loss / dy; *loss += loss
__global__ void k_mse(const float* y, const float2* tgt, const int* idx, int64_t toff,
                      const double* w, float dscale, float* dy, double* loss, int S, int64_t P) {
  __shared__ double red[NT];
  const int64_t total = static_cast<int64_t>(S) * P;
  const double mse_w = 1.0 / (2.0 * static_cast<double>(P));
  double acc = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * NT) {
    const int s = static_cast<int>(i / P);
    const int64_t p = i - s * P;
    const int64_t src = (idx ? idx[s] : s) + toff;
    const float2 t = tgt[src * P + p];
    const int64_t o = 2 * static_cast<int64_t>(s) * P + p;
    const double ws = (w ? w[s] : mse_w) / S;
    const float scale = static_cast<float>(2.0 * ws * dscale);
    const float d0 = y[o] - t.x, d1 = y[o + P] - t.y;
    dy[o] = scale * d0;
    dy[o + P] = scale * d1;
    acc += ws * (static_cast<double>(d0) * d0 + static_cast<double>(d1) * d1);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = NT / 2; k > 0; k >>= 1) {
    if (static_cast<int>(threadIdx.x) < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0]);
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int count, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__device__ __forceinline__ uint16_t to_bf16(float a) {
  return static_cast<uint16_t>(pack_bf16(a, 0.0f) & 0xFFFFu);
}

// wf[co][tap * cin_pad + ci] = W[co][ci][tap];  wt[ci][tap * cinT_pad + co] = W[co][ci][8 - tap]
__global__ void k_pack_weights(const float* W, int cout, int cin, uint16_t* wf, int cout_pad,
                               int cin_pad, uint16_t* wt, int cinT_pad, int coutT_pad) {
  const int KP = kpad_of(cin_pad);
  const int nf = cout_pad * KP;
  const int KT = kpad_of(cinT_pad);
  const int nt = wt ? coutT_pad * KT : 0;
  for (int i = blockIdx.x * NT + threadIdx.x; i < nf + nt; i += gridDim.x * NT) {
    if (i < nf) {
      const int co = i / KP, k = i - co * KP;
      const int tap = k / cin_pad, ci = k - tap * cin_pad;
      const bool ok = co < cout && tap < 9 && ci < cin;
      wf[i] = to_bf16(ok ? W[(co * cin + ci) * 9 + tap] : 0.0f);
    } else {
      const int j = i - nf;
      const int ci = j / KT, k = j - ci * KT;
      const int tap = k / cinT_pad, co = k - tap * cinT_pad;
      const bool ok = ci < cin && tap < 9 && co < cout;
      wt[j] = to_bf16(ok ? W[(co * cin + ci) * 9 + (8 - tap)] : 0.0f);
    }
  }
}

__global__ void k_diff_norms(const float2* a, const float2* b, int64_t n, double* acc) {
  __shared__ double r0[NT], r1[NT];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * NT) {
    const float2 x = a[i], y = b[i];
    const double dr = static_cast<double>(x.x) - y.x, di = static_cast<double>(x.y) - y.y;
    s0 += dr * dr + di * di;
    s1 += static_cast<double>(y.x) * y.x + static_cast<double>(y.y) * y.y;
  }
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&acc[0], r0[0]);
    atomicAdd(&acc[1], r1[0]);
  }
}

__global__ void k_zero(float* p, int64_t count) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * NT)
    p[i] = 0.0f;
}

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
    else
      cus = 1;
  }
  return cus;
}

int grid_for(int64_t work, int per_cu) {
  const int64_t cap = static_cast<int64_t>(device_cus()) * per_cu;
  const int64_t g = (work + NT - 1) / NT;
  return static_cast<int>(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

int conv_kpad(int cin_pad) { return kpad_of(cin_pad); }

hipError_t launch_conv(const ConvArgs& a, int cin_pad, int cout_pad, hipStream_t s) {
  if (a.n1 % TW != 0 || a.n1 <= 0 || a.n2 <= 0 || a.S <= 0) return hipErrorInvalidValue;
  if (a.cin > cin_pad || a.cout > cout_pad) return hipErrorInvalidValue;
  const int ntiles = a.S * ((a.n2 + TR - 1) / TR) * (a.n1 / TW);
  const int grid = ntiles < 2 * device_cus() ? ntiles : 2 * device_cus();
#define CGL_CONV(CI, CO, E)                                                            \
  if (cin_pad == CI && cout_pad == CO && a.epi == E) {                                 \
    hipLaunchKernelGGL((k_conv<CI, CO, E>), dim3(grid), dim3(NT), 0, s, a, ntiles);    \
    return hipGetLastError();                                                          \
  }
  CGL_CONV(8, 48, CEPI_SILU)
  CGL_CONV(48, 48, CEPI_RES)
  CGL_CONV(48, 16, CEPI_OUT)
  CGL_CONV(8, 48, CEPI_BWD)
  CGL_CONV(48, 48, CEPI_BWD)
#undef CGL_CONV
  return hipErrorInvalidValue;
}

int wgrad_grid(int S, int n1, int n2) {
  const int ntiles = S * ((n2 + TR - 1) / TR) * (n1 / TW);
  const int cap = 2 * device_cus();
  return ntiles < cap ? ntiles : cap;
}

hipError_t launch_wgrad(const WgradArgs& a, float* part, float* grad, hipStream_t s) {
  if (a.n1 % TW != 0 || a.n1 <= 0 || a.n2 <= 0 || a.S <= 0) return hipErrorInvalidValue;
  const int ntiles = a.S * ((a.n2 + TR - 1) / TR) * (a.n1 / TW);
  const int G = wgrad_grid(a.S, a.n1, a.n2);
  if (a.cin == SUR_CIN && a.cout == SUR_C) {
    hipLaunchKernelGGL((k_wgrad<8, 3>), dim3(G), dim3(NT), 0, s, a, part, ntiles);
  } else if (a.cin == SUR_C && a.cout == SUR_C) {
    hipLaunchKernelGGL((k_wgrad<48, 3>), dim3(G), dim3(NT), 0, s, a, part, ntiles);
  } else if (a.cin == SUR_C && a.cout == 2) {
    hipLaunchKernelGGL((k_wgrad<48, 1>), dim3(G), dim3(NT), 0, s, a, part, ntiles);
  } else {
    return hipErrorInvalidValue;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int L = a.cout * a.cin * 9 + a.cout;
  hipLaunchKernelGGL(k_reduce_parts, dim3((L + RJ - 1) / RJ), dim3(NT), 0, s, part, G, L, grad);
  return hipGetLastError();
}

hipError_t launch_sur_pack(const void* u, const int* idx, const float* cstd, float* x, int S,
                           int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_input, dim3(grid_for(S * P, 8)), dim3(NT), 0, s,
                     static_cast<const float2*>(u), idx, cstd, x, S, P);
  return hipGetLastError();
}

hipError_t launch_sur_pack_base(const void* b, const int* idx, float* xb, int S, int64_t P,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_pack_base, dim3(grid_for(S * P, 8)), dim3(NT), 0, s,
                     static_cast<const float2*>(b), idx, xb, S, P);
  return hipGetLastError();
}

hipError_t launch_sur_unpack(const float* y, void* out, int S, int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack, dim3(grid_for(S * P, 8)), dim3(NT), 0, s, y,
                     static_cast<float2*>(out), S, P);
  return hipGetLastError();
}

hipError_t launch_mse(const float* y, const void* target, const int* idx, int64_t toff,
                      double* wbuf, float dscale, float* dy, double* loss, int S, int64_t P,
                      hipStream_t s) {
  if (wbuf) {
    hipLaunchKernelGGL(k_rel_weights, dim3(S), dim3(NT), 0, s, static_cast<const float2*>(target),
                       idx, toff, wbuf, P);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_mse, dim3(grid_for(S * P, 4)), dim3(NT), 0, s, y,
                     static_cast<const float2*>(target), idx, toff, wbuf, dscale, dy, loss, S, P);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int count, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((count + NT - 1) / NT), dim3(NT), 0, s, p, g, m, v, count, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const float* W, int cout, int cin, uint16_t* wf, int cout_pad,
                               int cin_pad, uint16_t* wt, int cinT_pad, int coutT_pad,
                               hipStream_t s) {
  const int64_t n = static_cast<int64_t>(cout_pad) * kpad_of(cin_pad) +
                    (wt ? static_cast<int64_t>(coutT_pad) * kpad_of(cinT_pad) : 0);
  hipLaunchKernelGGL(k_pack_weights, dim3(grid_for(n, 1)), dim3(NT), 0, s, W, cout, cin, wf,
                     cout_pad, cin_pad, wt, cinT_pad, coutT_pad);
  return hipGetLastError();
}

hipError_t launch_diff_norms(const void* a, const void* b, int64_t n, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_diff_norms, dim3(grid_for(n, 2)), dim3(NT), 0, s,
                     static_cast<const float2*>(a), static_cast<const float2*>(b), n, acc);
  return hipGetLastError();
}

hipError_t launch_zero(float* p, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(grid_for(count, 8)), dim3(NT), 0, s, p, count);
  return hipGetLastError();
}

}  // namespace cgl
