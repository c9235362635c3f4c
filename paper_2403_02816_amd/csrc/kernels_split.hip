// Split-precision mu-mode product on CDNA4 BF16 MFMA (v_mfma_f32_32x32x16_bf16)
// with FP32 accumulation.
//
// Every operand is a sum of three bf16 terms (hi + mid + lo, each the bf16
// rounding of what the previous terms left over), which carries ~24
// significant bits.  Of the nine term products the six with i + j <= 2 are
// kept (the dropped ones are below FP32 rounding of the result).  The complex
// product is split into four real products,
//   Re y += Re M Re x - Im M Im x,   Im y += Im M Re x + Re M Im x,
// so one workgroup tile costs 6 x 4 MFMAs per 16-deep contraction step.
// Operator planes come pre-split from the host (split_layout.hpp); the state
// is split on the fly while it is staged into LDS (the state arrives as
// complex64, or complex128 when the plan keeps an FP64 master state).
//
// Tiling: a workgroup (4 waves) owns 64 complex output rows x 64 fibres;
// each wave owns one 32 x 32 block (one accumulator for the real part, one
// for the imaginary part).  A stage covers 16 complex contraction indices:
// 6 operator planes (64 rows x 16) and 6 state planes (64 fibres x 16), rows
// padded to 48 bytes so the 16-byte MFMA operand reads hit distinct LDS banks.
#include "kernels.hpp"
#include "pointwise.hpp"
#include "split_layout.hpp"

namespace cgl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(8)));

namespace {

constexpr int PT = SPK_P;    // 64 complex rows
constexpr int FT = SP_FT;    // 64 fibres
constexpr int KS = SPK_K;    // 16 complex contraction indices per stage
constexpr int PITCH = 24;    // LDS row pitch in bf16 (48 bytes)

__device__ __forceinline__ int64_t fibre_base(int64_t f, int64_t R, int n) {
  return (R == 1) ? f * (int64_t)n : (f % R) + (f / R) * R * (int64_t)n;
}

__device__ __forceinline__ unsigned xcd_remap(unsigned h, unsigned G) {
  return ((G & 7u) == 0u) ? (h & 7u) * (G >> 3) + (h >> 3) : h;
}

// three bf16 terms of x (RNE at each level; remainders exact in FP64)
__device__ __forceinline__ void split3(double x, unsigned short t[3]) {
  double r = x;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const __bf16 h = static_cast<__bf16>(static_cast<float>(r));
    t[i] = __builtin_bit_cast(unsigned short, h);
    r -= static_cast<double>(static_cast<float>(h));
  }
}

__device__ __forceinline__ cd load_c(const void* p, int64_t off, bool f64) {
  if (f64) {
    const double2 v = reinterpret_cast<const double2*>(p)[off];
    return {v.x, v.y};
  }
  const float2 v = reinterpret_cast<const float2*>(p)[off];
  return {static_cast<double>(v.x), static_cast<double>(v.y)};
}

// two adjacent complex elements at off, off+1
__device__ __forceinline__ void load_c2(const void* p, int64_t off, bool f64, cd& x, cd& y) {
  if (f64) {
    const double2* q = reinterpret_cast<const double2*>(p) + off;
    const double2 a = q[0], b = q[1];
    x = {a.x, a.y};
    y = {b.x, b.y};
  } else {
    const f32x4u v = *reinterpret_cast<const f32x4u*>(reinterpret_cast<const float*>(p) + 2 * off);
    x = {static_cast<double>(v[0]), static_cast<double>(v[1])};
    y = {static_cast<double>(v[2]), static_cast<double>(v[3])};
  }
}

__device__ __forceinline__ void store_c(void* p, int64_t off, bool f64, cd v) {
  if (f64)
    reinterpret_cast<double2*>(p)[off] = double2{v.re, v.im};
  else
    reinterpret_cast<float2*>(p)[off] = float2{static_cast<float>(v.re), static_cast<float>(v.im)};
}

__device__ __forceinline__ bf16x8 neg8(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

template <bool CONTIG>
__global__ __launch_bounds__(256) void k_pass_split(PassSplit a) {
  __shared__ __attribute__((aligned(16))) unsigned short sA[6][PT][PITCH];
  __shared__ __attribute__((aligned(16))) unsigned short sB[6][FT][PITCH];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wp = wave & 1;
  const int wf = wave >> 1;
  const int nP = a.Pp / PT;
  const int nKS = a.Kp / KS;
  const unsigned w = xcd_remap(blockIdx.x, gridDim.x);
  const int pt = static_cast<int>(w % nP);
  const int64_t f0 = static_cast<int64_t>(w / nP) * FT;
  const unsigned short* opblk = a.op + static_cast<size_t>(pt) * nKS * (6 * PT * KS);
  const bool if64 = a.in_f64 != 0;
  const bool of64 = a.out_f64 != 0;

  // staging assignment: two fibres (fl[0], fl[1]) x two contraction indices (2kp, 2kp+1)
  int fl[2], kp;
  if (CONTIG) {
    fl[0] = tid >> 3;
    fl[1] = fl[0] + 32;
    kp = tid & 7;
  } else {
    fl[0] = 2 * (tid & 31);
    fl[1] = fl[0] + 1;
    kp = tid >> 5;
  }
  int64_t gb[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int64_t f = f0 + fl[i];
    gb[i] = (f < a.F) ? fibre_base(f, a.R, a.n) : -1;
  }
  const bool pairF = (!CONTIG) && gb[0] >= 0 && gb[1] == gb[0] + 1;

  f32x16 accr, acci;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    accr[r] = 0.0f;
    acci[r] = 0.0f;
  }
  unsigned flag = 0;

  const int row = lane & 31;
  const int kh = (lane >> 5) * 8;

  for (int ks = 0; ks < nKS; ++ks) {
    // ---- operator stage: 768 chunks of 16 bytes
    {
      const u32x4* src = reinterpret_cast<const u32x4*>(opblk + static_cast<size_t>(ks) * (6 * PT * KS));
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int c = tid + 256 * j;
        const u32x4 v = src[c];
        const int q = c >> 7;
        const int r = (c >> 1) & 63;
        const int h = (c & 1) * 8;
        *reinterpret_cast<u32x4*>(&sA[q][r][h]) = v;
      }
    }
    // ---- state stage: 4 complex values per thread
    {
      const int k = ks * KS + 2 * kp;
      cd v[2][2];  // [fibre i][k offset]
#pragma unroll
      for (int i = 0; i < 2; ++i) v[i][0] = v[i][1] = cd{0.0, 0.0};
      if (CONTIG) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          if (gb[i] < 0) continue;
          if (k + 1 < a.n) {
            load_c2(a.in0, gb[i] + k, if64, v[i][0], v[i][1]);
          } else if (k < a.n) {
            v[i][0] = load_c(a.in0, gb[i] + k, if64);
          }
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          if (k + kk >= a.n) continue;
          if (pairF) {
            load_c2(a.in0, gb[0] + a.R * (int64_t)(k + kk), if64, v[0][kk], v[1][kk]);
          } else {
#pragma unroll
            for (int i = 0; i < 2; ++i)
              if (gb[i] >= 0) v[i][kk] = load_c(a.in0, gb[i] + a.R * (int64_t)(k + kk), if64);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          if (a.pro == PRO_FLOW) {
            v[i][kk] = half_flow(v[i][kk], a.nl, flag);
          } else if (a.pro == PRO_G) {
            v[i][kk] = g_cgl(v[i][kk], a.nl);
          }
        }
      // split and write: plane q (0..2 re terms, 3..5 im terms), two k per u32
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        unsigned short r0[3], r1[3], i0[3], i1[3];
        split3(v[i][0].re, r0);
        split3(v[i][1].re, r1);
        split3(v[i][0].im, i0);
        split3(v[i][1].im, i1);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          *reinterpret_cast<unsigned*>(&sB[t][fl[i]][2 * kp]) =
              static_cast<unsigned>(r0[t]) | (static_cast<unsigned>(r1[t]) << 16);
          *reinterpret_cast<unsigned*>(&sB[3 + t][fl[i]][2 * kp]) =
              static_cast<unsigned>(i0[t]) | (static_cast<unsigned>(i1[t]) << 16);
        }
      }
    }
    __syncthreads();
    // ---- MFMA: 6 term products x 4 real products
    {
      bf16x8 ar[3], ai[3], an[3], br[3], bi[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        ar[t] = *reinterpret_cast<const bf16x8*>(&sA[t][wp * 32 + row][kh]);
        ai[t] = *reinterpret_cast<const bf16x8*>(&sA[3 + t][wp * 32 + row][kh]);
        an[t] = neg8(ai[t]);
        br[t] = *reinterpret_cast<const bf16x8*>(&sB[t][wf * 32 + row][kh]);
        bi[t] = *reinterpret_cast<const bf16x8*>(&sB[3 + t][wf * 32 + row][kh]);
      }
      // term pairs (i, j) with i + j <= 2, smallest first
      constexpr int PI[6] = {2, 1, 0, 1, 0, 0};
      constexpr int PJ[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int ti = PI[q], tj = PJ[q];
        accr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ti], br[tj], accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai[ti], br[tj], acci, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(an[ti], bi[tj], accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ti], bi[tj], acci, 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // ---- epilogue: lane holds rows 8q + 4(lane/32) + s (q, s < 4) of fibre column lane%32
  const int64_t f = f0 + wf * 32 + (lane & 31);
  if (f < a.F) {
    const int64_t base = fibre_base(f, a.R, a.n);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = pt * PT + wp * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (m >= a.n) continue;
      const int64_t off = base + a.R * (int64_t)m;
      const cd y = {static_cast<double>(accr[r]), static_cast<double>(acci[r])};
      if (a.epi == EPI_NONE) {
        store_c(a.out0, off, of64, y);
      } else if (a.epi == EPI_FLOW) {
        const cd z = half_flow(y, a.nl, flag);
        if (!finite2(z)) flag |= FLAG_NONFINITE;
        store_c(a.out0, off, of64, z);
      } else {
        const cd x = load_c(a.aux, off, false);
        if (a.epi == EPI_L4_R1) {  // y = Q, x = P
          cd X, Y;
          lawson_r1(x, y, a.nl, X, Y);
          store_c(a.out0, off, of64, X);
          store_c(a.out1, off, of64, Y);
        } else {  // EPI_L4_R2: y = H Y, x = H X
          const cd z = lawson_r2(x, y, a.nl);
          if (!finite2(z)) flag |= FLAG_NONFINITE;
          store_c(a.out0, off, of64, z);
        }
      }
    }
  }
  if (flag) atomicOr(a.flag, flag);
}

}  // namespace

hipError_t launch_pass_split(const PassSplit& a, hipStream_t s) {
  if (a.Pp % PT != 0 || a.Kp % KS != 0 || a.Kp < a.n || a.Pp < a.n || a.F <= 0)
    return hipErrorInvalidValue;
  if (!a.in0 || !a.out0 || !a.op || !a.flag) return hipErrorInvalidValue;
  if ((a.epi == EPI_L4_R1 || a.epi == EPI_L4_R2) && !a.aux) return hipErrorInvalidValue;
  if (a.epi == EPI_L4_R1 && !a.out1) return hipErrorInvalidValue;
  const int64_t nF = (a.F + FT - 1) / FT;
  const int64_t G = nF * (a.Pp / PT);
  if (G > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(G)), block(256);
  if (a.R == 1)
    hipLaunchKernelGGL(k_pass_split<true>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(k_pass_split<false>, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace cgl
