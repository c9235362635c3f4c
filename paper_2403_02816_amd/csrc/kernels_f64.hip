// FP64 mu-mode product on CDNA4 FP64 MFMA (v_mfma_f64_16x16x4_f64).
//
// One workgroup (4 waves) computes a 64 (real rows of the 2n x 2n embedding,
// i.e. 32 complex outputs) x 64 (fibres) tile of  out = M_emb * in_emb.  The
// contraction runs in stages of 16 real rows (8 complex) staged in LDS:
//   - operator stage: 16 x 64 doubles of the embedding (rows k', p' fastest),
//   - input stage: 8 complex elements of 64 fibres, loaded with 16-byte
//     loads that are coalesced along the contiguous direction (along the
//     fibre when mu = 1, across fibres when mu > 1), split into re/im rows.
// Each wave owns a 32 x 32 sub-tile = 2 x 2 MFMA blocks.  The accumulator of
// lane l holds rows l/16 + 4r (r < 4) of a 16-row block; the host orders the
// embedding's rows so that these are two whole complex numbers.
// Workgroups are remapped so that the P-tiles sharing one input tile run on
// the same XCD (its L2 keeps the input tile for all of them).  The next
// stage's operator and input values are loaded into registers before the
// current stage's MFMAs; three workgroups fit on a CU (168 VGPRs, 20 KB LDS).
#include "kernels.hpp"
#include "pointwise.hpp"

namespace cgl {

typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int PT = F64_PT;
constexpr int FT = F64_FT;
constexpr int KC = F64_KC;
constexpr int LDP = PT + 16;  // LDS row pitch in doubles (two rows cover all banks)
constexpr int LDF = FT + 16;

__device__ __forceinline__ int64_t fibre_base(int64_t f, int64_t R, int n) {
  return (R == 1) ? f * (int64_t)n : (f % R) + (f / R) * R * (int64_t)n;
}

__device__ __forceinline__ unsigned xcd_remap(unsigned h, unsigned G) {
  return ((G & 7u) == 0u) ? (h & 7u) * (G >> 3) + (h >> 3) : h;
}

template <bool CONTIG>
__global__ __launch_bounds__(256, 3) void k_pass_f64(PassF64 a) {
  __shared__ double sOp[KC][LDP];
  __shared__ double sIn[KC][LDF];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wp = wave & 1;
  const int wf = wave >> 1;
  const int nP = a.Pp / PT;
  const unsigned w = xcd_remap(blockIdx.x, gridDim.x);
  const int pt = static_cast<int>(w % nP);
  const int64_t f0 = static_cast<int64_t>(w / nP) * FT;
  const int p0 = pt * PT;

  // staging assignment: NJ complex input elements and NJ operator pairs per
  // thread and stage (KC/2 complex contraction indices x 64 fibres)
  constexpr int KCC = KC / 2;
  constexpr int NJ = KCC * FT / 256;
  static_assert(NJ * 256 == KCC * FT && NJ * 256 == KC * PT / 2, "stage must split evenly");
  int fl[NJ], kl[NJ];
  int64_t gbase[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int e = tid + 256 * j;
    if (CONTIG) {
      fl[j] = e / KCC;
      kl[j] = e % KCC;
    } else {
      fl[j] = e % FT;
      kl[j] = e / FT;
    }
    const int64_t f = f0 + fl[j];
    gbase[j] = (f < a.F) ? fibre_base(f, a.R, a.n) : -1;
  }

  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  unsigned flag = 0;

  // the next stage's operator and input values, loaded into registers before
  // the current stage's MFMAs so that their latency overlaps the math
  double2 opv[NJ];
  cd xin[NJ];
  bool xok[NJ];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int e = tid + 256 * j;
      opv[j] = *reinterpret_cast<const double2*>(a.op + (int64_t)(k0 + e / (PT / 2)) * a.Pp + p0 +
                                                 2 * (e % (PT / 2)));
      const int k = (k0 >> 1) + kl[j];
      xok[j] = gbase[j] >= 0 && k < a.n;
      xin[j] = {0.0, 0.0};
      if (xok[j]) {
        const double2 v =
            *reinterpret_cast<const double2*>(a.in0 + 2 * (gbase[j] + a.R * (int64_t)k));
        xin[j] = {v.x, v.y};
      }
    }
  };

  load_stage(0);
  for (int k0 = 0; k0 < a.Kp; k0 += KC) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int e = tid + 256 * j;
      const int kr = e / (PT / 2);
      const int c2 = e % (PT / 2);
      sOp[kr][2 * c2] = opv[j].x;
      sOp[kr][2 * c2 + 1] = opv[j].y;
      cd x = xin[j];
      if (xok[j]) {
        if (a.pro == PRO_FLOW) {
          x = flow_in(x, a.nl.tf, a.nl, flag);
        } else if (a.pro == PRO_G) {
          x = g_cgl(x, a.nl);
        }
      }
      sIn[2 * kl[j]][fl[j]] = x.re;
      sIn[2 * kl[j] + 1][fl[j]] = x.im;
    }
    __syncthreads();
    if (k0 + KC < a.Kp) load_stage(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int kr = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int pb = 0; pb < 2; ++pb) av[pb] = sOp[kr][wp * 32 + pb * 16 + (lane & 15)];
#pragma unroll
      for (int fb = 0; fb < 2; ++fb) bv[fb] = sIn[kr][wf * 32 + fb * 16 + (lane & 15)];
#pragma unroll
      for (int pb = 0; pb < 2; ++pb)
#pragma unroll
        for (int fb = 0; fb < 2; ++fb)
          acc[pb][fb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[pb], bv[fb], acc[pb][fb], 0, 0, 0);
    }
    __syncthreads();
  }

  // epilogue: the accumulator of lane l holds rows g + 4r (g = l/16, r < 4)
  // of a 16-row block b; the host's row permutation makes registers (0, 1)
  // the (re, im) of output m = 8b + g and registers (2, 3) those of m + 4.
  // For the epilogues with an auxiliary input (Lawson combinations, split4)
  // the 8 auxiliary values of the lane are loaded before the first store
  // (stores could alias them).
  const bool lawson = a.epi == EPI_L4_R1 || a.epi == EPI_L4_R2 || a.epi == EPI_RICH ||
                      a.epi == EPI_L2;
  double2 xa[2][2][2];
#pragma unroll
  for (int pb = 0; pb < 2; ++pb)
#pragma unroll
    for (int fb = 0; fb < 2; ++fb)
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int m = 8 * ((p0 + wp * 32 + pb * 16) >> 4) + (lane >> 4) + 4 * hh;
        const int64_t f = f0 + wf * 32 + fb * 16 + (lane & 15);
        xa[pb][fb][hh] = double2{0.0, 0.0};
        if (lawson && f < a.F && m < a.n)
          xa[pb][fb][hh] = *reinterpret_cast<const double2*>(
              a.aux + 2 * (fibre_base(f, a.R, a.n) + a.R * (int64_t)m));
      }
#pragma unroll
  for (int pb = 0; pb < 2; ++pb) {
#pragma unroll
    for (int fb = 0; fb < 2; ++fb) {
      const int mblk = 8 * ((p0 + wp * 32 + pb * 16) >> 4) + (lane >> 4);
      const int64_t f = f0 + wf * 32 + fb * 16 + (lane & 15);
      if (f >= a.F) continue;
      const int64_t base = fibre_base(f, a.R, a.n);
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int m = mblk + 4 * hh;
        if (m >= a.n) continue;
        const int64_t off = 2 * (base + a.R * (int64_t)m);
        const cd y = {acc[pb][fb][2 * hh], acc[pb][fb][2 * hh + 1]};
        if (a.epi == EPI_NONE) {
          *reinterpret_cast<double2*>(a.out0 + off) = double2{y.re, y.im};
        } else if (a.epi == EPI_FLOW || a.epi == EPI_MID) {
          const cd z = a.epi == EPI_FLOW ? flow_out(y, a.nl.tf, a.nl, flag)
                                         : flow_mid(y, a.nl.tf, a.nl, flag);
          if (!finite2(z)) flag |= FLAG_NONFINITE;
          *reinterpret_cast<double2*>(a.out0 + off) = double2{z.re, z.im};
        } else {
          const cd x = {xa[pb][fb][hh].x, xa[pb][fb][hh].y};
          if (a.epi == EPI_L4_R1) {  // y = Q, x = P
            cd X, Y;
            lawson_r1(x, y, a.nl, X, Y);
            *reinterpret_cast<double2*>(a.out0 + off) = double2{X.re, X.im};
            *reinterpret_cast<double2*>(a.out1 + off) = double2{Y.re, Y.im};
          } else {
            // EPI_L4_R2: y = H Y, x = H X; EPI_RICH: x = the full Strang
            // step; EPI_L2: y = Q, x = P
            const cd z = a.epi == EPI_L4_R2 ? lawson_r2(x, y, a.nl)
                         : a.epi == EPI_RICH ? richardson(y, x, a.nl, flag)
                                             : lawson2(x, y, a.nl, 0.5 * a.nl.tau);
            if (!finite2(z)) flag |= FLAG_NONFINITE;
            *reinterpret_cast<double2*>(a.out0 + off) = double2{z.re, z.im};
          }
        }
      }
    }
  }
  if (flag) atomicOr(a.flag, flag);
}

__global__ void k_clear_flag(unsigned* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0u;
}

}  // namespace

hipError_t launch_pass_f64(const PassF64& a, hipStream_t s) {
  if (a.Pp % PT != 0 || a.Kp % KC != 0 || a.Kp < 2 * a.n || a.Pp < 2 * a.n || a.F <= 0)
    return hipErrorInvalidValue;
  if (!a.in0 || !a.out0 || !a.op || !a.flag) return hipErrorInvalidValue;
  if ((a.epi == EPI_L4_R1 || a.epi == EPI_L4_R2 || a.epi == EPI_RICH || a.epi == EPI_L2) && !a.aux)
    return hipErrorInvalidValue;
  if (a.epi == EPI_L4_R1 && !a.out1) return hipErrorInvalidValue;
  if (a.epi < EPI_NONE || a.epi > EPI_L2) return hipErrorInvalidValue;
  const int64_t nF = (a.F + FT - 1) / FT;
  const int64_t G = nF * (a.Pp / PT);
  if (G > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(G)), block(256);
  if (a.R == 1)
    hipLaunchKernelGGL(k_pass_f64<true>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(k_pass_f64<false>, grid, block, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_clear_flag(unsigned* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, flag);
  return hipGetLastError();
}

}  // namespace cgl
