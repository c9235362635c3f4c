// Split-precision mu-mode product on CDNA4 BF16 MFMA (v_mfma_f32_32x32x16_bf16)
// with FP32 accumulation.
//
// Every operand is a sum of three bf16 terms (hi + mid + lo, each the bf16
// rounding of what the previous terms left over), which carries the 24
// significant bits of an FP32 value.  Of the nine term products the six with
// i + j <= 2 are kept (the dropped ones are below FP32 rounding of the
// result).  The complex product is split into four real products,
//   Re y += Re M Re x - Im M Im x,   Im y += Im M Re x + Re M Im x,
// so one 32 x 32 output block costs 6 x 4 MFMAs per 16-deep contraction step.
// Operator planes come pre-split from the host (split_layout.hpp); the state
// is split on the fly (packed FP32 -> bf16 conversions) while it is staged
// into LDS.  The state arrives as complex64, or complex128 when the plan
// keeps an FP64 master state.
//
// Tiling: a workgroup (4 waves, 2 x 2) owns PT complex output rows x 64
// fibres; each wave owns PT/64 blocks of 32 x 32 (one FP32 accumulator for the
// real part, one for the imaginary part, per block).  A stage covers KS
// complex contraction indices: 6 operator planes (PT rows x KS) and 6 state
// planes (64 fibres x KS), rows padded by 16 bytes so the 16-byte MFMA operand
// reads of 16 lanes hit distinct LDS banks.  Two shapes are compiled,
// (PT, KS) = (64, 32) and (128, 16); the plan's autotuner picks one per
// direction.  The next stage's global loads are issued into registers before
// the current stage's MFMAs, so their latency overlaps the math.
#include <type_traits>

#include "kernels.hpp"
#include "pointwise.hpp"
#include "split_layout.hpp"

namespace cgl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int FT = SP_FT;  // 64 fibres

// Wave-uniform values read from the first lane: a buffer resource built from
// them is scalar.  (Fields of a work item loaded from memory the kernel also
// writes come back in vector registers; a buffer resource built from those
// turns every load through it into a waterfall loop.)
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return reinterpret_cast<P*>((static_cast<uint64_t>(hi) << 32) | lo);
}

// Barrier between the stages of a pipelined product.  A wave waits for its
// LDS accesses and for every vector-memory operation but the last NV: the
// operator copies to LDS are issued before the state loads of a later stage,
// so the copies have landed while those NV loads stay in flight across the
// barrier (the release fence of __syncthreads() would wait for them too and
// cut their prefetch distance to one stage).  The fences order LDS only.
template <int NV>
__device__ __forceinline__ void stage_barrier() {
  static_assert(NV >= 0 && NV < 16, "vmcnt field");
  __builtin_amdgcn_s_waitcnt(0x0070 | NV);  // vmcnt(NV) expcnt(7) lgkmcnt(0)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int64_t fibre_base(int64_t f, int64_t R, int n) {
  return (R == 1) ? f * (int64_t)n : (f % R) + (f / R) * R * (int64_t)n;
}

// start of fibre f < F in an output of stride R; a stride of at least F (the
// rotated layouts, R = F) leaves f as it is, without a 64-bit division
__device__ __forceinline__ int64_t fibre_start(int64_t f, int64_t R, int n, int64_t F) {
  return R >= F ? f : fibre_base(f, R, n);
}

__device__ __forceinline__ unsigned xcd_remap(unsigned h, unsigned G) {
  return ((G & 7u) == 0u) ? (h & 7u) * (G >> 3) + (h >> 3) : h;
}

// three bf16 terms of two FP32 values (packed conversion, RNE); the
// remainders are exact in FP32
__device__ __forceinline__ void split3x2(float x0, float x1, unsigned t[3]) {
  f32x2 r = {x0, x1};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const bf16x2 h = __builtin_convertvector(r, bf16x2);
    t[i] = __builtin_bit_cast(unsigned, h);
    r = r - __builtin_convertvector(h, f32x2);
  }
}

__device__ __forceinline__ cf load_cf(const void* p, int64_t off, bool f64) {
  if (f64) {
    const double2 v = reinterpret_cast<const double2*>(p)[off];
    return {static_cast<float>(v.x), static_cast<float>(v.y)};
  }
  const float2 v = reinterpret_cast<const float2*>(p)[off];
  return {v.x, v.y};
}

// two adjacent complex elements at off, off+1
__device__ __forceinline__ void load_cf2(const void* p, int64_t off, bool f64, cf& x, cf& y) {
  if (f64) {
    const double2* q = reinterpret_cast<const double2*>(p) + off;
    const double2 a = q[0], b = q[1];
    x = {static_cast<float>(a.x), static_cast<float>(a.y)};
    y = {static_cast<float>(b.x), static_cast<float>(b.y)};
  } else {
    const f32x4u v = *reinterpret_cast<const f32x4u*>(reinterpret_cast<const float*>(p) + 2 * off);
    x = {v[0], v[1]};
    y = {v[2], v[3]};
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

// Staging geometry of one thread: FI fibres x KJ consecutive contraction
// indices.  Contiguous contraction axis: 1 fibre x KS/4 indices (4 threads
// cover the KS indices of a fibre, 8 consecutive lanes 8 fibres); strided: 2
// adjacent fibres x KS/8 indices (32 threads cover 64 adjacent fibres of one
// index with 16-byte loads).
template <int KS, bool CONTIG>
struct Stage {
  static constexpr int FI = CONTIG ? 1 : 2;
  static constexpr int KJ = CONTIG ? KS / 4 : KS / 8;
};

// stores the packed bf16 terms of KJ consecutive indices (KJ/2 u32)
template <int KJ>
__device__ __forceinline__ void store_terms(unsigned short* dst, const unsigned* v) {
  if constexpr (KJ == 8) {
    *reinterpret_cast<u32x4*>(dst) = u32x4{v[0], v[1], v[2], v[3]};
  } else if constexpr (KJ == 4) {
    *reinterpret_cast<u32x2*>(dst) = u32x2{v[0], v[1]};
  } else {
    *reinterpret_cast<unsigned*>(dst) = v[0];
  }
}

template <int PT, int KS>
struct Lds {
  static constexpr int PITCH = KS + 8;  // LDS row pitch in bf16
  unsigned short A[6][PT][PITCH];
  unsigned short B[6][FT][PITCH];
};

// Epilogue of a tile: the accumulators of a wave (PB blocks of 32 x 32; lane
// holds rows 8q + 4(lane/32) + s (q, s < 4) of fibre column lane%32) written
// to the output with the output stride, through the pointwise epilogue when
// there is one.  lds_mem: at least 64 x 65 float2 of workgroup memory that is
// free (every wave is past its last read of the stage buffers).
constexpr int EPI_LDS_BYTES = 64 * (SP_FT + 1) * 8;

template <int PT>
__device__ __forceinline__ void split_epilogue(const PassSplit& a, int pt, int64_t f0,
                                               f32x16 (&accr)[PT / 64], f32x16 (&acci)[PT / 64],
                                               unsigned& flag, void* lds_mem) {
  constexpr int PB = PT / 64;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wp = wave & 1;
  const int wf = wave >> 1;
  const bool of64 = a.out_f64 != 0;
  if (a.epi == EPI_NONE) {
    const int64_t f = f0 + wf * 32 + (lane & 31);
    if (f < a.F) {
      const int64_t base = fibre_start(f, a.R_out, a.n, a.F);
#pragma unroll
      for (int b = 0; b < PB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = pt * PT + wp * (PT / 2) + b * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          if (m >= a.n) continue;
          const int64_t off = base + a.R_out * (int64_t)m;
          if (of64)
            reinterpret_cast<double2*>(a.out0)[off] =
                double2{static_cast<double>(accr[b][r]), static_cast<double>(acci[b][r])};
          else
            reinterpret_cast<float2*>(a.out0)[off] = float2{accr[b][r], acci[b][r]};
        }
    }
  } else {
    // pointwise epilogues (flow, Lawson4 combinations) are long FP64 code:
    // the accumulators go through LDS, 64 rows at a time, and one copy of
    // the code runs in a loop over the elements (consecutive threads take
    // consecutive fibres of one row)
    constexpr int EP = FT + 1;  // row pitch in float2
    float2* sE = reinterpret_cast<float2*>(lds_mem);
    // a thread keeps one fibre (column fc = tid mod FT) in the loops below
    static_assert(256 % FT == 0, "one fibre per thread");
    const int fc = tid % FT;
    const int64_t f = f0 + fc;
    const int64_t fst = f < a.F ? fibre_start(f, a.R_out, a.n, a.F) : 0;
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      // rows wp * (PT / 2) + b * 32 + [0, 32) of the tile -> LDS rows wp * 32 + [0, 32)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int lr = wp * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        sE[lr * EP + wf * 32 + (lane & 31)] = float2{accr[b][r], acci[b][r]};
      }
      __syncthreads();
#pragma unroll 1
      for (int e = tid; e < 64 * FT; e += 256) {
        const int lr = e / FT;
        const int m = pt * PT + (lr / 32) * (PT / 2) + b * 32 + (lr % 32);
        if (m >= a.n || f >= a.F) continue;
        const int64_t off = fst + a.R_out * (int64_t)m;
        const float2 v = sE[lr * EP + fc];
        const cd y = {static_cast<double>(v.x), static_cast<double>(v.y)};
        if (a.epi == EPI_FLOW || a.epi == EPI_MID) {
          const cd z = a.epi == EPI_FLOW ? flow_out(y, a.nl.tf, a.nl, flag)
                                         : flow_mid(y, a.nl.tf, a.nl, flag);
          if (!finite2(z)) flag |= FLAG_NONFINITE;
          store_c(a.out0, off, of64, z);
        } else {
          const cd x = load_c(a.aux, off, a.aux_f64 != 0);
          if (a.epi == EPI_L4_R1) {  // y = Q, x = P
            cd X, Y;
            lawson_r1(x, y, a.nl, X, Y);
            store_c(a.out0, off, of64, X);
            store_c(a.out1, off, of64, Y);
          } else {
            // EPI_L4_R2: y = H Y, x = H X; EPI_RICH: x = the full Strang
            // step; EPI_L2: y = Q, x = P
            const cd z = a.epi == EPI_L4_R2 ? lawson_r2(x, y, a.nl)
                         : a.epi == EPI_RICH ? richardson(y, x, a.nl, flag)
                                             : lawson2(x, y, a.nl, 0.5 * a.nl.tau);
            if (!finite2(z)) flag |= FLAG_NONFINITE;
            store_c(a.out0, off, of64, z);
          }
        }
      }
      // LDS is read here until every thread is done: the next block, or the
      // next work item of a persistent grid, stages into it afterwards
      __syncthreads();
    }
  }
}

// One workgroup tile: output rows [pt*PT, pt*PT + PT) x fibres [f0, f0 + 64)
// of the pass described by a.  Every thread of the workgroup calls it.
template <int PT, int KS, bool CONTIG, int PRO, bool IN64>
__device__ __forceinline__ void split_tile(const PassSplit& a, int pt, int64_t f0,
                                           Lds<PT, KS>& lds) {
  constexpr int FI = Stage<KS, CONTIG>::FI;
  constexpr int KJ = Stage<KS, CONTIG>::KJ;
  constexpr int PB = PT / 64;          // 32-row blocks per wave
  constexpr int CPS = PT * KS / 8;     // 16-byte chunks per plane per stage
  constexpr int OPCH = 6 * CPS / 256;  // operator chunks per thread per stage
  static_assert(OPCH * 256 == 6 * CPS, "operator stage must split evenly");
  auto& sA = lds.A;
  auto& sB = lds.B;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wp = wave & 1;
  const int wf = wave >> 1;
  const int nKS = a.Kp / KS;
  const u32x4* opblk =
      reinterpret_cast<const u32x4*>(a.op + static_cast<size_t>(pt) * nKS * (6 * PT * KS));
  // every fibre of the tile exists and every stage is full: no masks needed
  const bool full = (f0 + FT <= a.F) && (a.n % KS == 0);

  // this thread's fibres and first contraction index within a stage
  int fl[FI];
  int k0t;
  if (CONTIG) {
    // 8 consecutive lanes take 8 fibres (LDS rows) at one index chunk
    fl[0] = (tid & 7) + 8 * (tid >> 5);
    k0t = KJ * ((tid >> 3) & 3);
  } else {
    fl[0] = 2 * (tid & 31);
    fl[FI - 1] = fl[0] + 1;
    k0t = KJ * (tid >> 5);
  }
  int64_t gb[FI];
#pragma unroll
  for (int i = 0; i < FI; ++i) {
    const int64_t f = f0 + fl[i];
    gb[i] = (f < a.F) ? fibre_base(f, a.R, a.n) : -1;
  }
  const bool pairF = (!CONTIG) && gb[0] >= 0 && gb[FI - 1] == gb[0] + 1;
  // contiguous fast path: a running pointer to this thread's first element
  const char* inp = reinterpret_cast<const char*>(a.in0) +
                    (CONTIG ? (gb[0] >= 0 ? gb[0] : 0) + k0t : 0) * (IN64 ? 16 : 8);

  u32x4 opr[OPCH];  // prefetched operator chunks
  cf vin[FI][KJ];   // prefetched state values

  auto load_stage = [&](int ks) {
    const u32x4* src = opblk + static_cast<size_t>(ks) * (6 * CPS);
#pragma unroll
    for (int j = 0; j < OPCH; ++j) opr[j] = src[tid + 256 * j];
    if (CONTIG && full) {
      const char* q = inp + static_cast<size_t>(ks) * KS * (IN64 ? 16 : 8);
#pragma unroll
      for (int j = 0; j < KJ; j += 2) {
        if (IN64) {
          const double2 x = reinterpret_cast<const double2*>(q)[j];
          const double2 y = reinterpret_cast<const double2*>(q)[j + 1];
          vin[0][j] = cf{static_cast<float>(x.x), static_cast<float>(x.y)};
          vin[0][j + 1] = cf{static_cast<float>(y.x), static_cast<float>(y.y)};
        } else {
          const f32x4u v = reinterpret_cast<const f32x4u*>(q)[j / 2];
          vin[0][j] = cf{v[0], v[1]};
          vin[0][j + 1] = cf{v[2], v[3]};
        }
      }
      return;
    }
    const int kb = ks * KS + k0t;
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
      for (int j = 0; j < KJ; ++j) vin[i][j] = cf{0.0f, 0.0f};
    if (CONTIG) {
      if (gb[0] >= 0) {
#pragma unroll
        for (int j = 0; j < KJ; ++j)
          if (kb + j < a.n) vin[0][j] = load_cf(a.in0, gb[0] + kb + j, IN64);
      }
    } else {
#pragma unroll
      for (int j = 0; j < KJ; ++j) {
        const int k = kb + j;
        if (k >= a.n) continue;
        if (pairF) {
          load_cf2(a.in0, gb[0] + a.R * (int64_t)k, IN64, vin[0][j], vin[FI - 1][j]);
        } else {
#pragma unroll
          for (int i = 0; i < FI; ++i)
            if (gb[i] >= 0) vin[i][j] = load_cf(a.in0, gb[i] + a.R * (int64_t)k, IN64);
        }
      }
    }
  };

  f32x16 accr[PB], acci[PB];
#pragma unroll
  for (int b = 0; b < PB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accr[b][r] = 0.0f;
      acci[b][r] = 0.0f;
    }
  unsigned flag = 0;
  const int row = lane & 31;
  const int kh = (lane >> 5) * 8;

  load_stage(0);
  for (int ks = 0; ks < nKS; ++ks) {
    // ---- registers -> LDS: operator planes as they are; state through the
    // prologue and split into bf16 terms
#pragma unroll
    for (int j = 0; j < OPCH; ++j) {
      const int c = tid + 256 * j;
      *reinterpret_cast<u32x4*>(&sA[c / CPS][c % PT][8 * ((c / PT) % (KS / 8))]) = opr[j];
    }
#pragma unroll
    for (int i = 0; i < FI; ++i) {
      if (PRO == PRO_FLOW) {
#pragma unroll
        for (int j = 0; j < KJ; ++j) vin[i][j] = flow_in_f(vin[i][j], a.nl, flag);
      } else if (PRO == PRO_G) {
#pragma unroll
        for (int j = 0; j < KJ; ++j) vin[i][j] = g_cgl_f(vin[i][j], a.nl);
      }
      unsigned tr[3][KJ / 2], ti[3][KJ / 2];
#pragma unroll
      for (int j = 0; j < KJ; j += 2) {
        unsigned t3[3];
        split3x2(vin[i][j].re, vin[i][j + 1].re, t3);
#pragma unroll
        for (int t = 0; t < 3; ++t) tr[t][j / 2] = t3[t];
        split3x2(vin[i][j].im, vin[i][j + 1].im, t3);
#pragma unroll
        for (int t = 0; t < 3; ++t) ti[t][j / 2] = t3[t];
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        store_terms<KJ>(&sB[t][fl[i]][k0t], tr[t]);
        store_terms<KJ>(&sB[3 + t][fl[i]][k0t], ti[t]);
      }
    }
    __syncthreads();
    if (ks + 1 < nKS) load_stage(ks + 1);
    // ---- MFMA: 16-deep steps, 6 term products x 4 real products per block
#pragma unroll
    for (int kk = 0; kk < KS; kk += 16) {
      bf16x8 br[3], bi[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        br[t] = *reinterpret_cast<const bf16x8*>(&sB[t][wf * 32 + row][kk + kh]);
        bi[t] = *reinterpret_cast<const bf16x8*>(&sB[3 + t][wf * 32 + row][kk + kh]);
      }
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        bf16x8 ar[3], ai[3], an[3];
        const int prow = wp * (PT / 2) + b * 32 + row;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          ar[t] = *reinterpret_cast<const bf16x8*>(&sA[t][prow][kk + kh]);
          ai[t] = *reinterpret_cast<const bf16x8*>(&sA[3 + t][prow][kk + kh]);
          an[t] = neg8(ai[t]);
        }
        // term pairs (i, j) with i + j <= 2, smallest first
        constexpr int PI[6] = {2, 1, 0, 1, 0, 0};
        constexpr int PJ[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const int ti_ = PI[q], tj = PJ[q];
          accr[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ti_], br[tj], accr[b], 0, 0, 0);
          acci[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai[ti_], br[tj], acci[b], 0, 0, 0);
          accr[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(an[ti_], bi[tj], accr[b], 0, 0, 0);
          acci[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ti_], bi[tj], acci[b], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  static_assert(EPI_LDS_BYTES <= static_cast<int>(sizeof(Lds<PT, KS>)), "epilogue staging fits");
  split_epilogue<PT>(a, pt, f0, accr, acci, flag, &lds);
  if (flag) atomicOr(a.flag, flag);
}

// ---- Direct-to-LDS variant (contiguous contraction axis, 16-deep stages).
//
// The operator planes of a stage are stored in global memory as the exact
// image of their LDS tile, so they are copied with buffer loads that write
// LDS directly (no registers, no LDS store instructions).  Both the operator
// and the state tiles are double-buffered and unpadded; 16-byte chunks are
// XOR-swizzled by row (dma_chunk) so that the MFMA operand reads of
// consecutive lanes (consecutive rows, one chunk) fall on distinct banks.
// One barrier per stage: during stage ks the waves read their stage-ks
// fragments, start the copy of the operator of stage ks + 1 into the other
// buffer, issue the state loads of stage ks + 2, run the MFMAs, and split the
// state of stage ks + 1 into the other state buffer.
template <int PT, int KS>
struct LdsD {
  unsigned short A[2][6 * PT * KS];
  unsigned short B[2][6 * FT * KS];
};

// Stages [k0, k1) of the contraction (k1 < 0: every stage).  part == nullptr:
// the epilogue stores the tile; otherwise the raw FP32 accumulators go to
// part (the tile's slot of a split contraction, reduced by k_split_reduce).
template <int PT, int KS, int PRO, bool IN64>
__device__ __forceinline__ void split_tile_dma(const PassSplit& a, int pt, int64_t f0,
                                               LdsD<PT, KS>& lds, int k0 = 0, int k1 = -1,
                                               float* part = nullptr) {
  static_assert(KS == 16, "one 16-deep MFMA step per stage");
  constexpr int KJ = KS / 4;               // state elements per thread and stage
  constexpr int PB = PT / 64;              // 32-row blocks per wave
  constexpr int ABYTES = 12 * PT * KS;     // operator image of one stage
  constexpr int NDMA = ABYTES / 4096;      // 1 KB copies per wave and stage
  static_assert(NDMA * 4096 == ABYTES, "operator stage must split evenly");
  constexpr int ESZ = IN64 ? 16 : 8;
  constexpr int NV = IN64 ? KJ : KJ / 2;   // buffer loads of one stage's state
  constexpr unsigned OOR = 0x80000000u;    // out of range of both buffers

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wp = wave & 1;
  const int wf = wave >> 1;
  const int nKS = uniform_i32(a.Kp / KS);
  const int kend = k1 < 0 ? nKS : k1;  // stages past kend read out of range (zero)
  const __amdgpu_buffer_rsrc_t ors = __builtin_amdgcn_make_buffer_rsrc(
      uniform_ptr(const_cast<uint16_t*>(a.op + static_cast<size_t>(pt) * nKS * (6 * PT * KS))),
      0, nKS * ABYTES, 0x00020000);
  // state: 8 consecutive lanes take 8 fibres at one index chunk; the buffer
  // range ends at the end of the tensor (fibres past F read zero)
  const int fl = (tid & 7) + 8 * (tid >> 5);
  const int k0t = KJ * ((tid >> 3) & 3);
  const int64_t srem = (a.F - f0) * static_cast<int64_t>(a.n) * ESZ;
  const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
      uniform_ptr(const_cast<char*>(reinterpret_cast<const char*>(a.in0) +
                                    f0 * static_cast<int64_t>(a.n) * ESZ)),
      0, uniform_i32(static_cast<int>(srem < 0x7fffffffll ? srem : 0x7fffffffll)), 0x00020000);
  const unsigned svo = static_cast<unsigned>((fl * a.n + k0t) * ESZ);

  auto copy_op = [&](int ks, int buf) __attribute__((always_inline)) {
    const unsigned o = ks < kend ? static_cast<unsigned>(ks * ABYTES) : OOR;
#pragma unroll
    for (int j = 0; j < NDMA; ++j) {
      const int blk = wave + 4 * j;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          ors, (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(lds.A[buf]) + blk * 1024),
          16, o + static_cast<unsigned>(blk * 1024 + lane * 16), 0, 0, 0);
    }
  };
  auto load_state = [&](int ks, f32x4 (&v)[KJ / 2]) __attribute__((always_inline)) {
    const unsigned o = ks < kend ? svo + static_cast<unsigned>(ks * KS * ESZ) : OOR;
#pragma unroll
    for (int j = 0; j < KJ; j += 2) {
      if constexpr (IN64) {
        const double2 x = __builtin_bit_cast(
            double2, __builtin_amdgcn_raw_buffer_load_b128(srs, o + j * 16, 0, 0));
        const double2 y = __builtin_bit_cast(
            double2, __builtin_amdgcn_raw_buffer_load_b128(srs, o + j * 16 + 16, 0, 0));
        v[j / 2] = f32x4{static_cast<float>(x.x), static_cast<float>(x.y),
                         static_cast<float>(y.x), static_cast<float>(y.y)};
      } else {
        v[j / 2] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(srs, o + j * 8, 0, 0));
      }
    }
  };
  unsigned flag = 0;
  // prologue flow, bf16 split and store of the state of stage ks (indices
  // k >= n, read from the next fibre, become zero)
  auto store_state = [&](int ks, const f32x4 (&v)[KJ / 2], int buf) __attribute__((always_inline)) {
    cf w[KJ];
#pragma unroll
    for (int j = 0; j < KJ; ++j) {
      w[j] = cf{v[j / 2][2 * (j % 2)], v[j / 2][2 * (j % 2) + 1]};
      if (ks * KS + k0t + j >= a.n) w[j] = cf{0.0f, 0.0f};
      if (PRO == PRO_FLOW) w[j] = flow_in_f(w[j], a.nl, flag);
      else if (PRO == PRO_G) w[j] = g_cgl_f(w[j], a.nl);
    }
    unsigned tr[3][KJ / 2], ti[3][KJ / 2];
#pragma unroll
    for (int j = 0; j < KJ; j += 2) {
      unsigned t3[3];
      split3x2(w[j].re, w[j + 1].re, t3);
#pragma unroll
      for (int t = 0; t < 3; ++t) tr[t][j / 2] = t3[t];
      split3x2(w[j].im, w[j + 1].im, t3);
#pragma unroll
      for (int t = 0; t < 3; ++t) ti[t][j / 2] = t3[t];
    }
    const int off = fl * KS + dma_chunk(fl, k0t / 8) * 8 + k0t % 8;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      store_terms<KJ>(&lds.B[buf][t * FT * KS + off], tr[t]);
      store_terms<KJ>(&lds.B[buf][(3 + t) * FT * KS + off], ti[t]);
    }
  };

  f32x16 accr[PB], acci[PB];
#pragma unroll
  for (int b = 0; b < PB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accr[b][r] = 0.0f;
      acci[b][r] = 0.0f;
    }
  const int row = lane & 31;
  const int ch = lane >> 5;  // chunk of the 16-deep step this lane supplies

  // stage ks: fragments of buffer (ks - k0) % 2, copies into the other buffer
  auto stage = [&](int ks, f32x4 (&vload)[KJ / 2], const f32x4 (&vstore)[KJ / 2])
      __attribute__((always_inline)) {
    const int cur = (ks - k0) & 1;
    bf16x8 br[3], bi[3], ar[PB][3], ai[PB][3];
    {
      const int rb = wf * 32 + row;
      const int o = rb * KS + dma_chunk(rb, ch) * 8;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        br[t] = *reinterpret_cast<const bf16x8*>(&lds.B[cur][t * FT * KS + o]);
        bi[t] = *reinterpret_cast<const bf16x8*>(&lds.B[cur][(3 + t) * FT * KS + o]);
      }
    }
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      const int ra = wp * (PT / 2) + b * 32 + row;
      const int o = ra * KS + dma_chunk(ra, ch) * 8;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        ar[b][t] = *reinterpret_cast<const bf16x8*>(&lds.A[cur][t * PT * KS + o]);
        ai[b][t] = *reinterpret_cast<const bf16x8*>(&lds.A[cur][(3 + t) * PT * KS + o]);
      }
    }
    // the copies and loads go out before the MFMAs (the scheduler would sink
    // them behind the math), the copies first: the barrier at the end of the
    // stage waits for them, the state loads get two stages to arrive
    copy_op(ks + 1, cur ^ 1);
    __builtin_amdgcn_sched_barrier(0);
    load_state(ks + 2, vload);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      bf16x8 an[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) an[t] = neg8(ai[b][t]);
      constexpr int PI[6] = {2, 1, 0, 1, 0, 0};
      constexpr int PJ[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int ti_ = PI[q], tj = PJ[q];
        accr[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[b][ti_], br[tj], accr[b], 0, 0, 0);
        acci[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai[b][ti_], br[tj], acci[b], 0, 0, 0);
        accr[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(an[ti_], bi[tj], accr[b], 0, 0, 0);
        acci[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[b][ti_], bi[tj], acci[b], 0, 0, 0);
      }
    }
    store_state(ks + 1, vstore, cur ^ 1);
    stage_barrier<NV>();
  };

  f32x4 sv[2][KJ / 2];
  copy_op(k0, 0);
  load_state(k0, sv[0]);
  load_state(k0 + 1, sv[1]);
  store_state(k0, sv[0], 0);
  stage_barrier<NV>();
  int ks = k0;
  for (; ks + 1 < kend; ks += 2) {
    stage(ks, sv[0], sv[1]);
    stage(ks + 1, sv[1], sv[0]);
  }
  if (ks < kend) stage(ks, sv[0], sv[1]);
  // the copies issued by the last stage (out of range: zeros) still write
  // the other operator buffer, which the epilogue reuses
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  __syncthreads();
  if (part) {
    // raw accumulators, lane-interleaved: entry (b, r) of thread tid at
    // part[((b * 32 + r) * 256) + tid] (r < 16 real, 16 + r imaginary)
#pragma unroll
    for (int b = 0; b < PB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        part[(b * 32 + r) * 256 + tid] = accr[b][r];
        part[(b * 32 + 16 + r) * 256 + tid] = acci[b][r];
      }
  } else {
    static_assert(EPI_LDS_BYTES <= static_cast<int>(sizeof(LdsD<PT, KS>)), "epilogue staging fits");
    split_epilogue<PT>(a, pt, f0, accr, acci, flag, &lds);
  }
  if (flag) atomicOr(a.flag, flag);
}

template <int PT, int KS, bool CONTIG, int PRO, bool IN64>
__global__ __launch_bounds__(256, 2) void k_pass_split(PassSplit a) {
  __shared__ __attribute__((aligned(16))) Lds<PT, KS> lds;
  const int nP = a.Pp / PT;
  const unsigned w = xcd_remap(blockIdx.x, gridDim.x);
  split_tile<PT, KS, CONTIG, PRO, IN64>(a, static_cast<int>(w % nP),
                                       static_cast<int64_t>(w / nP) * FT, lds);
}

// ---- Paired pass: one direction of the two exponential actions of a
// Lawson round in one launch.  A workgroup applies its operator tile to the
// tiles of both inputs (in0 for the first action, in1 for the second, or, in
// the first pass of the first round, in0 and g(in0)), so each operator stage
// is copied to LDS once for two products, and the round's stage combination
// runs in the epilogue with both results at hand (no auxiliary tensor, no
// cross-stream join).  PT rows x 64 fibres, 16-deep stages, direct-to-LDS
// operator copies as above; two accumulator sets per wave, each wave 32 rows
// x 32 fibres.  Two shapes: PT = 64 (4 waves, two workgroups per CU) and
// PT = 128 (8 waves, one workgroup per CU: the state tile of a stage is
// split into bf16 terms once for twice the rows).
template <int PT, int KS>
struct LdsP {
  unsigned short A[2][6 * PT * KS];
  unsigned short B[2][2][6 * FT * KS];
};

template <int PT>
struct PairGeom {
  static constexpr int NW = PT / 16;          // waves
  static constexpr int NT = NW * 64;          // threads
  static constexpr int RB = PT / 32;          // 32-row blocks (waves along the rows)
  static constexpr int TPT = NT == 256 ? 2 : 1;  // state tensors a thread stages
  static_assert(PT == 64 || PT == 128, "paired tile shapes");
};

// Epilogue of a paired tile: y0, y1 the two results of a point, both held
// by the same lane (the two accumulator sets have one layout).  EPI_NONE:
// out0 = y0, out1 = y1.  EPI_L4_R1: (P, Q) = (y0, y1) -> out0 = X, out1 = Y.
// EPI_L4_R2: (HX, HY) = (y0, y1) -> out0 = u_{n+1}.  EPI_L2: (P, Q) =
// (E u, E g(u)) -> out0 = u_{n+1} of Lawson2b.  Every kind stores
// straight from the accumulators: lanes 0..31 of a row take 32 consecutive
// fibres, which are adjacent in the output (R_out = F).
template <int PT>
__device__ __forceinline__ void pair_epilogue(const PassSplit& a, int pt, int64_t f0,
                                              f32x16 (&accr)[2], f32x16 (&acci)[2],
                                              unsigned& flag) {
  using G = PairGeom<PT>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wp = wave % G::RB;
  const int wf = wave / G::RB;
  const bool of64 = a.out_f64 != 0;
  const int64_t f = f0 + wf * 32 + (lane & 31);
  if (f >= a.F) return;
  // accumulator entry r holds row m1 + dm(r); its output element is o0 + R_out dm(r)
  const int m1 = pt * PT + wp * 32 + 4 * (lane >> 5);
  const int64_t Ro = a.R_out;
  const int64_t o0 = fibre_start(f, a.R_out, a.n, a.F) + Ro * m1;
  const bool full = pt * PT + PT <= a.n;  // uniform: the tile has no rows past n
  auto each = [&](auto&& fn) __attribute__((always_inline)) {
    if (full) {
#pragma unroll
      for (int r = 0; r < 16; ++r) fn(r, Ro * (8 * (r >> 2) + (r & 3)));
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (m1 + 8 * (r >> 2) + (r & 3) < a.n) fn(r, Ro * (8 * (r >> 2) + (r & 3)));
    }
  };
  if (a.epi == EPI_NONE) {
    float2* q0 = reinterpret_cast<float2*>(a.out0) + o0;
    float2* q1 = reinterpret_cast<float2*>(a.out1) + o0;
    each([&](int r, int64_t d) __attribute__((always_inline)) {
      q0[d] = float2{accr[0][r], acci[0][r]};
      q1[d] = float2{accr[1][r], acci[1][r]};
    });
  } else if (a.epi == EPI_L4_R1) {
    float2* q0 = reinterpret_cast<float2*>(a.out0) + o0;
    float2* q1 = reinterpret_cast<float2*>(a.out1) + o0;
    const L4Coef c = lawson_coef(a.nl.tau);
    each([&](int r, int64_t d) __attribute__((always_inline)) {
      const cd P = {static_cast<double>(accr[0][r]), static_cast<double>(acci[0][r])};
      const cd Q = {static_cast<double>(accr[1][r]), static_cast<double>(acci[1][r])};
      cd X, Y;
      lawson_r1(P, Q, a.nl, c, X, Y);
      q0[d] = float2{static_cast<float>(X.re), static_cast<float>(X.im)};
      q1[d] = float2{static_cast<float>(Y.re), static_cast<float>(Y.im)};
    });
  } else if (a.epi == EPI_L4_R2) {
    void* q0 = of64 ? static_cast<void*>(reinterpret_cast<double2*>(a.out0) + o0)
                    : static_cast<void*>(reinterpret_cast<float2*>(a.out0) + o0);
    const double t6 = a.nl.tau / 6.0;
    each([&](int r, int64_t d) __attribute__((always_inline)) {
      const cd HX = {static_cast<double>(accr[0][r]), static_cast<double>(acci[0][r])};
      const cd HY = {static_cast<double>(accr[1][r]), static_cast<double>(acci[1][r])};
      const cd z = lawson_r2(HX, HY, a.nl, t6);
      if (!finite2(z)) flag |= FLAG_NONFINITE;
      store_c(q0, d, of64, z);
    });
  } else {  // EPI_L2
    void* q0 = of64 ? static_cast<void*>(reinterpret_cast<double2*>(a.out0) + o0)
                    : static_cast<void*>(reinterpret_cast<float2*>(a.out0) + o0);
    const double h = 0.5 * a.nl.tau;
    each([&](int r, int64_t d) __attribute__((always_inline)) {
      const cd P = {static_cast<double>(accr[0][r]), static_cast<double>(acci[0][r])};
      const cd Q = {static_cast<double>(accr[1][r]), static_cast<double>(acci[1][r])};
      const cd z = lawson2(P, Q, a.nl, h);
      if (!finite2(z)) flag |= FLAG_NONFINITE;
      store_c(q0, d, of64, z);
    });
  }
}

// One work item of the paired pass (a row tile x fibre tile of one
// direction).  SAMEG: both products read in0; the second applies g first
// (P = H u and Q = H g(u)).  Otherwise the inputs are in0 and in1
// (complex64).  Staging of a stage's state tile (64 fibres x 16 indices of
// both tensors): with 4 waves every thread stages its 4 indices of one fibre
// of both tensors; with 8 waves threads 0..255 stage the first tensor and
// 256..511 the second.  prefetch() issues the item's first loads (operator
// stage 0 to LDS buffer 0, the state of stages 0 and 1 to registers); run()
// multiplies every stage and returns with both LDS buffers free (the last
// copies landed, every wave past its last read), so a persistent workgroup
// can issue the next item's first loads before this item's epilogue.
// SKIP: a wave whose 32 x 32 block lies wholly in the padding skips its
// products (the batched pass, whose small grids pad often; on the large
// grids of a single-instance pass the branch costs more than it saves).
template <bool SAMEG, bool IN64, int PT, bool SKIP = false>
struct PairItem {
  using G = PairGeom<PT>;
  static constexpr int KS = 16;
  static constexpr int KJ = KS / 4;
  static constexpr int ABYTES = 12 * PT * KS;
  static constexpr int NDMA = ABYTES / (G::NW * 1024);  // 1 KB copies per wave and stage
  static_assert(NDMA * G::NW * 1024 == ABYTES, "operator stage must split evenly");
  static constexpr int ESZ = IN64 ? 16 : 8;
  // state tensors this thread loads: both inputs (or u once) with 4 waves,
  // its own tensor's input with 8
  static constexpr int NL = G::TPT == 2 ? (SAMEG ? 1 : 2) : 1;
  static constexpr unsigned OOR = 0x80000000u;
  static_assert(!IN64 || SAMEG, "a complex128 input occurs only in the first pass");
  using SV = f32x4[NL][KJ / 2];
  using Lds = LdsP<PT, 16>;

  PassSplit a;
  int pt;
  int64_t f0;
  int nKS;
  __amdgpu_buffer_rsrc_t ors;
  __amdgpu_buffer_rsrc_t srs[NL];
  unsigned svo;
  int fl, k0t, ts0;
  bool live;  // this wave's 32 x 32 block has a row below n and a fibre below F

  __device__ __forceinline__ PairItem(const PassSplit& a_, int pt_, int64_t f0_)
      : a(a_), pt(pt_), f0(f0_) {
    const int tid = threadIdx.x;
    {
      const int wave = tid >> 6;
      live = pt * PT + (wave % G::RB) * 32 < a.n && f0 + (wave / G::RB) * 32 < a.F;
    }
    nKS = uniform_i32(a.Kp / KS);
    ors = __builtin_amdgcn_make_buffer_rsrc(
        uniform_ptr(const_cast<uint16_t*>(a.op + static_cast<size_t>(pt) * nKS * (6 * PT * KS))),
        0, nKS * ABYTES, 0x00020000);
    const int sid = tid & 255;                 // position within a 256-thread staging group
    // first tensor this thread stages; wave-uniform, and read from the first
    // lane so that the state buffer resource it selects stays scalar (a
    // per-lane resource makes every state load a waterfall loop)
    ts0 = G::TPT == 2 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 8);
    fl = (sid & 7) + 8 * (sid >> 5);
    k0t = KJ * ((sid >> 3) & 3);
    const int64_t srem = (a.F - f0) * static_cast<int64_t>(a.n) * ESZ;
    const int rnum = uniform_i32(static_cast<int>(srem < 0x7fffffffll ? srem : 0x7fffffffll));
    const int64_t tile0 = f0 * static_cast<int64_t>(a.n) * ESZ;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      // load i reads in1 for the second tensor of a pair of distinct inputs
      const bool second = !SAMEG && (G::TPT == 2 ? i == 1 : ts0 == 1);
      srs[i] = __builtin_amdgcn_make_buffer_rsrc(
          uniform_ptr(const_cast<char*>(reinterpret_cast<const char*>(second ? a.in1 : a.in0) + tile0)),
          0, rnum, 0x00020000);
    }
    svo = static_cast<unsigned>((fl * a.n + k0t) * ESZ);
  }

  __device__ __forceinline__ void copy_op(int ks, int buf, Lds& lds) const {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const unsigned o = ks < nKS ? static_cast<unsigned>(ks * ABYTES) : OOR;
#pragma unroll
    for (int j = 0; j < NDMA; ++j) {
      const int blk = wave + G::NW * j;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          ors, (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(lds.A[buf]) + blk * 1024),
          16, o + static_cast<unsigned>(blk * 1024 + lane * 16), 0, 0, 0);
    }
  }

  __device__ __forceinline__ void load_state(int ks, SV& v) const {
    const unsigned o = ks < nKS ? svo + static_cast<unsigned>(ks * KS * ESZ) : OOR;
#pragma unroll
    for (int i = 0; i < NL; ++i)
#pragma unroll
      for (int j = 0; j < KJ; j += 2) {
        if constexpr (IN64) {
          const double2 x = __builtin_bit_cast(
              double2, __builtin_amdgcn_raw_buffer_load_b128(srs[i], o + j * 16, 0, 0));
          const double2 y = __builtin_bit_cast(
              double2, __builtin_amdgcn_raw_buffer_load_b128(srs[i], o + j * 16 + 16, 0, 0));
          v[i][j / 2] = f32x4{static_cast<float>(x.x), static_cast<float>(x.y),
                              static_cast<float>(y.x), static_cast<float>(y.y)};
        } else {
          v[i][j / 2] =
              __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(srs[i], o + j * 8, 0, 0));
        }
      }
  }

  __device__ __forceinline__ void store_state(int ks, const SV& v, int buf, Lds& lds) const {
    const int off = fl * KS + dma_chunk(fl, k0t / 8) * 8 + k0t % 8;
#pragma unroll
    for (int t = 0; t < G::TPT; ++t) {
      const int tt = ts0 + t;                             // tensor staged
      const int li = G::TPT == 2 ? (SAMEG ? 0 : t) : 0;   // its load
      cf w[KJ];
#pragma unroll
      for (int j = 0; j < KJ; ++j) {
        w[j] = cf{v[li][j / 2][2 * (j % 2)], v[li][j / 2][2 * (j % 2) + 1]};
        if (ks * KS + k0t + j >= a.n) w[j] = cf{0.0f, 0.0f};
        if (SAMEG && tt == 1) w[j] = g_cgl_f(w[j], a.nl);
      }
      unsigned tr[3][KJ / 2], ti[3][KJ / 2];
#pragma unroll
      for (int j = 0; j < KJ; j += 2) {
        unsigned t3[3];
        split3x2(w[j].re, w[j + 1].re, t3);
#pragma unroll
        for (int q = 0; q < 3; ++q) tr[q][j / 2] = t3[q];
        split3x2(w[j].im, w[j + 1].im, t3);
#pragma unroll
        for (int q = 0; q < 3; ++q) ti[q][j / 2] = t3[q];
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        store_terms<KJ>(&lds.B[buf][tt][q * FT * KS + off], tr[q]);
        store_terms<KJ>(&lds.B[buf][tt][(3 + q) * FT * KS + off], ti[q]);
      }
    }
  }

  __device__ __forceinline__ void stage(int ks, SV& vload, const SV& vstore, f32x16 (&accr)[2],
                                        f32x16 (&acci)[2], Lds& lds) const {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wp = wave % G::RB;
    const int wf = wave / G::RB;
    const int row = lane & 31;
    const int ch = lane >> 5;
    const int cur = ks & 1;
    bf16x8 br[2][3], bi[2][3], ar[3], ai[3];
    {
      const int rb = wf * 32 + row;
      const int o = rb * KS + dma_chunk(rb, ch) * 8;
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          br[t][q] = *reinterpret_cast<const bf16x8*>(&lds.B[cur][t][q * FT * KS + o]);
          bi[t][q] = *reinterpret_cast<const bf16x8*>(&lds.B[cur][t][(3 + q) * FT * KS + o]);
        }
    }
    {
      const int ra = wp * 32 + row;
      const int o = ra * KS + dma_chunk(ra, ch) * 8;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        ar[q] = *reinterpret_cast<const bf16x8*>(&lds.A[cur][q * PT * KS + o]);
        ai[q] = *reinterpret_cast<const bf16x8*>(&lds.A[cur][(3 + q) * PT * KS + o]);
      }
    }
    load_state(ks + 2, vload);
    copy_op(ks + 1, cur ^ 1, lds);
    __builtin_amdgcn_sched_barrier(0);
    // a wave whose block lies wholly in the padding (rows past n or fibres
    // past F) skips its products: the matrix cores go to the other waves
    if (!SKIP || live) {
      bf16x8 an[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) an[q] = neg8(ai[q]);
      constexpr int PI[6] = {2, 1, 0, 1, 0, 0};
      constexpr int PJ[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const int ti_ = PI[q], tj = PJ[q];
          accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ti_], br[t][tj], accr[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai[ti_], br[t][tj], acci[t], 0, 0, 0);
          accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(an[ti_], bi[t][tj], accr[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ti_], bi[t][tj], acci[t], 0, 0, 0);
        }
    }
    store_state(ks + 1, vstore, cur ^ 1, lds);
    __syncthreads();
  }

  __device__ __forceinline__ void prefetch(SV (&sv)[2], Lds& lds) const {
    copy_op(0, 0, lds);
    load_state(0, sv[0]);
    load_state(1, sv[1]);
  }

  __device__ __forceinline__ void run(SV (&sv)[2], f32x16 (&accr)[2], f32x16 (&acci)[2],
                                      Lds& lds) const {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        accr[t][r] = 0.0f;
        acci[t][r] = 0.0f;
      }
    store_state(0, sv[0], 0, lds);
    __syncthreads();
    int ks = 0;
    for (; ks + 1 < nKS; ks += 2) {
      stage(ks, sv[0], sv[1], accr, acci, lds);
      stage(ks + 1, sv[1], sv[0], accr, acci, lds);
    }
    if (ks < nKS) stage(ks, sv[0], sv[1], accr, acci, lds);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the last copies write the other buffer
    __syncthreads();
  }
};

template <bool SAMEG, bool IN64, int PT, bool SKIP = false>
__device__ __forceinline__ void split_tile_pair(const PassSplit& a, int pt, int64_t f0,
                                                LdsP<PT, 16>& lds) {
  using It = PairItem<SAMEG, IN64, PT, SKIP>;
  const It it(a, pt, f0);
  typename It::SV sv[2];
  it.prefetch(sv, lds);
  f32x16 accr[2], acci[2];
  it.run(sv, accr, acci, lds);
  unsigned flag = 0;
  pair_epilogue<PT>(a, pt, f0, accr, acci, flag);
  if (flag) atomicOr(a.flag, flag);
}

template <bool SAMEG, bool IN64, int PT>
__global__ __launch_bounds__(PT * 4, PT == 64 ? 2 : 1) void k_pass_split_pair(PassSplit a) {
  __shared__ __attribute__((aligned(16))) LdsP<PT, 16> lds;
  const int nP = a.Pp / PT;
  const unsigned w = xcd_remap(blockIdx.x, gridDim.x);
  split_tile_pair<SAMEG, IN64, PT>(a, static_cast<int>(w % nP), static_cast<int64_t>(w / nP) * FT,
                                   lds);
}

template <int PT, int KS, int PRO, bool IN64>
__global__ __launch_bounds__(256, 2) void k_pass_split_dma(PassSplit a) {
  __shared__ __attribute__((aligned(16))) LdsD<PT, KS> lds;
  const int nP = a.Pp / PT;
  const unsigned w = xcd_remap(blockIdx.x, gridDim.x);
  split_tile_dma<PT, KS, PRO, IN64>(a, static_cast<int>(w % nP), static_cast<int64_t>(w / nP) * FT,
                                    lds);
}

// Split contraction (small passes: too few tiles to fill the chip).  The
// grid is S x G tiles; the workgroup of split s takes stages
// [s * a.kchunk, (s + 1) * a.kchunk) of its tile and writes its raw
// accumulators to the workspace slot (s * G + tile); k_split_reduce sums the
// S slots of a tile in split order and runs the epilogue.
template <int PT, int KS, int PRO, bool IN64>
__global__ __launch_bounds__(256, 2) void k_pass_split_dma_part(PassSplit a) {
  __shared__ __attribute__((aligned(16))) LdsD<PT, KS> lds;
  constexpr int SLOT = (PT / 64) * 32 * 256;  // floats per tile slot
  const int nP = a.Pp / PT;
  const unsigned G = gridDim.x / static_cast<unsigned>(a.ksplit);
  const unsigned h = xcd_remap(blockIdx.x, gridDim.x);
  const unsigned sp = h / G, w = h % G;
  const int k0 = static_cast<int>(sp) * a.kchunk;
  const int k1 = k0 + a.kchunk < a.Kp / KS ? k0 + a.kchunk : a.Kp / KS;
  split_tile_dma<PT, KS, PRO, IN64>(a, static_cast<int>(w % nP), static_cast<int64_t>(w / nP) * FT,
                                    lds, k0, k1, a.ws + (static_cast<size_t>(sp) * G + w) * SLOT);
}

template <int PT>
__global__ __launch_bounds__(256, 2) void k_split_reduce(PassSplit a) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[EPI_LDS_BYTES];
  constexpr int PB = PT / 64;
  constexpr int SLOT = PB * 32 * 256;
  const int nP = a.Pp / PT;
  const unsigned G = gridDim.x, w = blockIdx.x;
  const int tid = threadIdx.x;
  f32x16 accr[PB], acci[PB];
#pragma unroll
  for (int b = 0; b < PB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accr[b][r] = 0.0f;
      acci[b][r] = 0.0f;
    }
  // per 32-row block, the loads of every split (at most 4) are issued
  // before the first sum; the sums run in split order
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    float v[4][32];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
#pragma unroll
      for (int r = 0; r < 32; ++r) v[sp][r] = 0.0f;
      if (sp < a.ksplit) {
        const float* q = a.ws + (static_cast<size_t>(sp) * G + w) * SLOT + b * 32 * 256 + tid;
#pragma unroll
        for (int r = 0; r < 32; ++r) v[sp][r] = q[r * 256];
      }
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        accr[b][r] += v[sp][r];
        acci[b][r] += v[sp][16 + r];
      }
  }
  unsigned flag = 0;
  split_epilogue<PT>(a, static_cast<int>(w % nP), static_cast<int64_t>(w / nP) * FT, accr, acci,
                     flag, lds);
  if (flag) atomicOr(a.flag, flag);
}

// Batched form: a persistent grid walks a table of (instance, p-tile, fibre
// tile) entries; each instance has its own grid size, coefficients and
// operator planes, and lives at its own offset in every batched tensor.
template <int PT, int KS, int PRO, bool IN64, bool DMA>
__global__ __launch_bounds__(256, 2) void k_pass_split_batched(PassBatch b) {
  // DMA: the direct-to-LDS tile (operator planes in the LDS-image layout)
  __shared__ __attribute__((aligned(16))) std::conditional_t<DMA, LdsD<PT, KS>, Lds<PT, KS>> lds;
  for (int t = blockIdx.x; t < b.ntiles; t += gridDim.x) {
    const BatchTile tl = b.tiles[t];
    if (tl.inst < 0) continue;  // padding entry of the table
    const BatchInstance& in = b.inst[tl.inst];
    PassSplit a{};
    const size_t esz_in = IN64 ? 16 : 8, esz_out = b.out_f64 ? 16 : 8;
    a.in0 = static_cast<const char*>(b.in0) + in.off * esz_in;
    a.aux = b.aux ? static_cast<const char*>(b.aux) + in.off * 8 : nullptr;
    a.out0 = static_cast<char*>(b.out0) + in.off * esz_out;
    a.out1 = b.out1 ? static_cast<char*>(b.out1) + in.off * esz_out : nullptr;
    a.op = b.which == 0 ? in.opE[b.tile] : in.opH[b.tile];
    a.R = 1;
    a.R_out = in.F;
    a.F = in.F;
    a.n = in.n;
    a.Pp = in.Pp[b.tile];
    a.Kp = in.Kp[b.tile];
    a.pro = PRO;
    a.epi = b.epi;
    a.in_f64 = IN64 ? 1 : 0;
    a.out_f64 = b.out_f64;
    a.aux_f64 = b.aux_f64;
    a.tile = b.tile;
    a.nl = in.nl;
    a.nl.tf = b.tf;
    a.flag = b.flag;
    if constexpr (DMA)
      split_tile_dma<PT, KS, PRO, IN64>(a, tl.pt, static_cast<int64_t>(tl.ft) * FT, lds);
    else
      split_tile<PT, KS, true, PRO, IN64>(a, tl.pt, static_cast<int64_t>(tl.ft) * FT, lds);
  }
}

// The pass arguments of one work item of a batched paired pass.
template <bool SAMEG, bool IN64>
__device__ __forceinline__ PassSplit batch_pair_item(const PassBatch& b, const BatchTile& tl) {
  const BatchInstance& in = b.inst[tl.inst];
  PassSplit a{};
  const size_t esz_in = IN64 ? 16 : 8, esz_out = b.out_f64 ? 16 : 8;
  a.in0 = static_cast<const char*>(b.in0) + in.off * esz_in;
  a.in1 = b.in1 ? static_cast<const char*>(b.in1) + in.off * 8 : nullptr;
  a.out0 = static_cast<char*>(b.out0) + in.off * esz_out;
  a.out1 = b.out1 ? static_cast<char*>(b.out1) + in.off * 8 : nullptr;
  a.op = b.which == 0 ? in.opE[b.tile] : in.opH[b.tile];
  a.R = 1;
  a.R_out = in.F;
  a.F = in.F;
  a.n = in.n;
  a.Pp = in.Pp[b.tile];
  a.Kp = in.Kp[b.tile];
  a.pro = SAMEG ? PRO_G : PRO_NONE;
  a.epi = b.epi;
  a.in_f64 = IN64 ? 1 : 0;
  a.out_f64 = b.out_f64;
  a.tile = b.tile;
  a.nl = in.nl;
  a.nl.tf = b.tf;
  a.flag = b.flag;
  return a;
}

// the next entry of the table this workgroup walks (entries t, t + G, ...),
// skipping padding; b.ntiles when there is none
__device__ __forceinline__ int next_batch_item(const PassBatch& b, int t) {
  while (t < b.ntiles && b.tiles[t].inst < 0) t += gridDim.x;
  return t;
}

// Paired pass over every instance of a batched plan (persistent grid).  The
// items are short (4-12 stages at the sweep's sizes), so with 64-row tiles
// the next item's first loads are issued before the current item's
// epilogue: its operator stage and state tiles are in flight while the
// epilogue computes and stores.  The first pass of a round (SAMEG) and the
// 128-row tile run their items one after the other: their registers would
// not hold both (the compiler spills).
template <bool SAMEG, bool IN64, int PT>
__global__ __launch_bounds__(PT * 4, PT == 64 ? 2 : 1) void k_pass_split_batched_pair(PassBatch b) {
  using It = PairItem<SAMEG, IN64, PT, true>;
  __shared__ __attribute__((aligned(16))) LdsP<PT, 16> lds;
  if constexpr (SAMEG || PT != 64) {
    for (int t = blockIdx.x; t < b.ntiles; t += gridDim.x) {
      const BatchTile tl = b.tiles[t];
      if (tl.inst < 0) continue;  // padding entry of the table
      split_tile_pair<SAMEG, IN64, PT, true>(batch_pair_item<SAMEG, IN64>(b, tl), tl.pt,
                                             static_cast<int64_t>(tl.ft) * FT, lds);
    }
  } else {
    int t = next_batch_item(b, blockIdx.x);
    if (t >= b.ntiles) return;
    BatchTile tl = b.tiles[t];
    It cur(batch_pair_item<SAMEG, IN64>(b, tl), tl.pt, static_cast<int64_t>(tl.ft) * FT);
    typename It::SV sv[2];
    cur.prefetch(sv, lds);
    for (;;) {
      f32x16 accr[2], acci[2];
      cur.run(sv, accr, acci, lds);
      // both LDS buffers are free: start the next item before this epilogue
      t = next_batch_item(b, t + gridDim.x);
      const bool more = t < b.ntiles;
      if (more) {
        tl = b.tiles[t];
        const It nxt(batch_pair_item<SAMEG, IN64>(b, tl), tl.pt, static_cast<int64_t>(tl.ft) * FT);
        nxt.prefetch(sv, lds);
        unsigned flag = 0;
        pair_epilogue<PT>(cur.a, cur.pt, cur.f0, accr, acci, flag);
        if (flag) atomicOr(cur.a.flag, flag);
        cur = nxt;
      } else {
        unsigned flag = 0;
        pair_epilogue<PT>(cur.a, cur.pt, cur.f0, accr, acci, flag);
        if (flag) atomicOr(cur.a.flag, flag);
        break;
      }
    }
  }
}

template <int PT, int KS, bool CONTIG, int PRO>
void launch_pro(const PassSplit& a, dim3 grid, hipStream_t s) {
  if (a.in_f64)
    hipLaunchKernelGGL((k_pass_split<PT, KS, CONTIG, PRO, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_pass_split<PT, KS, CONTIG, PRO, false>), grid, dim3(256), 0, s, a);
}

template <int PT, int KS, bool CONTIG>
void launch_contig(const PassSplit& a, dim3 grid, hipStream_t s) {
  if (a.pro == PRO_FLOW)
    launch_pro<PT, KS, CONTIG, PRO_FLOW>(a, grid, s);
  else if (a.pro == PRO_G)
    launch_pro<PT, KS, CONTIG, PRO_G>(a, grid, s);
  else
    launch_pro<PT, KS, CONTIG, PRO_NONE>(a, grid, s);
}

template <int PT, int KS>
void launch_tile(const PassSplit& a, dim3 grid, hipStream_t s) {
  if (a.R == 1)
    launch_contig<PT, KS, true>(a, grid, s);
  else
    launch_contig<PT, KS, false>(a, grid, s);
}

template <int PT, int KS, int PRO>
void launch_dma_pro(const PassSplit& a, dim3 grid, hipStream_t s) {
  if (a.in_f64)
    hipLaunchKernelGGL((k_pass_split_dma<PT, KS, PRO, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_pass_split_dma<PT, KS, PRO, false>), grid, dim3(256), 0, s, a);
}

template <int PT, int KS, int PRO>
void launch_dma_part_pro(const PassSplit& a, dim3 grid, hipStream_t s) {
  if (a.in_f64)
    hipLaunchKernelGGL((k_pass_split_dma_part<PT, KS, PRO, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_pass_split_dma_part<PT, KS, PRO, false>), grid, dim3(256), 0, s, a);
}

template <int PT, int KS>
void launch_tile_dma(const PassSplit& a, dim3 grid, hipStream_t s) {
  if (a.ksplit > 1) {  // split contraction: partial products, then the reduction
    const dim3 pgrid(grid.x * static_cast<unsigned>(a.ksplit));
    if (a.pro == PRO_FLOW)
      launch_dma_part_pro<PT, KS, PRO_FLOW>(a, pgrid, s);
    else if (a.pro == PRO_G)
      launch_dma_part_pro<PT, KS, PRO_G>(a, pgrid, s);
    else
      launch_dma_part_pro<PT, KS, PRO_NONE>(a, pgrid, s);
    hipLaunchKernelGGL((k_split_reduce<PT>), grid, dim3(256), 0, s, a);
    return;
  }
  if (a.pro == PRO_FLOW)
    launch_dma_pro<PT, KS, PRO_FLOW>(a, grid, s);
  else if (a.pro == PRO_G)
    launch_dma_pro<PT, KS, PRO_G>(a, grid, s);
  else
    launch_dma_pro<PT, KS, PRO_NONE>(a, grid, s);
}

}  // namespace

template <int PT, int KS, bool DMA>
void launch_batched_tile(const PassBatch& b, dim3 grid, hipStream_t s) {
  if (b.pro == PRO_G) {
    if (b.in_f64)
      hipLaunchKernelGGL((k_pass_split_batched<PT, KS, PRO_G, true, DMA>), grid, dim3(256), 0, s, b);
    else
      hipLaunchKernelGGL((k_pass_split_batched<PT, KS, PRO_G, false, DMA>), grid, dim3(256), 0, s, b);
  } else if (b.pro == PRO_FLOW) {
    if (b.in_f64)
      hipLaunchKernelGGL((k_pass_split_batched<PT, KS, PRO_FLOW, true, DMA>), grid, dim3(256), 0, s, b);
    else
      hipLaunchKernelGGL((k_pass_split_batched<PT, KS, PRO_FLOW, false, DMA>), grid, dim3(256), 0, s, b);
  } else {
    if (b.in_f64)
      hipLaunchKernelGGL((k_pass_split_batched<PT, KS, PRO_NONE, true, DMA>), grid, dim3(256), 0, s, b);
    else
      hipLaunchKernelGGL((k_pass_split_batched<PT, KS, PRO_NONE, false, DMA>), grid, dim3(256), 0, s, b);
  }
}

hipError_t launch_pass_split_batched(const PassBatch& b, int nwg, hipStream_t s) {
  if (b.tile < 0 || b.tile >= SPLIT_NTILES_BATCHED || b.ntiles <= 0 || nwg <= 0)
    return hipErrorInvalidValue;
  if (!b.in0 || !b.out0 || !b.inst || !b.tiles || !b.flag) return hipErrorInvalidValue;
  if ((b.epi == EPI_L4_R1 || b.epi == EPI_L4_R2 || b.epi == EPI_RICH || b.epi == EPI_L2) && !b.aux)
    return hipErrorInvalidValue;
  if (b.epi == EPI_L4_R1 && !b.out1) return hipErrorInvalidValue;
  if (b.epi < EPI_NONE || b.epi > EPI_L2) return hipErrorInvalidValue;
  if (b.pro != PRO_NONE && b.pro != PRO_FLOW && b.pro != PRO_G) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(nwg < b.ntiles ? nwg : b.ntiles));
  switch (b.tile) {
    case 0: launch_batched_tile<64, 32, false>(b, grid, s); break;
    case 1: launch_batched_tile<128, 16, false>(b, grid, s); break;
    case 2: launch_batched_tile<64, 16, true>(b, grid, s); break;
    default: launch_batched_tile<128, 16, true>(b, grid, s); break;
  }
  return hipGetLastError();
}

template <int PT>
void launch_batched_pair_tile(const PassBatch& b, int nwg, hipStream_t s) {
  // one 8-wave workgroup per CU for 128 rows (its LDS), two 4-wave ones for 64
  const int g = PT == 64 ? nwg : (nwg + 1) / 2;
  const dim3 grid(static_cast<unsigned>(g < b.ntiles ? g : b.ntiles)), block(PT * 4);
  if (b.pro == PRO_G) {
    if (b.in_f64)
      hipLaunchKernelGGL((k_pass_split_batched_pair<true, true, PT>), grid, block, 0, s, b);
    else
      hipLaunchKernelGGL((k_pass_split_batched_pair<true, false, PT>), grid, block, 0, s, b);
  } else {
    hipLaunchKernelGGL((k_pass_split_batched_pair<false, false, PT>), grid, block, 0, s, b);
  }
}

hipError_t launch_pass_split_batched_pair(const PassBatch& b, int nwg, hipStream_t s) {
  if ((b.tile != 2 && b.tile != 3) || b.ntiles <= 0 || nwg <= 0) return hipErrorInvalidValue;
  if (!b.in0 || !b.out0 || !b.inst || !b.tiles || !b.flag) return hipErrorInvalidValue;
  const bool sameg = b.pro == PRO_G;
  if (b.pro != PRO_NONE && !sameg) return hipErrorInvalidValue;
  if (!sameg && (!b.in1 || b.in_f64)) return hipErrorInvalidValue;
  if (b.epi != EPI_NONE && b.epi != EPI_L4_R1 && b.epi != EPI_L4_R2 && b.epi != EPI_L2)
    return hipErrorInvalidValue;
  if (b.epi != EPI_L4_R2 && b.epi != EPI_L2 && (!b.out1 || b.out_f64)) return hipErrorInvalidValue;
  if (b.tile == 2)
    launch_batched_pair_tile<64>(b, nwg, s);
  else
    launch_batched_pair_tile<128>(b, nwg, s);
  return hipGetLastError();
}

template <int PT>
void launch_pair_tile(const PassSplit& a, dim3 grid, hipStream_t s) {
  const dim3 block(PT * 4);
  if (a.pro == PRO_G) {
    if (a.in_f64)
      hipLaunchKernelGGL((k_pass_split_pair<true, true, PT>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_pass_split_pair<true, false, PT>), grid, block, 0, s, a);
  } else {
    hipLaunchKernelGGL((k_pass_split_pair<false, false, PT>), grid, block, 0, s, a);
  }
}

hipError_t launch_pass_split_pair(const PassSplit& a, hipStream_t s) {
  // the operator planes must be those of a direct-to-LDS shape (64 or 128 x 16)
  if (a.tile != 2 && a.tile != 3) return hipErrorInvalidValue;
  const int PT = SPLIT_TILES[a.tile].PT;
  if (a.R != 1 || a.Pp % PT != 0 || a.Kp % 16 != 0 || a.Kp < a.n || a.Pp < a.n || a.F <= 0)
    return hipErrorInvalidValue;
  if (!a.in0 || !a.out0 || !a.op || !a.flag) return hipErrorInvalidValue;
  const bool sameg = a.pro == PRO_G;
  if (a.pro != PRO_NONE && !sameg) return hipErrorInvalidValue;
  if (!sameg && (!a.in1 || a.in_f64)) return hipErrorInvalidValue;
  if (a.epi != EPI_NONE && a.epi != EPI_L4_R1 && a.epi != EPI_L4_R2 && a.epi != EPI_L2)
    return hipErrorInvalidValue;
  if (a.epi != EPI_L4_R2 && a.epi != EPI_L2 && (!a.out1 || a.out_f64)) return hipErrorInvalidValue;
  const int64_t nF = (a.F + FT - 1) / FT;
  const int64_t G = nF * (a.Pp / PT);
  if (G > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(G));
  if (PT == 64)
    launch_pair_tile<64>(a, grid, s);
  else
    launch_pair_tile<128>(a, grid, s);
  return hipGetLastError();
}

hipError_t launch_pass_split(const PassSplit& a, hipStream_t s) {
  if (a.tile < 0 || a.tile >= SPLIT_NTILES) return hipErrorInvalidValue;
  const int PT = SPLIT_TILES[a.tile].PT, KS = SPLIT_TILES[a.tile].KS;
  if (a.Pp % PT != 0 || a.Kp % KS != 0 || a.Kp < a.n || a.Pp < a.n || a.F <= 0)
    return hipErrorInvalidValue;
  if (!a.in0 || !a.out0 || !a.op || !a.flag) return hipErrorInvalidValue;
  if ((a.epi == EPI_L4_R1 || a.epi == EPI_L4_R2 || a.epi == EPI_RICH || a.epi == EPI_L2) && !a.aux)
    return hipErrorInvalidValue;
  if (a.epi == EPI_L4_R1 && !a.out1) return hipErrorInvalidValue;
  if (a.epi < EPI_NONE || a.epi > EPI_L2) return hipErrorInvalidValue;
  if (a.R_out < 1 || (a.pro != PRO_NONE && a.pro != PRO_FLOW && a.pro != PRO_G))
    return hipErrorInvalidValue;
  const int64_t nF = (a.F + FT - 1) / FT;
  const int64_t G = nF * (a.Pp / PT);
  if (G > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(G));
  if (SPLIT_TILES[a.tile].dma && a.R != 1) return hipErrorInvalidValue;
  if (a.ksplit > 1) {  // split contraction: the direct-to-LDS shapes only, a workspace that fits
    const int nKS = a.Kp / KS;
    if (!SPLIT_TILES[a.tile].dma || !a.ws || a.kchunk < 1 || a.ksplit > nKS || a.ksplit > 4 ||
        static_cast<int64_t>(a.ksplit - 1) * a.kchunk >= nKS ||
        static_cast<int64_t>(a.ksplit) * a.kchunk < nKS ||
        a.ksplit * G * (PT / 64) * 32 * 256 > a.ws_floats)
      return hipErrorInvalidValue;
  }
  switch (a.tile) {
    case 0: launch_tile<64, 32>(a, grid, s); break;
    case 1: launch_tile<128, 16>(a, grid, s); break;
    case 2: launch_tile_dma<64, 16>(a, grid, s); break;
    default: launch_tile_dma<128, 16>(a, grid, s); break;
  }
  return hipGetLastError();
}

}  // namespace cgl
