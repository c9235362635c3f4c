// Fourier pass: the exponential of one periodic direction (Section 3.2),
// applied along every fibre as F^{-1} diag(e) F with a length-n discrete
// Fourier transform (n a power of two, 8 <= n <= 1024), the pointwise product
// with the direction's factors e_k = exp(t A_mu)_kk and the inverse
// transform.  One read and one write of the tensor per pass (HBM-bound), the
// same pass interface as the mu-mode product kernels: the stepper's prologue
// on the staged input, its epilogue before the store, contiguous or strided
// fibres, rotated or in-place output.
//
// A workgroup stages FPW whole fibres in LDS (each as an N1 x N2 array,
// element j = N2 j1 + j2 at row j1, column j2, N = N1 N2, N1 >= N2) and runs
// the four-step transform on them:
//   forward:  for each column j2, a length-N1 DFT over j1, times w_N^{j2 k1};
//             for each row k1, a length-N2 DFT over j2 -> X[k1 + N1 k2];
//   product:  X[k] *= e_k;
//   inverse:  for each row k1, the inverse length-N2 DFT over k2, times
//             w_N^{-j2 k1}; for each column j2, the inverse length-N1 DFT
//             over k1, times 1/N -> x[N2 j1 + j2],
// w_N = exp(-2 pi i / N).  The row step's thread keeps the row from the end
// of the forward transform to the start of the inverse one, so a fibre goes
// through LDS three times.  The short DFTs run in registers (iterative
// radix-2, twiddles from an LDS copy of the table exp(-2 pi i k / N)).
// Arithmetic in T: double for complex128 passes, float for complex64 ones.
#include <type_traits>

#include "kernels.hpp"
#include "pointwise.hpp"

namespace cgl {

namespace {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a times the conjugate of b
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
constexpr int bitrev(int v, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
  return r;
}

// x times w_N^q (forward) or its conjugate (inverse).  In FP32 the table
// entries w = 1 (q = 0) and w = -i (q = N/4) are applied exactly, without a
// product (in FP64, at its register bound, this measured slower)
template <int N, bool INV, typename T>
__device__ __forceinline__ cx<T> twiddle(cx<T> x, int q, const cx<T>* tw) {
  if (sizeof(T) == 4 && q == 0) return x;
  if (sizeof(T) == 4 && q == N / 4) return INV ? cx<T>{-x.im, x.re} : cx<T>{x.im, -x.re};
  const cx<T> w = tw[q];
  return INV ? cmulc(x, w) : cmul(x, w);
}

// Length-M DFT of x in natural order (M a power of two <= 32), forward
// (sum_j x_j w_M^{jk}) or inverse (sum_k x_k w_M^{-jk}, unscaled).  tw holds
// w_N^q, q < N, and w_M = w_N^S with S = N / M.
template <int M, int S, bool INV, typename T>
__device__ __forceinline__ void dft(cx<T> (&x)[M], const cx<T>* tw) {
  constexpr int B = ilog2(M);
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const int j = bitrev(i, B);
    if (j > i) {
      const cx<T> t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
#pragma unroll
  for (int len = 2; len <= M; len <<= 1) {
#pragma unroll
    for (int i = 0; i < M; i += len)
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        // the loops unroll completely, so the table index is a constant
        const cx<T> v = twiddle<M * S, INV>(x[i + j + len / 2], j * (M / len) * S, tw);
        const cx<T> u = x[i + j];
        x[i + j] = {u.re + v.re, u.im + v.im};
        x[i + j + len / 2] = {u.re - v.re, u.im - v.im};
      }
  }
}

template <int N>
struct FftGeom {
  static constexpr int B = ilog2(N);
  static constexpr int N1 = 1 << ((B + 1) / 2);  // rows
  static constexpr int N2 = N / N1;              // columns (N2 <= N1)
  static_assert((1 << B) == N && N >= 8 && N <= 1024, "power-of-two lengths 8 .. 1024");
};

// Fibres per workgroup and the LDS layout of the staged fibres: element
// (j1, j2) of fibre fl at fl * FS + j1 * P + j2 (complex units).
// complex64 (FF): in the transform phases consecutive threads take
// consecutive fibres, so the 16 lanes that share an LDS cycle (8-byte
// accesses, 32 banks) cover FPW fibres x G = 16 / FPW rows or columns:
// FS = G mod 16 spreads the fibres and, when G > 1, a row pitch P = 1 mod 16
// spreads the rows.  With G = 1 the rows stay unpadded, so a contiguous run of
// 16 elements of one fibre (the staging of a contiguous fibre) is
// conflict-free as well.  complex128: consecutive threads take consecutive
// columns (rows) of one fibre, rows padded by one element (measured faster
// for 16-byte elements, whose kernel is at its register bound).
// threads per workgroup: 512 for the complex64 length-128 pass (32 fibres:
// 256-byte runs of a strided tensor per index), 256 otherwise
template <typename T, int N>
constexpr int fft_threads() { return sizeof(T) == 4 && N == 128 ? 512 : 256; }

template <typename T, int N>
struct FftTile {
  using Gm = FftGeom<N>;
  static constexpr int NT = fft_threads<T, N>();
  static constexpr int FPW_MAX = NT / Gm::N1;
  static constexpr int FPW_LDS = (sizeof(T) == 8 ? 2048 : 4096) * (NT / 256) / N;
  static constexpr int FPW = FPW_MAX < FPW_LDS ? FPW_MAX : (FPW_LDS > 0 ? FPW_LDS : 1);
  static constexpr int EPT = FPW * N / NT;  // tensor elements per thread
  static_assert(EPT * NT == FPW * N, "a workgroup's fibres fill its threads evenly");
  static constexpr bool FF = sizeof(T) == 4;
  static constexpr int G = FPW >= 16 ? 1 : 16 / FPW;
  static constexpr int P = FF && G == 1 ? Gm::N2 : Gm::N2 + 1;
  static constexpr int FS = FF ? Gm::N1 * P + (((G - Gm::N1 * P) % 16) + 16) % 16 : Gm::N1 * P;
  static_assert(!FF || (FS % 16 == G % 16 && FS >= Gm::N1 * P), "fibre stride");
};

// Offsets of a workgroup's elements in a tensor whose fibres have stride R
// (fibre f starts at (f mod R) + (f div R) R n).  Element i of a thread is
// e = tid + NT i: with R = 1 (contiguous fibres) fibre e / n, index e mod n;
// otherwise fibre e mod FPW, index e / FPW, so all elements of a thread lie
// on one fibre, whose start is computed once.  The first fibre f0 is a
// multiple of FPW: when R is one too, the workgroup's fibres share f div R,
// a division of uniform values.
template <int N, int FPW, int NT>
struct ElemAddr {
  static_assert(NT % FPW == 0, "a thread keeps one fibre when R > 1");
  bool contig;
  int64_t R, fst;  // fst: start of the thread's fibre (R > 1)
  __device__ __forceinline__ ElemAddr(int64_t f0, int64_t R_, int tid) : contig(R_ == 1), R(R_), fst(0) {
    if (!contig) {
      const int fl = tid % FPW;
      if (R % FPW == 0) {
        const int64_t q = f0 / R;
        fst = (f0 - q * R) + fl + q * R * N;
      } else {
        const int64_t f = f0 + fl;
        fst = (f % R) + (f / R) * R * N;
      }
    }
  }
  __device__ __forceinline__ int fl(int e) const { return contig ? e / N : e % FPW; }
  __device__ __forceinline__ int k(int e) const { return contig ? e % N : e / FPW; }
  __device__ __forceinline__ int64_t off(int64_t f0, int e) const {
    return contig ? f0 * N + e : fst + R * static_cast<int64_t>(e / FPW);
  }
};

// raw element of a complex64 (float2) or complex128 (double2) tensor
template <bool F64>
using Raw = std::conditional_t<F64, double2, float2>;

template <bool F64>
__device__ __forceinline__ Raw<F64> load_raw(const void* p, int64_t off) {
  return reinterpret_cast<const Raw<F64>*>(p)[off];
}

template <typename R>
__device__ __forceinline__ cd to_cd(R v) {
  return {static_cast<double>(v.x), static_cast<double>(v.y)};
}

template <typename T>
__device__ __forceinline__ cd load_in(const void* p, int64_t off, bool f64) {
  if (f64) {
    const double2 v = reinterpret_cast<const double2*>(p)[off];
    return {v.x, v.y};
  }
  const float2 v = reinterpret_cast<const float2*>(p)[off];
  return {static_cast<double>(v.x), static_cast<double>(v.y)};
}

__device__ __forceinline__ void store_out(void* p, int64_t off, bool f64, cd v) {
  if (f64)
    reinterpret_cast<double2*>(p)[off] = double2{v.re, v.im};
  else
    reinterpret_cast<float2*>(p)[off] = float2{static_cast<float>(v.re), static_cast<float>(v.im)};
}

// IN64: the input tensor is complex128 (always for T = double; for T = float
// the first pass of a plan whose state is complex128)
// Lengths up to 128 keep four workgroups (16 waves) per CU resident (at most
// 128 VGPRs): a 128^3 pass is then one round of workgroups.
template <typename T, int N, bool IN64>
__global__ __launch_bounds__((fft_threads<T, N>()), N <= 128 ? 4 : 1) void k_pass_fft(PassFFT a) {
  using G = FftGeom<N>;
  using Tl = FftTile<T, N>;
  constexpr int N1 = G::N1, N2 = G::N2;
  constexpr int FPW = Tl::FPW, EPT = Tl::EPT, NT = Tl::NT;
  constexpr int P = Tl::P, FS = Tl::FS;  // LDS row pitch and fibre stride (complex)
  constexpr bool FF = Tl::FF;            // fibres across consecutive threads
  __shared__ cx<T> tile[FPW * FS];
  __shared__ cx<T> tw[N];
  __shared__ cx<T> efac[N];  // the direction's factors e_k
  const int tid = threadIdx.x;
  const int64_t f0 = static_cast<int64_t>(blockIdx.x) * FPW;
  const bool out64 = a.out_f64 != 0;
  unsigned flag = 0;

  // stage the fibres (consecutive threads take consecutive elements of a
  // contiguous fibre, or consecutive fibres of one index when strided): every
  // load of the thread is issued before the first is used, then the
  // prologue and the LDS stores
  const ElemAddr<N, FPW, NT> ain(f0, a.R, tid);
  Raw<IN64> raw[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + NT * i;
    raw[i] = Raw<IN64>{0, 0};
    if (f0 + ain.fl(e) < a.F) raw[i] = load_raw<IN64>(a.in0, ain.off(f0, e));
  }
  // the twiddle table and the factors, loaded behind the tensor's elements
  for (int q = tid; q < N; q += NT) {
    const double2 w = reinterpret_cast<const double2*>(a.tw)[q];
    tw[q] = {static_cast<T>(w.x), static_cast<T>(w.y)};
    efac[q] = reinterpret_cast<const cx<T>*>(a.fac)[q];
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + NT * i;
    const int fl = ain.fl(e), k = ain.k(e);
    cx<T> w = {static_cast<T>(raw[i].x), static_cast<T>(raw[i].y)};
    if (a.pro != PRO_NONE && f0 + fl < a.F) {  // the prologue in FP64
      cd v = to_cd(raw[i]);
      if (a.pro == PRO_FLOW)
        v = flow_in(v, a.nl.tf, a.nl, flag);
      else
        v = g_cgl(v, a.nl);
      w = {static_cast<T>(v.re), static_cast<T>(v.im)};
    }
    tile[fl * FS + (k / N2) * P + (k % N2)] = w;
  }
  __syncthreads();
  // forward, columns: length-N1 DFTs over j1, twiddle w_N^{j2 k1}
  if (tid < FPW * N2) {
    const int fl = FF ? tid % FPW : tid / N2, j2 = FF ? tid / FPW : tid % N2;
    cx<T>* t = tile + fl * FS + j2;
    cx<T> x[N1];
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) x[j1] = t[j1 * P];
    dft<N1, N2, false>(x, tw);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) t[k1 * P] = cmul(x[k1], tw[(j2 * k1) & (N - 1)]);
  }
  __syncthreads();
  // rows: length-N2 DFT over j2 (X[k1 + N1 k2]), the factors, the inverse
  // length-N2 DFT over k2 and the twiddle w_N^{-j2 k1}
  if (tid < FPW * N1) {
    const int fl = FF ? tid % FPW : tid / N1, k1 = FF ? tid / FPW : tid % N1;
    cx<T>* t = tile + fl * FS + k1 * P;
    cx<T> y[N2];
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2) y[j2] = t[j2];
    dft<N2, N1, false>(y, tw);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) y[k2] = cmul(y[k2], efac[k1 + N1 * k2]);
    dft<N2, N1, true>(y, tw);
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2) t[j2] = cmulc(y[j2], tw[(j2 * k1) & (N - 1)]);
  }
  __syncthreads();
  // inverse, columns: length-N1 inverse DFTs over k1, scaled by 1/N
  const T sc = static_cast<T>(1.0 / N);
  if (tid < FPW * N2) {
    const int fl = FF ? tid % FPW : tid / N2, j2 = FF ? tid / FPW : tid % N2;
    cx<T>* t = tile + fl * FS + j2;
    cx<T> x[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) x[k1] = t[k1 * P];
    dft<N1, N2, true>(x, tw);
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) t[j1 * P] = {x[j1].re * sc, x[j1].im * sc};
  }
  __syncthreads();
  // store with the epilogue (consecutive threads take consecutive output
  // elements: along the fibre when the output stride is 1, across fibres
  // otherwise); an epilogue with an auxiliary tensor issues all of the
  // thread's auxiliary loads first
  const bool has_aux = a.epi == EPI_L4_R1 || a.epi == EPI_L4_R2 || a.epi == EPI_RICH ||
                       a.epi == EPI_L2;
  const ElemAddr<N, FPW, NT> aout(f0, a.R_out, tid);
  cd xa[EPT];
  if (has_aux) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + NT * i;
      xa[i] = cd{0.0, 0.0};
      if (f0 + aout.fl(e) < a.F) xa[i] = load_in<T>(a.aux, aout.off(f0, e), a.aux_f64 != 0);
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + NT * i;
    const int fl = aout.fl(e), m = aout.k(e);
    if (f0 + fl >= a.F) continue;
    const int64_t off = aout.off(f0, e);
    const cx<T> c = tile[fl * FS + (m / N2) * P + (m % N2)];
    const cd y = {static_cast<double>(c.re), static_cast<double>(c.im)};
    if (a.epi == EPI_NONE) {
      if (out64)
        reinterpret_cast<double2*>(a.out0)[off] = double2{static_cast<double>(c.re), static_cast<double>(c.im)};
      else
        reinterpret_cast<float2*>(a.out0)[off] = float2{static_cast<float>(c.re), static_cast<float>(c.im)};
    } else if (a.epi == EPI_FLOW || a.epi == EPI_MID) {
      const cd z = a.epi == EPI_FLOW ? flow_out(y, a.nl.tf, a.nl, flag)
                                     : flow_mid(y, a.nl.tf, a.nl, flag);
      if (!finite2(z)) flag |= FLAG_NONFINITE;
      store_out(a.out0, off, out64, z);
    } else {
      const cd x = xa[i];
      if (a.epi == EPI_L4_R1) {  // y = Q, x = P
        cd X, Y;
        lawson_r1(x, y, a.nl, X, Y);
        store_out(a.out0, off, out64, X);
        store_out(a.out1, off, out64, Y);
      } else {
        const cd z = a.epi == EPI_L4_R2 ? lawson_r2(x, y, a.nl)
                     : a.epi == EPI_RICH ? richardson(y, x, a.nl, flag)
                                         : lawson2(x, y, a.nl, 0.5 * a.nl.tau);
        if (!finite2(z)) flag |= FLAG_NONFINITE;
        store_out(a.out0, off, out64, z);
      }
    }
  }
  if (flag) atomicOr(a.flag, flag);
}

template <typename T, int N>
hipError_t launch_n(const PassFFT& a, hipStream_t s) {
  constexpr int FPW = FftTile<T, N>::FPW;
  const int64_t G = (a.F + FPW - 1) / FPW;
  if (G > 0x7fffffffLL) return hipErrorInvalidValue;
  if constexpr (sizeof(T) == 8) {
    if (!a.in_f64) return hipErrorInvalidValue;  // FP64 passes read complex128
    hipLaunchKernelGGL((k_pass_fft<T, N, true>), dim3(static_cast<unsigned>(G)), dim3(fft_threads<T, N>()), 0, s, a);
  } else if (a.in_f64) {
    hipLaunchKernelGGL((k_pass_fft<T, N, true>), dim3(static_cast<unsigned>(G)), dim3(fft_threads<T, N>()), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_pass_fft<T, N, false>), dim3(static_cast<unsigned>(G)), dim3(fft_threads<T, N>()), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_t(const PassFFT& a, hipStream_t s) {
  switch (a.n) {
    case 8: return launch_n<T, 8>(a, s);
    case 16: return launch_n<T, 16>(a, s);
    case 32: return launch_n<T, 32>(a, s);
    case 64: return launch_n<T, 64>(a, s);
    case 128: return launch_n<T, 128>(a, s);
    case 256: return launch_n<T, 256>(a, s);
    case 512: return launch_n<T, 512>(a, s);
    case 1024: return launch_n<T, 1024>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool fft_length_supported(int64_t n) { return n >= 8 && n <= 1024 && (n & (n - 1)) == 0; }

hipError_t launch_pass_fft(const PassFFT& a, hipStream_t s) {
  if (!fft_length_supported(a.n) || a.F <= 0 || a.R < 1 || a.R_out < 1) return hipErrorInvalidValue;
  if (!a.in0 || !a.out0 || !a.fac || !a.tw || !a.flag) return hipErrorInvalidValue;
  if ((a.epi == EPI_L4_R1 || a.epi == EPI_L4_R2 || a.epi == EPI_RICH || a.epi == EPI_L2) && !a.aux)
    return hipErrorInvalidValue;
  if (a.epi == EPI_L4_R1 && !a.out1) return hipErrorInvalidValue;
  if (a.epi < EPI_NONE || a.epi > EPI_L2) return hipErrorInvalidValue;
  if (a.pro != PRO_NONE && a.pro != PRO_FLOW && a.pro != PRO_G) return hipErrorInvalidValue;
  return a.fp64 ? launch_t<double>(a, s) : launch_t<float>(a, s);
}

}  // namespace cgl
