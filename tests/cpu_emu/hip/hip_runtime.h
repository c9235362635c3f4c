// Host emulation of the subset of the HIP runtime and device builtins used by
// libcgl, for running the library's kernels on the CPU under AddressSanitizer.
// Test infrastructure only: a workgroup runs as blockDim.x host threads with a
// std::barrier for __syncthreads(); MFMA builtins are emulated per wave with
// the operand/accumulator lane layouts measured on gfx950; device memory is
// host memory; graph capture records launches and replays them.
#pragma once

#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>
using std::isfinite;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) alignas(n)
// a device symbol's host name is its address in the emulation
#define HIP_SYMBOL(x) (&(x))

struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct double2 { double x, y; };
struct float2 { float x, y; };

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipStreamCaptureModeThreadLocal = 1 };
struct ihipStream_t { int dummy; };
typedef ihipStream_t* hipStream_t;
struct ihipEvent_t { int dummy; };
typedef ihipEvent_t* hipEvent_t;
struct emu_graph { std::vector<std::function<void()>> ops; };
typedef emu_graph* hipGraph_t;
typedef emu_graph* hipGraphExec_t;
typedef int hipStreamCaptureMode;

namespace emu {
inline thread_local dim3 tIdx, bIdx;
inline dim3 gDim, bDim;
inline std::barrier<>* block_barrier = nullptr;
inline std::vector<std::unique_ptr<std::barrier<>>> wave_barriers;
inline std::mutex atomic_mu;
inline bool capturing = false;
inline emu_graph* capture_graph = nullptr;
// per-wave operand exchange for MFMA emulation (16 bytes per lane per operand)
inline std::vector<std::vector<unsigned char>> xa, xb;
}  // namespace emu

#define threadIdx (emu::tIdx)
#define blockIdx (emu::bIdx)
#define gridDim (emu::gDim)
#define blockDim (emu::bDim)

inline void __syncthreads() { emu::block_barrier->arrive_and_wait(); }

inline unsigned atomicOr(unsigned* p, unsigned v) {
  std::lock_guard<std::mutex> g(emu::atomic_mu);
  unsigned o = *p;
  *p = o | v;
  return o;
}

namespace emu {
inline int lane() { return static_cast<int>(tIdx.x & 63); }
inline int wave() { return static_cast<int>(tIdx.x >> 6); }
template <class T>
inline void exchange(const T& a, const T& b) {
  static_assert(sizeof(T) <= 16, "operand too large");
  std::memcpy(&xa[wave()][lane() * 16], &a, sizeof(T));
  std::memcpy(&xb[wave()][lane() * 16], &b, sizeof(T));
  wave_barriers[wave()]->arrive_and_wait();
}
template <class T>
inline T get(const std::vector<unsigned char>& x, int l) {
  T v;
  std::memcpy(&v, &x[l * 16], sizeof(T));
  return v;
}
}  // namespace emu

typedef double emu_f64x4 __attribute__((ext_vector_type(4)));
typedef float emu_f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 emu_bf16x8 __attribute__((ext_vector_type(8)));

// D(16x16) += A(16x4) B(4x16); lane l: A[l%16][l/16], B[l/16][l%16],
// accumulator register r: row l/16 + 4r, column l%16.
inline emu_f64x4 emu_mfma_f64(double a, double b, emu_f64x4 c) {
  emu::exchange(a, b);
  const int l = emu::lane();
  emu_f64x4 d = c;
  for (int r = 0; r < 4; ++r) {
    const int row = l / 16 + 4 * r, col = l % 16;
    double s = 0.0;
    for (int k = 0; k < 4; ++k)
      s += emu::get<double>(emu::xa[emu::wave()], row + 16 * k) *
           emu::get<double>(emu::xb[emu::wave()], col + 16 * k);
    d[r] += s;
  }
  emu::wave_barriers[emu::wave()]->arrive_and_wait();
  return d;
}

// D(32x32) += A(32x16) B(16x32) in bf16 with FP32 accumulation; lane l:
// A[l%32][8(l/32)+e], B[8(l/32)+e][l%32], accumulator register r:
// row 8(r/4) + 4(l/32) + r%4, column l%32.
inline emu_f32x16 emu_mfma_bf16_32(emu_bf16x8 a, emu_bf16x8 b, emu_f32x16 c) {
  emu::exchange(a, b);
  const int l = emu::lane();
  emu_f32x16 d = c;
  for (int r = 0; r < 16; ++r) {
    const int row = 8 * (r / 4) + 4 * (l / 32) + r % 4, col = l % 32;
    double s = 0.0;
    for (int k = 0; k < 16; ++k) {
      const emu_bf16x8 av = emu::get<emu_bf16x8>(emu::xa[emu::wave()], row + 32 * (k / 8));
      const emu_bf16x8 bv = emu::get<emu_bf16x8>(emu::xb[emu::wave()], col + 32 * (k / 8));
      s += static_cast<double>(static_cast<float>(av[k % 8])) *
           static_cast<double>(static_cast<float>(bv[k % 8]));
    }
    d[r] = static_cast<float>(static_cast<double>(d[r]) + s);
  }
  emu::wave_barriers[emu::wave()]->arrive_and_wait();
  return d;
}

// D(16x16) += A(16x32) B(32x16) in bf16 with FP32 accumulation; lane l:
// A[l%16][8(l/16)+e], B[8(l/16)+e][l%16], accumulator register r: row
// 4(l/16) + r, column l%16.
typedef float emu_f32x4 __attribute__((ext_vector_type(4)));
inline emu_f32x4 emu_mfma_bf16_16(emu_bf16x8 a, emu_bf16x8 b, emu_f32x4 c) {
  emu::exchange(a, b);
  const int l = emu::lane();
  emu_f32x4 d = c;
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * (l / 16) + r, col = l % 16;
    double s = 0.0;
    for (int k = 0; k < 32; ++k) {
      const emu_bf16x8 av = emu::get<emu_bf16x8>(emu::xa[emu::wave()], row + 16 * (k / 8));
      const emu_bf16x8 bv = emu::get<emu_bf16x8>(emu::xb[emu::wave()], col + 16 * (k / 8));
      s += static_cast<double>(static_cast<float>(av[k % 8])) *
           static_cast<double>(static_cast<float>(bv[k % 8]));
    }
    d[r] = static_cast<float>(static_cast<double>(d[r]) + s);
  }
  emu::wave_barriers[emu::wave()]->arrive_and_wait();
  return d;
}

inline double atomicAdd(double* p, double v) {
  std::lock_guard<std::mutex> g(emu::atomic_mu);
  const double o = *p;
  *p = o + v;
  return o;
}

// raw buffer resource: base address and byte range; each dword of a load at
// or past the range reads as zero (as the hardware's range check returns)
struct emu_buffer_rsrc {
  const char* base;
  uint32_t num;
};
typedef emu_buffer_rsrc __amdgpu_buffer_rsrc_t;
typedef unsigned emu_u32x4 __attribute__((ext_vector_type(4)));
inline emu_buffer_rsrc __builtin_amdgcn_make_buffer_rsrc(void* p, short, int num, int) {
  return {static_cast<const char*>(p), static_cast<uint32_t>(num)};
}
inline unsigned emu_buffer_dword(emu_buffer_rsrc r, uint64_t o) {
  unsigned w = 0;
  if (o + 4 <= r.num) std::memcpy(&w, r.base + o, 4);
  return w;
}
inline emu_u32x4 __builtin_amdgcn_raw_buffer_load_b128(emu_buffer_rsrc r, unsigned voff, int soff,
                                                       int) {
  emu_u32x4 v;
  for (int i = 0; i < 4; ++i)
    v[i] = emu_buffer_dword(r, static_cast<uint64_t>(voff) + static_cast<uint64_t>(soff) + 4u * i);
  return v;
}
// buffer load to LDS: lane l of the wave writes its `size` bytes at
// lds + offset + l * size
inline void __builtin_amdgcn_raw_ptr_buffer_load_lds(emu_buffer_rsrc r,
                                                     __attribute__((address_space(3))) void* lds,
                                                     unsigned size, unsigned voff, unsigned soff,
                                                     unsigned off, unsigned) {
  char* d = reinterpret_cast<char*>(reinterpret_cast<uintptr_t>(lds)) + off +
            (emu::tIdx.x % 64u) * size;
  for (unsigned i = 0; i < size; i += 4) {
    const unsigned w = emu_buffer_dword(r, static_cast<uint64_t>(voff) + soff + off + i);
    std::memcpy(d + i, &w, 4);
  }
}
// v_readfirstlane: lane 0's value to every lane of the wave.  The library
// applies it to wave-uniform values only; the emulation checks that they are.
inline unsigned emu_readfirstlane(unsigned v) {
  emu::exchange(v, v);
  const unsigned r = emu::get<unsigned>(emu::xa[emu::wave()], 0);
  emu::wave_barriers[emu::wave()]->arrive_and_wait();
  if (r != v) {
    std::fprintf(stderr, "readfirstlane of a value that differs across the wave\n");
    std::abort();
  }
  return r;
}
#define __builtin_amdgcn_readfirstlane(v) emu_readfirstlane(static_cast<unsigned>(v))

#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __builtin_amdgcn_sched_group_barrier(m, n, id) ((void)0)
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)
#define __builtin_amdgcn_s_barrier() __syncthreads()
#define __builtin_amdgcn_fence(...) ((void)0)

#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) emu_mfma_f64((a), (b), (c))
#define __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, x, y, z) emu_mfma_bf16_32((a), (b), (c))
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, x, y, z) emu_mfma_bf16_16((a), (b), (c))

namespace emu {
// A persistent pool of host threads plays the workgroup's lanes: for every
// workgroup the launcher publishes the body and releases the pool through a
// start barrier, then waits at an end barrier.
struct Pool {
  unsigned nt = 0;
  std::vector<std::thread> th;
  std::unique_ptr<std::barrier<>> start, end, bar;
  std::function<void()> body;
  unsigned bx = 0;
  bool quit = false;
  void ensure(unsigned n) {
    if (n == nt) return;
    shutdown();
    nt = n;
    start.reset(new std::barrier<>(n + 1));
    end.reset(new std::barrier<>(n + 1));
    bar.reset(new std::barrier<>(n));
    for (unsigned t = 0; t < n; ++t)
      th.emplace_back([this, t]() {
        for (;;) {
          start->arrive_and_wait();
          if (quit) return;
          tIdx = dim3(t);
          bIdx = dim3(bx);
          body();
          end->arrive_and_wait();
        }
      });
  }
  void shutdown() {
    if (!nt) return;
    quit = true;
    start->arrive_and_wait();
    for (auto& x : th) x.join();
    th.clear();
    quit = false;
    nt = 0;
  }
  ~Pool() { shutdown(); }
};
inline Pool pool;

template <class K, class... Args>
void run_kernel(K kernel, dim3 grid, dim3 block, Args... args) {
  const unsigned nt = block.x;
  const unsigned nw = (nt + 63) / 64;
  pool.ensure(nt);
  gDim = grid;
  bDim = block;
  xa.assign(nw, std::vector<unsigned char>(64 * 16));
  xb.assign(nw, std::vector<unsigned char>(64 * 16));
  block_barrier = pool.bar.get();
  if (wave_barriers.size() != nw) {
    wave_barriers.clear();
    for (unsigned w = 0; w < nw; ++w) wave_barriers.emplace_back(new std::barrier<>(64));
  }
  pool.body = [=]() { kernel(args...); };
  for (unsigned bx = 0; bx < grid.x; ++bx) {
    pool.bx = bx;
    pool.start->arrive_and_wait();
    pool.end->arrive_and_wait();
  }
}
template <class K, class... Args>
void launch(K kernel, dim3 grid, dim3 block, Args... args) {
  if (capturing) {
    capture_graph->ops.push_back([=]() { run_kernel(kernel, grid, block, args...); });
  } else {
    run_kernel(kernel, grid, block, args...);
  }
}
}  // namespace emu

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  emu::launch(kernel, dim3(grid), dim3(block), __VA_ARGS__)

inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipMalloc(void** p, size_t n) {
  *p = std::malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipHostMalloc(void** p, size_t n) { return hipMalloc(p, n); }
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, int, hipStream_t) {
  if (emu::capturing) {
    emu::capture_graph->ops.push_back([=]() { std::memcpy(d, s, n); });
  } else {
    std::memcpy(d, s, n);
  }
  return hipSuccess;
}
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, int k) { return hipMemcpyAsync(d, s, n, k, nullptr); }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new ihipStream_t(); return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new ihipEvent_t(); return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = new ihipEvent_t(); return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
// elapsed times are not measured in the emulation: every candidate ties
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1.0f; return hipSuccess; }
struct hipDeviceProp_t { char gcnArchName[256]; };
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
enum { hipDeviceAttributeMultiprocessorCount = 1 };
// a small emulated device: few workgroups, so persistent grids loop over tiles
inline hipError_t hipDeviceGetAttribute(int* v, int, int) { *v = 2; return hipSuccess; }
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  std::strcpy(p->gcnArchName, "emu");
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, int) {
  emu::capturing = true;
  emu::capture_graph = new emu_graph();
  return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  emu::capturing = false;
  *g = emu::capture_graph;
  emu::capture_graph = nullptr;
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t) {
  *e = new emu_graph(*g);
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto& op : e->ops) op();
  return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
