// Test infrastructure: a CPU emulation of the HIP subset that libvpm uses,
// so that the CPU test suite can run the rollout kernels' logic against the
// oracle. It is never part of the product library.
//
// One OS thread per GPU thread; blocks run one after another; __syncthreads
// is a block barrier; cross-lane operations (shfl, readlane, readfirstlane,
// wave barrier) exchange through a per-wave buffer between two 64-thread
// barriers, so one reached by only part of a wave deadlocks (the test's
// timeout reports it). Device memory is host memory, filled with 0xff bytes
// on allocation (NaN floats) so that reads of unwritten memory show up.
// It checks indexing and synchronisation logic, not the compiler: code the
// compiler handles differently from its source (lane convergence inside
// loops) must still be checked on the GPU.
#pragma once
#include <algorithm>
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

using std::max;
using std::min;
using std::isfinite;
using std::isnan;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define __launch_bounds__(...)
#define __align__(n) alignas(n)
#define __shared__ static
#define __constant__
#define HIP_SYMBOL(x) (&(x))

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
typedef void *hipStream_t;
typedef void *hipEvent_t;
struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct double2 { double x, y; };
struct float2 { float x, y; };
struct int2 { int x, y; };
inline double2 make_double2(double a, double b) { return {a, b}; }
inline int2 make_int2(int a, int b) { return {a, b}; }
struct hipDeviceProp_t {
  char gcnArchName[256];
  int multiProcessorCount;
  size_t sharedMemPerBlock;
};
enum hipStreamCaptureStatus { hipStreamCaptureStatusNone = 0, hipStreamCaptureStatusActive = 1 };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
enum { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
enum { hipDeviceAttributeSharedMemPerBlockOptin = 1, hipDeviceAttributeMaxSharedMemoryPerBlock = 2,
       hipDeviceAttributeMultiprocessorCount = 3 };
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };

inline int emu_n_cu() { const char *s = getenv("EMU_N_CU"); return s ? atoi(s) : 4; }
template <class T> inline hipError_t hipMalloc(T **p, size_t n) {
  *p = static_cast<T *>(aligned_alloc(256, (n + 255) / 256 * 256 + 256));
  if (*p) memset((void *)*p, 0xff, n);  // poison: NaN floats, -1 ints
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void *p) { free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, int) { memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, int, hipStream_t) { memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
// the emulated device is the host: a device variable's address is its own
template <class T> inline hipError_t hipGetSymbolAddress(void **p, T *sym) {
  *p = static_cast<void *>(sym);
  return hipSuccess;
}
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) {
  memset(p, 0, sizeof(*p));
  strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
  p->multiProcessorCount = emu_n_cu();
  p->sharedMemPerBlock = 65536;
  return hipSuccess;
}
inline hipError_t hipDeviceGetAttribute(int *v, int attr, int) {
  *v = attr == hipDeviceAttributeMultiprocessorCount ? emu_n_cu()
       : attr == hipDeviceAttributeSharedMemPerBlockOptin ? 163840 : 65536;
  return hipSuccess;
}
inline hipError_t hipFuncSetAttribute(const void *, int, int) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = (void *)0x1; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = (void *)0x1; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus *s) { *s = hipStreamCaptureStatusNone; return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t) { return "emulated error"; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }

struct EmuBlock {
  std::unique_ptr<std::barrier<>> bar;
  std::vector<std::unique_ptr<std::barrier<>>> wbar;
  std::vector<uint64_t> wbuf;  // [waves][64]
  unsigned char *dyn = nullptr;
};
inline thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
inline thread_local EmuBlock *emu_blk = nullptr;

inline void __syncthreads() { emu_blk->bar->arrive_and_wait(); }
template <class T> inline T emu_exchange(T v, int src) {
  static_assert(sizeof(T) <= 8, "");
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  uint64_t raw = 0;
  memcpy(&raw, &v, sizeof(T));
  __atomic_store_n(&emu_blk->wbuf[w * 64 + l], raw, __ATOMIC_SEQ_CST);
  emu_blk->wbar[w]->arrive_and_wait();
  raw = __atomic_load_n(&emu_blk->wbuf[w * 64 + (src & 63)], __ATOMIC_SEQ_CST);
  emu_blk->wbar[w]->arrive_and_wait();
  T r;
  memcpy(&r, &raw, sizeof(T));
  return r;
}
template <class T> inline T __shfl(T v, int src, int = 64) { return emu_exchange(v, src); }
template <class T> inline T __shfl_xor(T v, int m, int = 64) { return emu_exchange(v, (int)(threadIdx.x & 63) ^ m); }
#define __builtin_amdgcn_readfirstlane(v) emu_exchange((v), 0)
// DPP: quad_perm, row_ror, row_bcast:15 and row_bcast:31 (the controls the
// kernels use); rows outside the row mask keep `old`
inline int emu_dpp(int old, int v, int ctrl, int row_mask) {
  const int l = threadIdx.x & 63, row = l >> 4;
  int src = l;
  if (ctrl < 0x100) src = (l & ~3) + ((ctrl >> (2 * (l & 3))) & 3);
  else if (ctrl > 0x120 && ctrl < 0x130) src = (l & ~15) + (((l & 15) - (ctrl - 0x120)) & 15);
  else if (ctrl == 0x142) src = row > 0 ? 16 * row - 1 : l;
  else if (ctrl == 0x143) src = 31;
  const int r = emu_exchange(v, src);
  return (row_mask >> row) & 1 ? r : old;
}
#define __builtin_amdgcn_update_dpp(old, v, ctrl, rm, bm, bc) emu_dpp((old), (v), (ctrl), (rm))
#define __builtin_amdgcn_readlane(v, j) emu_exchange((v), (j))
inline long long __double_as_longlong(double d) { long long r; memcpy(&r, &d, 8); return r; }
inline double __longlong_as_double(long long v) { double r; memcpy(&r, &v, 8); return r; }
#define __builtin_amdgcn_wave_barrier() emu_blk->wbar[threadIdx.x >> 6]->arrive_and_wait()
#define __builtin_amdgcn_fence(a, b) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __builtin_amdgcn_s_setprio(p) ((void)0)
#define __builtin_amdgcn_s_getreg(r) ((unsigned)(threadIdx.x >> 6) << 4)
#define __builtin_amdgcn_rsqf(x) (1.0f / std::sqrt((float)(x)))
#define __builtin_amdgcn_rcpf(x) (1.0f / (float)(x))
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt((double)(x)))
#define __builtin_amdgcn_rcp(x) (1.0 / (double)(x))
inline unsigned long long wall_clock64() { return 0; }
template <class T> inline T atomicAdd(T *p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }

inline void emu_thread_main(std::function<void()> *f) { (*f)(); }

template <class... P, class... A>
void emu_launch(void (*k)(P...), dim3 g, dim3 b, size_t shmem, A... args) {
  const unsigned nthr = b.x, nblk = g.x;
  for (unsigned bi = 0; bi < nblk; ++bi) {
    EmuBlock blk;
    blk.bar = std::make_unique<std::barrier<>>(nthr);
    for (unsigned w = 0; w < (nthr + 63) / 64; ++w) blk.wbar.push_back(std::make_unique<std::barrier<>>(64));
    blk.wbuf.assign(((nthr + 63) / 64) * 64, 0);
    std::vector<unsigned char> dyn(shmem + 64, 0xff);
    blk.dyn = reinterpret_cast<unsigned char *>((reinterpret_cast<uintptr_t>(dyn.data()) + 63) & ~uintptr_t(63));
    std::vector<std::function<void()>> fs(nthr);
    for (unsigned t = 0; t < nthr; ++t)
      fs[t] = [&, t] {
        threadIdx = dim3(t);
        blockIdx = dim3(bi);
        blockDim = b;
        gridDim = g;
        emu_blk = &blk;
        k(args...);
      };
    std::vector<std::thread> th;
    th.reserve(nthr);
    for (unsigned t = 0; t < nthr; ++t) th.emplace_back(emu_thread_main, &fs[t]);
    for (auto &x : th) x.join();
  }
}
#define hipLaunchKernelGGL(kern, grid, block, shmem, stream, ...) \
  emu_launch(kern, dim3(grid), dim3(block), (size_t)(shmem), __VA_ARGS__)
