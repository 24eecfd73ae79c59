// CPU stand-in for <hip/hip_runtime.h>, used only by the test-side kernel
// executor (tests/emu).  Each GPU thread runs as a cooperative fiber; wave
// intrinsics and __syncthreads are synchronisation points resolved when every
// lane of the wave (or every thread of the block) has reached them, so the
// kernel source runs unchanged on the CPU with lockstep semantics at those
// points.  Device memory is host memory.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __shared__ static __attribute__((section("emu_lds"), used))
#define __launch_bounds__(...)
#define __constant__ static const

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint2 {
  uint32_t x, y;
};
struct uint4 {
  uint32_t x, y, z, w;
};

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorNotReady = 600 };
typedef void *hipStream_t;
typedef void *hipEvent_t;
typedef void *hipGraph_t;
typedef void *hipGraphExec_t;
enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1, hipStreamCaptureModeRelaxed = 2 };
enum { hipErrorNotSupported = 801 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyHostToHost };
#define hipHostMallocDefault 0
#define hipEventDisableTiming 0
struct hipDeviceProp_t {
  int multiProcessorCount;
  size_t maxSharedMemoryPerMultiProcessor;
};

// ---- executor interface (tests/emu/emu_rt.cpp)
extern "C" {
uint64_t emu_wave_sync(int kind, uint64_t v, uint64_t aux);
void emu_block_sync(void);
unsigned emu_tid(void);
unsigned emu_bid(void);
unsigned emu_bdim(void);
unsigned emu_gdim(void);
void emu_run_grid(void (*fn)(void *), void *arg, unsigned grid, unsigned block);
int emu_n_cu(void);
}
enum { EMU_BALLOT = 1, EMU_READLANE = 2, EMU_FIRSTLANE = 3, EMU_SHFL_XOR = 4, EMU_WAVEBAR = 5, EMU_WRITELANE = 6,
       EMU_SHFL = 7 };

template <typename F>
static void emu_tramp(void *p) {
  (*static_cast<F *>(p))();
}
template <typename F>
static void emu_launch(F f, dim3 g, dim3 b) {
  emu_run_grid(&emu_tramp<F>, &f, g.x, b.x);
}
#define hipLaunchKernelGGL(k, g, b, sh, st, ...) emu_launch([=]() { k(__VA_ARGS__); }, dim3(g), dim3(b))

#define threadIdx (dim3(emu_tid()))
#define blockIdx (dim3(emu_bid()))
#define blockDim (dim3(emu_bdim()))
#define gridDim (dim3(emu_gdim()))

static inline void __syncthreads() { emu_block_sync(); }
static inline unsigned __lane_id() { return emu_tid() & 63u; }
static inline unsigned long long __ballot(int p) { return emu_wave_sync(EMU_BALLOT, p != 0, 0); }
static inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
static inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
template <typename T>
static inline T __shfl_xor(T v, int o) {
  return (T)emu_wave_sync(EMU_SHFL_XOR, (uint64_t)v, (uint64_t)o);
}
template <typename T>
static inline T __shfl(T v, int src) {
  return (T)emu_wave_sync(EMU_SHFL, (uint64_t)(uint32_t)v, (uint64_t)(uint32_t)src);
}
// writelane(value, lane, old): lane `lane` takes the (uniform) value, the others keep old
static inline int emu_writelane(uint32_t val, uint32_t l, uint32_t old) {
  return (int)emu_wave_sync(EMU_WRITELANE, old, ((uint64_t)val << 32) | (l & 63u));
}
#define __builtin_amdgcn_writelane(v, l, o) emu_writelane((uint32_t)(v), (uint32_t)(l), (uint32_t)(o))
static inline uint32_t __builtin_amdgcn_alignbit(uint32_t hi, uint32_t lo, uint32_t s) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> (s & 31u));
}
#define __builtin_amdgcn_readlane(v, l) ((int)emu_wave_sync(EMU_READLANE, (uint32_t)(v), (uint64_t)(l)))
// ds_bpermute(byte address, v): the v of lane (address / 4) mod 64
#define __builtin_amdgcn_ds_bpermute(a, v) \
  ((int)emu_wave_sync(EMU_SHFL, (uint64_t)(uint32_t)(v), (uint64_t)(((uint32_t)(a) >> 2) & 63u)))
#define __builtin_amdgcn_readfirstlane(v) ((int)emu_wave_sync(EMU_FIRSTLANE, (uint32_t)(v), 0))
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)
#define __builtin_amdgcn_wave_barrier() ((void)emu_wave_sync(EMU_WAVEBAR, 0, 0))

template <typename T>
static inline T atomicAdd(T *p, T v) {
  T o = *p;
  *p = o + v;
  return o;
}
template <typename T>
static inline T atomicMin(T *p, T v) {
  T o = *p;
  if (v < o) *p = v;
  return o;
}
template <typename T>
static inline T atomicXor(T *p, T v) {
  T o = *p;
  *p = o ^ v;
  return o;
}
template <typename T, typename U, typename V>
static inline T atomicCAS(T *p, U c, V v) {
  T o = *p;
  if (o == (T)c) *p = (T)v;
  return o;
}
#define __hip_atomic_load(p, order, scope) (*(p))
using std::max;
using std::min;

// ---- runtime API on host memory
static inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
  memcpy(d, s, n);
  return hipSuccess;
}
static inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
  memcpy(d, s, n);
  return hipSuccess;
}
static inline hipError_t hipHostMalloc(void **p, size_t n, int) {
  *p = malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorInvalidValue;
}
static inline hipError_t hipHostFree(void *p) {
  free(p);
  return hipSuccess;
}
static inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, int) {
  *e = (void *)1;
  return hipSuccess;
}
static inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
static inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
static inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
static inline hipError_t hipEventCreate(hipEvent_t *e) {
  *e = (void *)1;
  return hipSuccess;
}
static inline hipError_t hipEventElapsedTime(float *t, hipEvent_t, hipEvent_t) {
  *t = 0.f;
  return hipSuccess;
}
static inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
static inline hipError_t hipStreamQuery(hipStream_t) { return hipSuccess; }
static inline hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
static inline hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) {
  p->multiProcessorCount = emu_n_cu();
  p->maxSharedMemoryPerMultiProcessor = 160 * 1024;
  return hipSuccess;
}
static inline const char *hipGetErrorString(hipError_t) { return "emulated"; }
static inline hipError_t hipGetLastError() { return hipSuccess; }

// graphs are not emulated: capture fails, so the graph entry point reports it
static inline hipError_t hipStreamBeginCapture(hipStream_t, int) { return hipErrorNotSupported; }
static inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
  *g = nullptr;
  return hipErrorNotSupported;
}
static inline hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, void *, char *, size_t) {
  return hipErrorNotSupported;
}
static inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
static inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
static inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }

// streams and events of the serving loop: work runs synchronously at launch,
// so every stream is idle and every event has passed
#define hipStreamNonBlocking 1
static inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = (void *)1;
  return hipSuccess;
}
static inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
static inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
// static device arrays are host arrays; their "device address" is the host one
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))
#define hipErrorInvalidDevice 101
static inline hipError_t hipGetSymbolAddress(void **p, const void *sym) {
  *p = (void *)sym;
  return hipSuccess;
}
static inline hipError_t hipMalloc(void **p, size_t n) {
  *p = aligned_alloc(256, (n + 255) / 256 * 256);
  return *p ? hipSuccess : hipErrorInvalidValue;
}
static inline hipError_t hipFree(void *p) {
  free(p);
  return hipSuccess;
}
