// Minimal HIP-on-CPU shim used only by the host bounds check (tests/test_cpu_emu.py):
// the library sources are compiled for the host under AddressSanitizer and
// every kernel launch runs all blocks and threads one after another.  MFMA
// results are not emulated (no address in the kernels depends on data), so
// only the memory accesses are meaningful.
#pragma once
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <cstdint>
#include <sanitizer/asan_interface.h>
struct dim3 { unsigned x, y, z; dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {} };
struct uint3e { unsigned x, y, z; };
extern thread_local uint3e threadIdx, blockIdx, blockDim, gridDim;
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(x)
// occupancy hints apply to GPU kernels only
#define amdgpu_waves_per_eu(...) unused
#define __shared__ static
#define __align__(x) __attribute__((aligned(x)))
inline void __syncthreads() {}
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorNotSupported = 3 };
typedef void* hipStream_t;
typedef void* hipEvent_t;
typedef void* hipGraph_t;
typedef void* hipGraphExec_t;
enum { hipStreamNonBlocking = 1, hipStreamCaptureModeThreadLocal = 1 };
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = malloc(1); return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { free(s); return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, int) { return hipSuccess; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = malloc(1); return hipSuccess; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, void*, void*, size_t) { *e = malloc(1); return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) { free(g); return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) { free(e); return hipSuccess; }
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
inline const char* hipGetErrorString(hipError_t) { return "emu"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
// host build: a __device__ array is an ordinary global, its address the symbol's
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = (void*)sym; return hipSuccess; }
enum { hipDeviceAttributeMultiprocessorCount = 1 };
inline hipError_t hipDeviceGetAttribute(int* v, int, int) { *v = 256; return hipSuccess; }
template <typename F>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* nb, F, int, size_t) { *nb = 1; return hipSuccess; }
inline hipError_t hipMalloc(void** p, size_t n) { *p = malloc(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
template <typename T> inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
inline hipError_t hipFree(void* p) { free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = malloc(1); return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { free(e); return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* t, hipEvent_t, hipEvent_t) { *t = 0; return hipSuccess; }
typedef float emu_f4 __attribute__((ext_vector_type(4)));
typedef double emu_d4 __attribute__((ext_vector_type(4)));
inline emu_f4 emu_mfma_f(float a, float b, emu_f4 c) { return c + a * b; }
inline emu_d4 emu_mfma_d(double a, double b, emu_d4 c) { return c + a * b; }
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) emu_mfma_f(a, b, c)
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) emu_mfma_d(a, b, c)
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, x, y, z) (c)
// global-to-LDS copy: lane l's bytes land at dst + size * l
inline void emu_global_load_lds(const void* src, void* dst, unsigned size) {
  memcpy((char*)dst + (size_t)(threadIdx.x & 63) * size, src, size);
}
#define __builtin_amdgcn_global_load_lds(src, dst, size, off, aux) \
  emu_global_load_lds((const void*)(src), (void*)(dst), (size))
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)
#define __builtin_amdgcn_s_barrier() ((void)0)
#define __builtin_amdgcn_readfirstlane(x) (x)
// threads run one after another: a lane exchange returns the lane's own value
// (the emulator checks memory accesses, not the values)
template <typename T> inline T __shfl_xor(T v, int, int = 64) { return v; }
#define __builtin_amdgcn_sched_group_barrier(a, b, c) ((void)0)
inline unsigned __float_as_uint(float x) { unsigned u; memcpy(&u, &x, 4); return u; }
inline float __uint_as_float(unsigned u) { float x; memcpy(&x, &u, 4); return x; }
extern const char* g_emu_kernel;
template <typename K, typename... A>
inline void emu_launch(const char* name, K kernel, dim3 g, dim3 b, A... args) {
  g_emu_kernel = name;
  // a real dispatch packet holds each extent in work-items as 32 bits: a
  // launch past that would wrap on the device, so it stops the run here
  if ((unsigned long long)g.x * b.x >= (1ull << 32) || (unsigned long long)g.y * b.y >= (1ull << 32) ||
      (unsigned long long)g.z * b.z >= (1ull << 32)) {
    fprintf(stderr, "emu: %s launched with a grid past 2^32 work-items\n", name);
    abort();
  }
  gridDim = {g.x, g.y, g.z}; blockDim = {b.x, b.y, b.z};
  for (unsigned bz = 0; bz < g.z; ++bz) for (unsigned by = 0; by < g.y; ++by) for (unsigned bx = 0; bx < g.x; ++bx)
    for (unsigned tz = 0; tz < b.z; ++tz) for (unsigned ty = 0; ty < b.y; ++ty) for (unsigned tx = 0; tx < b.x; ++tx) {
      blockIdx = {bx, by, bz}; threadIdx = {tx, ty, tz};
      kernel(args...);
    }
}
#define hipLaunchKernelGGL(k, g, b, shm, st, ...) emu_launch(#k, k, dim3(g), dim3(b), __VA_ARGS__)
