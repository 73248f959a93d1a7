// Shared device helpers for the gfx950 SOX kernels: vector types, the
// 16x16x4 MFMA wrappers used by every contraction, and the XCD-aware
// block-to-tile remap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sox {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct vec4;
template <> struct vec4<float> { typedef f32x4 type; };
template <> struct vec4<double> { typedef f64x4 type; };
template <typename T> using vec4_t = typename vec4<T>::type;

// D = A*B + C on one 16x16 tile with a K-depth of 4.  Operand layout (both
// precisions): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].  The
// accumulator element r of lane l holds C[acc_row<T>(l / 16, r)][l % 16]:
// row 4 (l/16) + r for float32 and row (l/16) + 4 r for float64 (measured
// on gfx950 with a row/column-tagging probe).
__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// bfloat16 operands: 8 per lane and k chunks of 32 (v_mfma_f32_16x16x32_bf16).
// Lane l supplies A[l % 16][8 (l/16) + e] and B[8 (l/16) + e][l % 16], e = 0..7;
// the float32 accumulator has the same layout as the 16x16x4 float32 one.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short bf16_t;  // storage of one bfloat16

__device__ __forceinline__ f32x4 mfma16x16x32bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 16 bytes per lane from global memory straight into LDS (gfx950
// global_load_lds_dwordx4): the bytes of lane l land at lds + 16 l, so lds
// must be the same for every lane of the wavefront.  Completion is tracked
// by the vector-memory counter (wait_vm_all), not by the LDS counter.
__device__ __forceinline__ void global_to_lds16(const void* src, void* lds) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}
// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima)
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// s_waitcnt vmcnt(N) with the other counters at their maxima
template <int N> __device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt holds six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}

// Workgroup barrier without a memory fence.  __syncthreads() fences, and a
// fence makes every wavefront wait for all of its global-to-LDS copies
// still in flight; here the caller waits explicitly for the copies the
// other wavefronts are about to read.  The empty asm statements keep the
// compiler from moving memory accesses across the barrier.
__device__ __forceinline__ void barrier_nofence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Round-to-nearest-even float32 -> bfloat16 (one v_cvt_pk_bf16_f32 on
// gfx950) and back.
__device__ __forceinline__ bf16_t f32_to_bf16(float x) {
  return __builtin_bit_cast(bf16_t, (__bf16)x);
}
__device__ __forceinline__ float bf16_to_f32(bf16_t h) { return __uint_as_float((unsigned)h << 16); }

template <typename T> __device__ __forceinline__ int acc_row(int g, int r);
template <> __device__ __forceinline__ int acc_row<float>(int g, int r) { return 4 * g + r; }
template <> __device__ __forceinline__ int acc_row<double>(int g, int r) { return g + 4 * r; }

template <typename T> __device__ __forceinline__ vec4_t<T> zero4() {
  vec4_t<T> z;
  z[0] = T(0); z[1] = T(0); z[2] = T(0); z[3] = T(0);
  return z;
}

// Consecutive workgroup ids are dispatched round-robin over the 8 XCDs of
// the chip, each with its own L2.  Give every XCD a contiguous range of
// logical tiles so that tiles that share operands (same tau, same P panel)
// run behind the same L2.  Bijective on [0, nblocks).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int NX = 8;
  const int per = nblocks / NX;
  const int rem = nblocks % NX;
  const int xcd = bid % NX;
  const int local = bid / NX;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Flat elementwise launches.  A dispatch packet carries the grid size in
// work-items as a 32-bit value, so such a launch is capped at kGrid1dMax
// workgroups of 256 and its kernel strides over the rest of the range.
constexpr long kGrid1dMax = 1L << 20;
inline dim3 grid1d(long count) {
  long b = (count + 255) / 256;
  if (b < 1) b = 1;
  return dim3((unsigned)(b < kGrid1dMax ? b : kGrid1dMax));
}
// A dispatch packet carries each grid extent in work-items (workgroups times
// the workgroup size) as a 32-bit value, so an extent of 2^32 work-items or
// more wraps.  Every tiled launcher refuses such a grid (hipErrorInvalidValue)
// instead of launching it.
inline bool grid_fits(long wg_x, long threads, long wg_y = 1, long wg_z = 1) {
  constexpr long kLim = 1L << 32;
  return wg_x >= 1 && wg_y >= 1 && wg_z >= 1 && threads >= 1 && wg_x * threads < kLim &&
         wg_y < kLim && wg_z < kLim;
}

#define SOX_FOR_FLAT(i, count)                                                   \
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (long)(count); \
       i += (long)gridDim.x * blockDim.x)

}  // namespace sox
