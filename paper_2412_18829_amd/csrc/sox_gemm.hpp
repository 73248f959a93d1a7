// Generic batched MFMA GEMM used by the smaller contractions of the SOX
// chain (U-contraction, half projections, the A step, back-transform,
// G(tau) synthesis).  The operand access is supplied by a problem struct so
// that the same tile loop serves every layout:
//
//   C[b][i][j] = sum_k A(b, i, k) * B(b, j, k)
//
//   Prob::loadA4(b, i, k) -> vec4 of A(b, i, k .. k+3)   (zero outside range)
//   Prob::loadB4(b, j, k) -> vec4 of B(b, j, k .. k+3)
//   Prob::store(b, i, j, value)
//   Prob::M, Prob::N (store extents), Prob::K (multiple of 4 not required:
//   the loaders return zeros past the true depth)
//
// Workgroup = 4 wavefronts arranged WGR x WGC; each wavefront owns a
// (16 RB) x (16 CB) block of 16x16 MFMA tiles.  K advances in chunks of 16:
// lane l loads A[i = l%16][k0 + 4(l/16) + m], m = 0..3, as one vec4 and the
// same k pattern for B, so MFMA m sees the k-permutation k0 + 4g + m in both
// operands (a contraction is blind to the order of its k terms).
#pragma once

#include "sox_common.hpp"

namespace sox {

template <class Prob, typename Tacc, int WGR, int WGC, int RB, int CB>
__global__ __launch_bounds__(256) void gemm_kernel(const Prob p) {
  static_assert(WGR * WGC == 4, "four wavefronts per workgroup");
  using V4 = vec4_t<Tacc>;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15;
  const int g = lane >> 4;
  const int b = blockIdx.z;
  const int row0 = blockIdx.y * (WGR * RB * 16) + (wave / WGC) * (RB * 16);
  const int col0 = blockIdx.x * (WGC * CB * 16) + (wave % WGC) * (CB * 16);
  if (row0 >= p.M || col0 >= p.N) return;

  V4 acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = zero4<Tacc>();

  for (int k0 = 0; k0 < p.K; k0 += 16) {
    V4 a[RB], bb[CB];
#pragma unroll
    for (int i = 0; i < RB; ++i) a[i] = p.loadA4(b, row0 + 16 * i + li, k0 + 4 * g);
#pragma unroll
    for (int j = 0; j < CB; ++j) bb[j] = p.loadB4(b, col0 + 16 * j + li, k0 + 4 * g);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = mfma16x16x4(a[i][m], bb[j][m], acc[i][j]);
  }

#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + 16 * i + acc_row<Tacc>(g, r);
        const int col = col0 + 16 * j + li;
        if (row < p.M && col < p.N) p.store(b, row, col, acc[i][j][r]);
      }
}

template <class Prob, typename Tacc, int WGR, int WGC, int RB, int CB>
inline hipError_t launch_gemm(const Prob& p, int batch, hipStream_t s) {
  constexpr int TM = WGR * RB * 16;
  constexpr int TN = WGC * CB * 16;
  if (p.M <= 0 || p.N <= 0 || batch <= 0) return hipSuccess;
  const long gx = ((long)p.N + TN - 1) / TN, gy = ((long)p.M + TM - 1) / TM;
  if (!grid_fits(gx, 256, gy, batch)) return hipErrorInvalidValue;
  dim3 grid((unsigned)gx, (unsigned)gy, batch);
  hipLaunchKernelGGL((gemm_kernel<Prob, Tacc, WGR, WGC, RB, CB>), grid, dim3(256), 0, s, p);
  return hipGetLastError();
}

// masked scalar helpers ------------------------------------------------------
template <typename Tacc, typename Tsrc>
__device__ __forceinline__ vec4_t<Tacc> load4_strided(const Tsrc* base, long stride, int k,
                                                      int kmax) {
  vec4_t<Tacc> v;
#pragma unroll
  for (int m = 0; m < 4; ++m) v[m] = (k + m < kmax) ? Tacc(base[(long)(k + m) * stride]) : Tacc(0);
  return v;
}

}  // namespace sox
