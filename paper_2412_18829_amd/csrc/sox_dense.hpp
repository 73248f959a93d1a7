// Dense batched NT GEMM on MFMA for operands already laid out K-contiguous
// and zero padded along K (the big contractions: the A step and the
// W(Omega) GG(Omega) product):
//
//   C[b][i][j] (+)= alpha * sum_k A[b][i][k] * B[b][j][k]
//
// K must be a multiple of 16 and every row read must hold K values.  Rows
// i >= M (or j >= N) are read from the last valid row and zeroed, and are
// not stored, so M and N need not fill the tile.  The output is stored
// row-major (C[i*ldc + j]) or transposed (C[j*ldc + i]); in the transposed
// form each lane writes its four consecutive accumulator rows with one
// vector store (float32 rows 4g..4g+3 are consecutive).
//
// Schedule as in the fused kernel: the next 16-deep chunk is loaded, a
// scheduling barrier keeps those loads ahead of the current chunk's MFMAs,
// and the register hand-over (which waits for the loads) follows them.
#pragma once

#include "sox_common.hpp"

namespace sox {

template <typename T, typename TC> struct DenseArgs {
  const T* A;
  const T* B;
  TC* C;
  long lda, ldb, ldc;
  long sA, sB, sC;  // batch strides
  int M, N, K;
  int tiles_m, tiles_n;
  T alpha;
  int transposed;   // store C[j][i]
  int accumulate;   // C += result
  // row tiles fastest in the workgroup order: the row tiles sharing one B
  // column panel run back to back (same XCD, same L2) when B is the large
  // operand
  int m_fast = 0;
  // split-precision output (float32 results only, no accumulate): when set,
  // C is not written; each result x goes to Chi = bf16(x) and
  // Clo = bf16(x - Chi) at the offset C would have had
  bf16_t* Chi = nullptr;
  bf16_t* Clo = nullptr;
};

template <typename T, typename TC, int WGR, int WGC, int RB, int CB>
__global__ __launch_bounds__(256) void dense_nt_kernel(const DenseArgs<T, TC> p) {
  static_assert(WGR * WGC == 4, "four wavefronts per workgroup");
  using V4 = vec4_t<T>;
  const int b = blockIdx.y;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int tn = p.m_fast ? bid / p.tiles_m : bid % p.tiles_n;
  const int tm = p.m_fast ? bid % p.tiles_m : bid / p.tiles_n;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15;
  const int g = lane >> 4;
  const int row0 = tm * (WGR * RB * 16) + (wave / WGC) * (RB * 16);
  const int col0 = tn * (WGC * CB * 16) + (wave % WGC) * (CB * 16);

  const T* Ab = p.A + (long)b * p.sA + 4 * g;
  const T* Bb = p.B + (long)b * p.sB + 4 * g;
  const T* arow[RB];
  const T* brow[CB];
  bool aok[RB], bok[CB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int r = row0 + 16 * i + li;
    aok[i] = r < p.M;
    arow[i] = Ab + (long)(aok[i] ? r : p.M - 1) * p.lda;
  }
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int c = col0 + 16 * j + li;
    bok[j] = c < p.N;
    brow[j] = Bb + (long)(bok[j] ? c : p.N - 1) * p.ldb;
  }

  V4 acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = zero4<T>();

  V4 a[RB], bb[CB];
#pragma unroll
  for (int i = 0; i < RB; ++i) a[i] = aok[i] ? *(const V4*)(arow[i]) : zero4<T>();
#pragma unroll
  for (int j = 0; j < CB; ++j) bb[j] = bok[j] ? *(const V4*)(brow[j]) : zero4<T>();

  const int KC = p.K >> 4;
  for (int kc = 0; kc < KC; ++kc) {
    const int kn = (kc + 1 < KC) ? kc + 1 : kc;
    const long ko = (long)kn * 16;
    V4 an[RB], bn[CB];
#pragma unroll
    for (int i = 0; i < RB; ++i) an[i] = *(const V4*)(arow[i] + ko);
#pragma unroll
    for (int j = 0; j < CB; ++j) bn[j] = *(const V4*)(brow[j] + ko);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = mfma16x16x4(a[i][m], bb[j][m], acc[i][j]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < RB; ++i) a[i] = aok[i] ? an[i] : zero4<T>();
#pragma unroll
    for (int j = 0; j < CB; ++j) bb[j] = bok[j] ? bn[j] : zero4<T>();
  }

  TC* Cb = p.C + (long)b * p.sC;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + 16 * i + acc_row<T>(g, r);
        const int col = col0 + 16 * j + li;
        if (row < p.M && col < p.N) {
          const long off = p.transposed ? (long)col * p.ldc + row : (long)row * p.ldc + col;
          TC v = TC(p.alpha * acc[i][j][r]);
          if (p.Chi) {
            const float x = (float)v;
            const bf16_t h = f32_to_bf16(x);
            p.Chi[(long)b * p.sC + off] = h;
            p.Clo[(long)b * p.sC + off] = f32_to_bf16(x - bf16_to_f32(h));
          } else {
            if (p.accumulate) v += Cb[off];
            Cb[off] = v;
          }
        }
      }
}

template <typename T, typename TC, int WGR, int WGC, int RB, int CB>
inline hipError_t launch_dense(DenseArgs<T, TC> a, int batch, hipStream_t s) {
  constexpr int TM = WGR * RB * 16;
  constexpr int TN = WGC * CB * 16;
  if (a.M <= 0 || a.N <= 0 || batch <= 0) return hipSuccess;
  if (a.K % 16 != 0) return hipErrorInvalidValue;
  if (a.Chi && (sizeof(TC) != 4 || !a.Clo || a.accumulate)) return hipErrorInvalidValue;
  a.tiles_m = (a.M + TM - 1) / TM;
  a.tiles_n = (a.N + TN - 1) / TN;
  const long gx = (long)a.tiles_m * a.tiles_n;
  if (!grid_fits(gx, 256, batch)) return hipErrorInvalidValue;
  dim3 grid((unsigned)gx, batch);
  hipLaunchKernelGGL((dense_nt_kernel<T, TC, WGR, WGC, RB, CB>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace sox
