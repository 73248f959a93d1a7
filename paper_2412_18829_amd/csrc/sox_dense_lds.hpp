// LDS-staged float32 NT GEMM for the A step (the copy machinery of the
// LDS-staged fused kernel, sox_fused_lds.hpp, with one product):
//
//   C[row][col] = sum_k A[row][k] * B[col][k]
//
// A workgroup of four wavefronts owns a 128 x 128 block of C, each
// wavefront 64 x 64 (4 x 4 tiles of v_mfma_f32_16x16x4f32).  K runs in
// stages of 16 values (64 bytes per row): the stage's 128-row panels of A
// and B are copied straight into a ring of five LDS buffers four stages
// ahead of the MFMAs, with the same swizzled 64-byte rows, fence-free
// barriers, exact copy counting and buffer reuse rule as the fused kernel.  K must be a
// multiple of 16; rows and columns past M and N are read from the last
// valid row and not stored.
//
// blockIdx.y runs over a batch (operand and output strides sA, sB, sC).
// Rows come in groups (the A step: group = tau, rows = v padded to nP):
// row r is row r % rgroup of group r / rgroup, stored only when
// r % rgroup < rvalid, at C + group c_gstride + (r % rgroup) ldc + col.
// With Chi set the result x is stored as bf16 hi = bf16(x) and
// lo = bf16(x - hi) at the same offsets of Chi and Clo instead of C; with
// C64 set it is stored (or, with accumulate, added) in float64.
#pragma once

#include <type_traits>

#include "sox_common.hpp"
#include "sox_fused_lds.hpp"

namespace sox {

struct DenseLdsArgs {
  const float* A;
  const float* B;
  long lda, ldb;        // row strides (elements)
  int M, N, K;
  int rgroup, rvalid;   // row groups (see above)
  long c_gstride, ldc;  // C offsets (elements)
  float* C;
  bf16_t* Chi;
  bf16_t* Clo;
  long sA, sB, sC;      // batch strides (elements; blockIdx.y is the batch)
  int tiles_m, tiles_n;
  double* C64 = nullptr;  // float64 output instead of C (same offsets)
  int accumulate = 0;     // float64 output only: C64 += result
};

__global__ __launch_bounds__(256) void dense_lds_f32_kernel(const DenseLdsArgs p) {
  // [buffer][plane: A rows, B rows][row * 4 + swizzled segment]
  __shared__ u32x4 lds[kLdsBufs][2][kLdsPieces];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int tm = bid % p.tiles_m;  // row tiles fastest: they share the B panel
  const int tn = bid / p.tiles_m;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15;
  const int g = lane >> 4;
  const int M0 = tm * kLdsTile, N0 = tn * kLdsTile;
  const long bat = blockIdx.y;

  // copies: instruction h of wavefront w fills pieces 64 c .. 64 c + 63 (c = w + 4 h)
  const char* srca[2];
  const char* srcb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = wave + 4 * h;
    const int row = 16 * c + (lane >> 2);
    const int seg = (lane & 3) ^ ((row >> 1) & 3);
    const int ra = M0 + row < p.M ? M0 + row : p.M - 1;
    const int rb = N0 + row < p.N ? N0 + row : p.N - 1;
    srca[h] = (const char*)(p.A + bat * p.sA + (long)ra * p.lda) + 16 * seg;
    srcb[h] = (const char*)(p.B + bat * p.sB + (long)rb * p.ldb) + 16 * seg;
  }
  int sa[4], sb[4];
  const int sw = g ^ ((li >> 1) & 3);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sa[i] = ((wave >> 1) * 64 + 16 * i + li) * 4 + sw;
    sb[i] = ((wave & 1) * 64 + 16 * i + li) * 4 + sw;
  }
  const int KC = p.K / 16;
  const int c0 = 64 * wave, c1 = 64 * (wave + 4);
  int ck = 0;  // next chunk to copy, held at the last one past the end
  auto copy_stage = [&](int b) {
    const long ko = (long)ck * 64;
    global_to_lds16(srca[0] + ko, &lds[b][0][c0]);
    global_to_lds16(srca[1] + ko, &lds[b][0][c1]);
    global_to_lds16(srcb[0] + ko, &lds[b][1][c0]);
    global_to_lds16(srcb[1] + ko, &lds[b][1][c1]);
    ck += ck + 1 < KC ? 1 : 0;
  };
  auto frags = [&](int b, f32x4* fa, f32x4* fb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      fa[i] = __builtin_bit_cast(f32x4, lds[b][0][sa[i]]);
      fb[i] = __builtin_bit_cast(f32x4, lds[b][1][sb[i]]);
    }
  };
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = zero4<float>();
  auto mfma_stage = [&](const f32x4* fa, const f32x4* fb) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma16x16x4(fa[i][m], fb[j][m], acc[i][j]);
  };

  // Stage s (buffer s % 5): copy stage s + 4 into the buffer of stage s - 1
  // (whose fragments every wavefront consumed before the barrier that ended
  // stage s - 1), read the fragments of stage s + 1, MFMAs of stage s, wait
  // for the own copies of stage s + 2, barrier.
  copy_stage(0);
  copy_stage(1);
  copy_stage(2);
  copy_stage(3);
  wait_vm<8>();  // stages 0 and 1 landed
  barrier_nofence();
  f32x4 fa0[4], fb0[4], fa1[4], fb1[4];
  frags(0, fa0, fb0);
  int b1 = 1;  // buffer of stage s + 1
  auto next = [](int x) { return x + 1 == kLdsBufs ? 0 : x + 1; };
  auto back2 = [](int x) { return x >= 2 ? x - 2 : x + kLdsBufs - 2; };
  for (int s = 0; s < KC; s += 2) {
    copy_stage(back2(b1));
    frags(b1, fa1, fb1);
    mfma_stage(fa0, fb0);
    wait_vm<8>();
    barrier_nofence();
    b1 = next(b1);
    if (s + 1 < KC) {
      copy_stage(back2(b1));
      frags(b1, fa0, fb0);
      mfma_stage(fa1, fb1);
      wait_vm<8>();
      barrier_nofence();
      b1 = next(b1);
    }
  }
  wait_vm<0>();  // the repeated copies past the end

  const int Rw = M0 + (wave >> 1) * 64, Cw = N0 + (wave & 1) * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = Rw + 16 * i + 4 * g + r;
      const int grp = row / p.rgroup, rin = row - grp * p.rgroup;
      if (row >= p.M || rin >= p.rvalid) continue;
      const long base = bat * p.sC + (long)grp * p.c_gstride + (long)rin * p.ldc;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = Cw + 16 * j + li;
        if (col >= p.N) continue;
        const float x = acc[i][j][r];
        if (p.Chi) {
          const bf16_t hgh = f32_to_bf16(x);
          p.Chi[base + col] = hgh;
          p.Clo[base + col] = f32_to_bf16(x - bf16_to_f32(hgh));
        } else if (p.C64) {
          p.C64[base + col] = p.accumulate ? p.C64[base + col] + (double)x : (double)x;
        } else {
          p.C[base + col] = x;
        }
      }
    }
}

inline hipError_t launch_dense_lds_f32(DenseLdsArgs a, int batch, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || batch <= 0) return hipSuccess;
  if (batch > 65535) return hipErrorInvalidValue;
  if (a.K % 16 != 0 || a.K <= 0 || a.rgroup <= 0 || (a.Chi && !a.Clo) ||
      (!a.Chi && !a.C && !a.C64) || (a.accumulate && !a.C64))
    return hipErrorInvalidValue;
  a.tiles_m = (a.M + kLdsTile - 1) / kLdsTile;
  a.tiles_n = (a.N + kLdsTile - 1) / kLdsTile;
  const long nb = (long)a.tiles_m * a.tiles_n;
  if (nb > (1L << 31) - 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dense_lds_f32_kernel, dim3((unsigned)nb, (unsigned)batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace sox
