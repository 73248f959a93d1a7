// LDS-staged float32 NT GEMM for the A step, the U-contraction and
// W(Omega) GG(Omega) (the copy machinery of the LDS-staged fused kernel,
// sox_fused_lds.hpp, with one product):
//
//   C[row][col] = sum_k A[row][k] * B[col][k]
//
// A workgroup of four wavefronts computes about tpw of the 128 x 128 blocks
// of C (block b of the grid's w workgroups: b, b + w, b + 2 w, ...; row
// blocks fastest), each wavefront 64 x 64 of a block (4 x 4 tiles
// of v_mfma_f32_16x16x4f32).  K runs in stages of 16 values (64 bytes per
// row): the stage's 128-row panels of A and B are copied straight into a
// ring of five LDS buffers four stages ahead of the MFMAs, with the same
// swizzled 64-byte rows, fence-free barriers, exact copy counting and
// buffer reuse rule as the fused kernel.  The stages of a workgroup's
// blocks run back to back through the ring, so with a short K (the A step)
// the copies of the next block are in flight while the current block's
// MFMAs run and its results are stored.  K must be a multiple of 16; rows
// and columns past M and N are read from the last valid row and not
// stored.
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

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

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
  int tpw;              // output tiles per workgroup (set by the launcher)
  int vec;              // vector stores: 0 none, 1 four columns, 2 paired split planes (launcher)
  double* C64 = nullptr;  // float64 output instead of C (same offsets)
  int accumulate = 0;     // float64 output only: C64 += result
  // split addressing (defaults: plain rows and columns): B row r sits at
  // (r / bsplit) bhi + (r % bsplit) ldb, C column c at (c / csplit) chi + c % csplit
  int bsplit = 1 << 30;
  long bhi = 0;
  int csplit = 1 << 30;
  long chi = 0;
};

template <bool MULTI>
__global__ __launch_bounds__(256) void dense_lds_f32_kernel(const DenseLdsArgs p) {
  // [buffer][plane: A rows, B rows][row * 4 + swizzled segment]
  __shared__ u32x4 lds[kLdsBufs][2][kLdsPieces];
  // tiles wid, wid + nwg, wid + 2 nwg, ...: the workgroups resident at one
  // time work on neighbouring tiles, as with one tile per workgroup
  const long ntiles = (long)p.tiles_m * p.tiles_n;
  const long nwg = gridDim.x;
  const long wid = xcd_remap(blockIdx.x, gridDim.x);
  const int ntl = MULTI ? (int)((ntiles - wid + nwg - 1) / nwg) : 1;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15;
  const int g = lane >> 4;
  const long bat = blockIdx.y;
  const int KC = p.K / 16;
  const int nst = ntl * KC;  // stages of every tile of this workgroup, back to back

  // copies: instruction h of wavefront w fills pieces 64 c .. 64 c + 63 (c =
  // w + 4 h) from the rows of the tile under the copy cursor
  const char* srca[2];
  const char* srcb[2];
  auto set_src = [&](long tile) {
    const int M0 = (int)(tile % p.tiles_m) * kLdsTile;  // row tiles fastest: they share B
    const int N0 = (int)(tile / p.tiles_m) * kLdsTile;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = wave + 4 * h;
      const int row = 16 * c + (lane >> 2);
      const int seg = (lane & 3) ^ ((row >> 1) & 3);
      const int ra = M0 + row < p.M ? M0 + row : p.M - 1;
      const int rb = N0 + row < p.N ? N0 + row : p.N - 1;
      srca[h] = (const char*)(p.A + bat * p.sA + (long)ra * p.lda) + 16 * seg;
      srcb[h] = (const char*)(p.B + bat * p.sB + (long)(rb / p.bsplit) * p.bhi +
                              (long)(rb % p.bsplit) * p.ldb) + 16 * seg;
    }
  };
  set_src(wid);
  int sa[4], sb[4];
  const int sw = g ^ ((li >> 1) & 3);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sa[i] = ((wave >> 1) * 64 + 16 * i + li) * 4 + sw;
    sb[i] = ((wave & 1) * 64 + 16 * i + li) * 4 + sw;
  }
  const int c0 = 64 * wave, c1 = 64 * (wave + 4);
  // copy cursor: tile ct, chunk ck, stage cs; held at the last stage once
  // every stage is under way
  int ct = 0, ck = 0, cs = 0;
  auto copy_stage = [&](int b) {
    const long ko = (long)ck * 64;
    global_to_lds16(srca[0] + ko, &lds[b][0][c0]);
    global_to_lds16(srca[1] + ko, &lds[b][0][c1]);
    global_to_lds16(srcb[0] + ko, &lds[b][1][c0]);
    global_to_lds16(srcb[1] + ko, &lds[b][1][c1]);
    if constexpr (MULTI) {
      if (cs + 1 < nst) {
        ++cs;
        if (++ck == KC) {
          ck = 0;
          set_src(wid + ++ct * nwg);
        }
      }
    } else {
      ck += ck + 1 < KC ? 1 : 0;  // a select: the stage stays one basic block
    }
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
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma16x16x4(fb[j][m], fa[i][m], acc[i][j]);
  };
  // stores local tile tl and clears the accumulators for the next tile
  auto store_tile = [&](int tl) {
    const long tile = wid + tl * nwg;
    const int M0 = (int)(tile % p.tiles_m) * kLdsTile, N0 = (int)(tile / p.tiles_m) * kLdsTile;
    const int Rw = M0 + (wave >> 1) * 64, Cw = N0 + (wave & 1) * 64;
    // B rows are the MFMA's first operand, so lane (li, g) holds columns
    // 4 g .. 4 g + 3 of row li of each 16 x 16 tile: one 16-byte (float32),
    // two 8-byte (bf16 hi, lo) or two 16-byte (float64) stores per tile
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = Rw + 16 * i + li;
      const int grp = row / p.rgroup, rin = row - grp * p.rgroup;
      if (row >= p.M || rin >= p.rvalid) continue;
      const long base0 = bat * p.sC + (long)grp * p.c_gstride + (long)rin * p.ldc;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = Cw + 16 * j + 4 * g;
        if (col >= p.N) continue;
        // four consecutive columns stay in one split group (csplit % 4 == 0)
        const long base = base0 + (long)(col / p.csplit) * p.chi - col + col % p.csplit;
        const f32x4 x = acc[i][j];
        if (p.vec && col + 3 < p.N) {
          if (p.Chi) {
            // four values at once: packed round-to-nearest-even conversions
            const bf16x4 h = __builtin_convertvector(x, bf16x4);
            const bf16x4 l = __builtin_convertvector(x - __builtin_convertvector(h, f32x4), bf16x4);
            const u32x2 hv = __builtin_bit_cast(u32x2, h), lv = __builtin_bit_cast(u32x2, l);
            if (p.vec == 2) {
              // lanes g and g ^ 1 (same row, columns 8 (g / 2) .. + 7) trade
              // halves: the even lane stores the eight hi values, the odd
              // lane the eight lo values, one 16-byte store each
              const bool odd = g & 1;
              const u32x2 send = odd ? hv : lv;
              u32x2 recv;
              recv[0] = __shfl_xor(send[0], 16);
              recv[1] = __shfl_xor(send[1], 16);
              u32x4 o;
              o[0] = odd ? recv[0] : hv[0];
              o[1] = odd ? recv[1] : hv[1];
              o[2] = odd ? lv[0] : recv[0];
              o[3] = odd ? lv[1] : recv[1];
              *(u32x4*)(odd ? p.Clo + base + col - 4 : p.Chi + base + col) = o;
            } else {
              *(u32x2*)(p.Chi + base + col) = hv;
              *(u32x2*)(p.Clo + base + col) = lv;
            }
          } else if (p.C64) {
            f64x2* d = (f64x2*)(p.C64 + base + col);
            f64x2 lo, hi;
            lo[0] = x[0]; lo[1] = x[1]; hi[0] = x[2]; hi[1] = x[3];
            if (p.accumulate) {
              lo += d[0];
              hi += d[1];
            }
            d[0] = lo;
            d[1] = hi;
          } else {
            *(f32x4*)(p.C + base + col) = x;
          }
          continue;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (col + r >= p.N) continue;
          if (p.Chi) {
            const bf16_t hgh = f32_to_bf16(x[r]);
            p.Chi[base + col + r] = hgh;
            p.Clo[base + col + r] = f32_to_bf16(x[r] - bf16_to_f32(hgh));
          } else if (p.C64) {
            p.C64[base + col + r] = p.accumulate ? p.C64[base + col + r] + (double)x[r] : (double)x[r];
          } else {
            p.C[base + col + r] = x[r];
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = zero4<float>();
  };

  // Stage s (buffer s % 5): copy stage s + 4 into the buffer of stage s - 1
  // (whose fragments every wavefront consumed before the barrier that ended
  // stage s - 1), read the fragments of stage s + 1, MFMAs of stage s (and,
  // on a tile's last stage, its stores), wait for the own copies of stage
  // s + 2, barrier.  The copies of the next tile run ahead of the current
  // tile's MFMAs and stores like those of its own later stages.
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
  // Stages run in pairs (fragments of the first in fa0/fb0, of the second in
  // fa1/fb1) with no branch inside a pair, so the accumulators and fragments
  // keep their registers around the loop; an odd K ends with one more stage
  // (the launcher gives a workgroup several tiles only for an even number
  // of stages, so every tile starts on fa0/fb0).
  auto stage_a = [&]() {
    copy_stage(back2(b1));
    frags(b1, fa1, fb1);
    mfma_stage(fa0, fb0);
    wait_vm<8>();
    barrier_nofence();
    b1 = next(b1);
  };
  auto stage_b = [&]() {
    copy_stage(back2(b1));
    frags(b1, fa0, fb0);
    mfma_stage(fa1, fb1);
    wait_vm<8>();
    barrier_nofence();
    b1 = next(b1);
  };
  for (int tl = 0; tl < ntl; ++tl) {
    for (int kp = 0; kp < KC / 2; ++kp) {
      stage_a();
      stage_b();
    }
    if (KC & 1) stage_a();
    store_tile(tl);
  }
  wait_vm<0>();  // the repeated copies past the end
}

// The same NT product with both operands given as bf16 hi and lo planes
// (x = hi + lo) on the 16x16x32 bf16 MFMA, hi hi + hi lo + lo hi with
// float32 accumulation: C[row][col] = sum_k A[row][k] B[col][k] in float32.
// One 128 x 128 block of C per workgroup; a stage is 32 k (64 bytes per row
// and plane), four planes per stage (B hi, B lo, A hi, A lo) in the ring of
// five buffers (160 KB of LDS); K a multiple of 32.  W(Omega) GG(Omega) of
// the split-precision dynamic entry.
struct DenseLdsSplitArgs {
  const bf16_t* Ah;
  const bf16_t* Al;
  const bf16_t* Bh;
  const bf16_t* Bl;
  long lda, ldb, ldc;  // row strides (elements)
  long sA, sB, sC;     // batch strides (elements; the batch is the grid's slowest index)
  int M, N, K;
  float* C;
  int tiles_m, tiles_n;
  int vec;  // 16-byte stores allowed (set by the launcher)
  double* C64 = nullptr;  // float64 output instead of C (same offsets)
  // split addressing as for the float32 kernel
  int bsplit = 1 << 30;
  long bhi = 0;
  int csplit = 1 << 30;
  long chi = 0;
};

// PB = 4: four wavefronts of 64 x 64 of C; PB = 2: eight of 64 rows x 32
// columns, two per SIMD.
template <int PB = 4>
__global__ __launch_bounds__(1024 / PB) void dense_lds_bf16x3_kernel(const DenseLdsSplitArgs p) {
  constexpr int MODE = kLdsBf16x3;
  constexpr int NW = 16 / PB;    // wavefronts
  constexpr int CP = PB / 2;     // copies per wavefront, panel and plane
  constexpr int NBG = 8 / PB;    // wavefront groups over the B rows (C columns)
  // [buffer][plane: B rows hi, lo (first MFMA operand), A rows hi, lo][row * 4 + swizzled segment]
  __shared__ u32x4 lds[kLdsBufs][4][kLdsPieces];
  // one-dimensional grid over (batch, tile), batch-major, remapped so that
  // each XCD takes a contiguous range: the tiles of a batch share its A and B
  // operands in one L2 (with the batch on a second grid axis every XCD took
  // a share of every batch and read its A panel again)
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  const int ntl = p.tiles_m * p.tiles_n;
  const long bat = lg / ntl;
  const int bid = lg - (int)bat * ntl;
  const int M0 = (bid % p.tiles_m) * kLdsTile;  // row blocks fastest: they share B
  const int N0 = (bid / p.tiles_m) * kLdsTile;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15;
  const int g = lane >> 4;
  const char* srcb[2][CP];  // [plane][copy]
  const char* srca[2][CP];
#pragma unroll
  for (int h = 0; h < CP; ++h) {
    const int c = wave + NW * h;
    const int row = 16 * c + (lane >> 2);
    const int seg = (lane & 3) ^ ((row >> 1) & 3);
    const long ra = M0 + row < p.M ? M0 + row : p.M - 1;
    const long rb = N0 + row < p.N ? N0 + row : p.N - 1;
    const long oa = bat * p.sA + ra * p.lda,
               ob = bat * p.sB + (rb / p.bsplit) * p.bhi + (rb % p.bsplit) * p.ldb;
    srca[0][h] = (const char*)(p.Ah + oa) + 16 * seg;
    srca[1][h] = (const char*)(p.Al + oa) + 16 * seg;
    srcb[0][h] = (const char*)(p.Bh + ob) + 16 * seg;
    srcb[1][h] = (const char*)(p.Bl + ob) + 16 * seg;
  }
  // fragments: first operand B rows wb 16 PB + 16 i (i < PB), second A rows
  // wa 64 + 16 j
  const int wb = wave % NBG, wa = wave / NBG;
  int sb[4], sa[4];
  const int sw = g ^ ((li >> 1) & 3);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sb[i] = (wb * 16 * PB + 16 * (i < PB ? i : 0) + li) * 4 + sw;
    sa[i] = (wa * 64 + 16 * i + li) * 4 + sw;
  }
  const int KC = p.K / 32;
  int ck = 0;  // next chunk to copy, held at the last one past the end
  auto copy_stage = [&](int b) {
    const long ko = (long)ck * 64;
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int h = 0; h < CP; ++h) {
        const int ch = 64 * (wave + NW * h);
        global_to_lds16(srcb[q][h] + ko, &lds[b][q][ch]);
        global_to_lds16(srca[q][h] + ko, &lds[b][2 + q][ch]);
      }
    ck += ck + 1 < KC ? 1 : 0;
  };
  constexpr int kStageCopies = 4 * CP;  // per wavefront
  f32x4 acc[PB][4];
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = zero4<float>();
  LdsFrags<MODE, PB> f0, f1;
  auto next = [](int x) { return x + 1 == kLdsBufs ? 0 : x + 1; };
  auto back2 = [](int x) { return x >= 2 ? x - 2 : x + kLdsBufs - 2; };
  // the schedule of the float32 kernel: copy stage s + 4 into the buffer of
  // stage s - 1, read the fragments of stage s + 1, MFMAs of stage s, wait
  // for the own copies of stage s + 2, barrier
  copy_stage(0);
  copy_stage(1);
  copy_stage(2);
  copy_stage(3);
  wait_vm<2 * kStageCopies>();
  barrier_nofence();
  lds_frags<MODE, 2, PB>(lds[0], sb, sa, f0);
  int b1 = 1;
  auto stage_a = [&]() {
    copy_stage(back2(b1));
    lds_frags<MODE, 2, PB>(lds[b1], sb, sa, f1);
    lds_half_mfma<MODE, false, PB>(f0, acc);
    wait_vm<2 * kStageCopies>();
    barrier_nofence();
    b1 = next(b1);
  };
  auto stage_b = [&]() {
    copy_stage(back2(b1));
    lds_frags<MODE, 2, PB>(lds[b1], sb, sa, f0);
    lds_half_mfma<MODE, false, PB>(f1, acc);
    wait_vm<2 * kStageCopies>();
    barrier_nofence();
    b1 = next(b1);
  };
  for (int kp = 0; kp < KC / 2; ++kp) {
    stage_a();
    stage_b();
  }
  if (KC & 1) stage_a();
  wait_vm<0>();  // the repeated copies past the end

  // lane (li, g) holds C[row 16 j + li][columns 16 i + 4 g .. + 3]
  const int Rw = M0 + wa * 64, Cw = N0 + wb * 16 * PB;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = Rw + 16 * j + li;
    if (row >= p.M) continue;
    const long rbase = bat * p.sC + (long)row * p.ldc;
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int col = Cw + 16 * i + 4 * g;
      if (col >= p.N) continue;
      // four consecutive columns stay in one split group (csplit % 4 == 0)
      const long o = rbase + (long)(col / p.csplit) * p.chi + col % p.csplit;
      if (p.C64) {
        if (p.vec && col + 3 < p.N) {
          f64x2 lo, hi;
          lo[0] = acc[i][j][0]; lo[1] = acc[i][j][1];
          hi[0] = acc[i][j][2]; hi[1] = acc[i][j][3];
          *(f64x2*)(p.C64 + o) = lo;
          *(f64x2*)(p.C64 + o + 2) = hi;
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (col + r < p.N) p.C64[o + r] = acc[i][j][r];
        }
      } else if (p.vec && col + 3 < p.N) {
        *(f32x4*)(p.C + o) = acc[i][j];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (col + r < p.N) p.C[o + r] = acc[i][j][r];
      }
    }
  }
}

template <int PB = 4>
inline hipError_t launch_dense_lds_bf16x3(DenseLdsSplitArgs a, int batch, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || batch <= 0) return hipSuccess;
  if (batch > 65535 || a.K % 32 != 0 || a.K <= 0 || !a.Ah || !a.Al || !a.Bh || !a.Bl ||
      (!a.C && !a.C64) || a.bsplit <= 0 || a.csplit <= 0 ||
      (a.csplit < (1 << 30) && a.csplit % 4))
    return hipErrorInvalidValue;
  // 16-byte panel rows: row strides and batch strides multiples of 8 bf16
  if (a.lda % 8 || a.ldb % 8 || a.sA % 8 || a.sB % 8 || a.bhi % 8) return hipErrorInvalidValue;
  const bool split_ok = a.csplit >= (1 << 30) || (a.csplit % 4 == 0 && a.chi % 4 == 0);
  const uintptr_t out = a.C64 ? (uintptr_t)a.C64 : (uintptr_t)a.C;
  a.vec = (a.ldc % 4 == 0 && a.sC % 4 == 0 && out % 16 == 0 && split_ok) ? 1 : 0;
  a.tiles_m = (a.M + kLdsTile - 1) / kLdsTile;
  a.tiles_n = (a.N + kLdsTile - 1) / kLdsTile;
  const long nb = (long)a.tiles_m * a.tiles_n * batch;
  if (nb >= (1L << 31) || !grid_fits(nb, 1024 / PB)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((dense_lds_bf16x3_kernel<PB>), dim3((unsigned)nb), dim3(1024 / PB), 0, s, a);
  return hipGetLastError();
}

inline hipError_t launch_dense_lds_f32(DenseLdsArgs a, int batch, hipStream_t s,
                                      long wg_target = 0) {
  if (a.M <= 0 || a.N <= 0 || batch <= 0) return hipSuccess;
  if (batch > 65535) return hipErrorInvalidValue;
  if (a.K % 16 != 0 || a.K <= 0 || a.rgroup <= 0 || (a.Chi && !a.Clo) ||
      (!a.Chi && !a.C && !a.C64) || (a.accumulate && !a.C64) || a.bsplit <= 0 ||
      a.csplit <= 0 || (a.csplit < (1 << 30) && a.csplit % 4) || a.bhi % 4)
    return hipErrorInvalidValue;
  // vector stores of four consecutive columns: every row start a multiple of
  // four elements and the output 16-byte aligned
  {
    const uintptr_t out = a.Chi ? (uintptr_t)a.Chi | (uintptr_t)a.Clo
                                : a.C64 ? (uintptr_t)a.C64 : (uintptr_t)a.C;
    const long esz = a.Chi ? 2 : a.C64 ? 8 : 4;
    const bool split_ok = a.csplit >= (1 << 30) || (a.csplit % 4 == 0 && a.chi % 4 == 0);
    a.vec = (a.ldc % 4 == 0 && a.c_gstride % 4 == 0 && a.sC % 4 == 0 && split_ok &&
             out % (4 * esz < 16 ? 4 * esz : 16) == 0) ? 1 : 0;
    // split planes: paired 16-byte stores of eight columns when every row
    // start is a multiple of eight, N too (partner lanes are then both in
    // or both out of range) and both planes 16-byte aligned
    if (a.Chi && a.vec && a.ldc % 8 == 0 && a.c_gstride % 8 == 0 && a.sC % 8 == 0 &&
        a.N % 8 == 0 && out % 16 == 0 && a.csplit >= (1 << 30))
      a.vec = 2;
  }
  a.tiles_m = (a.M + kLdsTile - 1) / kLdsTile;
  a.tiles_n = (a.N + kLdsTile - 1) / kLdsTile;
  const long ntiles = (long)a.tiles_m * a.tiles_n;
  // short K (at most 8 stages, an even number): several tiles per workgroup, so that the
  // grid holds at most wg_target workgroups (all resident at once) and a
  // workgroup's copies for its next tile overlap its current tile.  Longer
  // K (or wg_target 0): one tile per workgroup (with 13 stages, C = 20800 x
  // 266240, the shared workgroups measured 4% slower: each tile's stores
  // hold up the next wait)
  long per = 1;
  if (wg_target > 0 && a.K <= 128 && a.K % 32 == 0)
    per = (ntiles * batch + wg_target - 1) / wg_target;
  a.tpw = (int)(per < 1 ? 1 : per > ntiles ? ntiles : per);
  const long nb = (ntiles + a.tpw - 1) / a.tpw;
  if (!grid_fits(nb, 256, batch)) return hipErrorInvalidValue;
  if (a.tpw > 1)
    hipLaunchKernelGGL(dense_lds_f32_kernel<true>, dim3((unsigned)nb, (unsigned)batch), dim3(256),
                       0, s, a);
  else
    hipLaunchKernelGGL(dense_lds_f32_kernel<false>, dim3((unsigned)nb, (unsigned)batch), dim3(256),
                       0, s, a);
  return hipGetLastError();
}

}  // namespace sox
