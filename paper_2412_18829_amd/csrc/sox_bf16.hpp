// Split-precision (bf16 x 3) variant of the fused B, C -> D contraction.
//
// Every float32 operand x is stored as x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (split_bf16_kernel).  Each product of the fused kernel
// then runs as hi*hi + hi*lo + lo*hi on the bf16 MFMA with float32
// accumulation; the dropped lo*lo term and the rounding of lo leave a
// relative error of about 2^-16 per product.  Operand layout, tiling and
// schedule follow fused_bcd_kernel (sox_fused.hpp) with 32-deep k chunks:
// lane (li, g) loads the 8 consecutive bf16 of its row at k0 + 8 g as one
// 16-byte vector, for hi and lo separately.
#pragma once

#include "sox_common.hpp"

namespace sox {

__global__ void split_bf16_kernel(const float* src, bf16_t* hi, bf16_t* lo, long count) {
  SOX_FOR_FLAT(idx, count) {
    const float x = src[idx];
    const bf16_t h = f32_to_bf16(x);
    hi[idx] = h;
    lo[idx] = f32_to_bf16(x - bf16_to_f32(h));
  }
}

struct FusedSplitArgs {
  const bf16_t *Ah, *Al, *Yh, *Yl, *Ph, *Pl, *Uh, *Ul;
  float* D;
  long a_tstride, a_vstride, y_tstride, p_tstride, u_rstride, u_vstride, d_tstride;
  int accumulate;
  int n, nP, NP;   // nP multiple of 32
  int tiles_p, tiles_r, n_tau;
  // split of the v sum over vsplit workgroups per tile (LDS-staged kernel
  // only): split s sums v in [s vchunk, (s+1) vchunk) into D + s d_sstride
  int vsplit = 1, vchunk = 1 << 30;
  long d_sstride = 0;
};

template <int WP, int WR>
__global__ __launch_bounds__(256) void fused_bcd_bf16x3_kernel(const FusedSplitArgs p) {
  constexpr int PB = WP / 16;
  constexpr int RB = WR / 16;
  typedef bf16x8 V8;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int rt = bid % p.tiles_r;
  const int tmp = bid / p.tiles_r;
  const int pt = tmp % p.tiles_p;
  const int t = tmp / p.tiles_p;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15;
  const int g = lane >> 4;
  const int P0 = pt * (2 * WP) + (wave >> 1) * WP;
  const int R0 = rt * (2 * WR) + (wave & 1) * WR;
  const long ld = p.nP;
  const long aoff = t * p.a_tstride + (long)(P0 + li) * ld + 8 * g;
  const long yoff = t * p.y_tstride + (long)(R0 + li) * ld + 8 * g;
  const long poff = t * p.p_tstride + (long)(P0 + li) * ld + 8 * g;
  const long uoff = (long)(R0 + li) * p.u_rstride + 8 * g;

  f32x4 accB[PB][RB], accC[PB][RB], dacc[PB][RB];
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      accB[i][j] = zero4<float>();
      accC[i][j] = zero4<float>();
      dacc[i][j] = zero4<float>();
    }

  const int KC = p.nP >> 5;
  const int nv = p.n;
  V8 ah[PB], al[PB], yh[RB], yl[RB], ph[PB], pl[PB], uh[RB], ul[RB];
#pragma unroll
  for (int i = 0; i < PB; ++i) {
    const long o = aoff + (long)(16 * i) * ld, q = poff + (long)(16 * i) * ld;
    ah[i] = *(const V8*)(p.Ah + o); al[i] = *(const V8*)(p.Al + o);
    ph[i] = *(const V8*)(p.Ph + q); pl[i] = *(const V8*)(p.Pl + q);
  }
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    const long o = yoff + (long)(16 * j) * ld, q = uoff + (long)(16 * j) * p.u_rstride;
    yh[j] = *(const V8*)(p.Yh + o); yl[j] = *(const V8*)(p.Yl + o);
    uh[j] = *(const V8*)(p.Uh + q); ul[j] = *(const V8*)(p.Ul + q);
  }

  for (int v = 0; v < nv; ++v) {
    for (int kc = 0; kc < KC; ++kc) {
      const bool wrap = (kc + 1 == KC);
      int vn = wrap ? v + 1 : v;
      int kn = wrap ? 0 : kc + 1;
      const bool last = vn >= nv;
      vn = last ? nv - 1 : vn;
      kn = last ? KC - 1 : kn;
      const long ko = (long)kn * 32;
      V8 ahn[PB], aln[PB], yhn[RB], yln[RB], phn[PB], pln[PB], uhn[RB], uln[RB];
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const long o = aoff + (long)vn * p.a_vstride + ko + (long)(16 * i) * ld;
        const long q = poff + ko + (long)(16 * i) * ld;
        ahn[i] = *(const V8*)(p.Ah + o); aln[i] = *(const V8*)(p.Al + o);
        phn[i] = *(const V8*)(p.Ph + q); pln[i] = *(const V8*)(p.Pl + q);
      }
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        const long o = yoff + ko + (long)(16 * j) * ld;
        const long q = uoff + (long)vn * p.u_vstride + ko + (long)(16 * j) * p.u_rstride;
        yhn[j] = *(const V8*)(p.Yh + o); yln[j] = *(const V8*)(p.Yl + o);
        uhn[j] = *(const V8*)(p.Uh + q); uln[j] = *(const V8*)(p.Ul + q);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < PB; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) {
          accB[i][j] = mfma16x16x32bf16(ah[i], yh[j], accB[i][j]);
          accC[i][j] = mfma16x16x32bf16(ph[i], uh[j], accC[i][j]);
          accB[i][j] = mfma16x16x32bf16(ah[i], yl[j], accB[i][j]);
          accC[i][j] = mfma16x16x32bf16(ph[i], ul[j], accC[i][j]);
          accB[i][j] = mfma16x16x32bf16(al[i], yh[j], accB[i][j]);
          accC[i][j] = mfma16x16x32bf16(pl[i], uh[j], accC[i][j]);
        }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < PB; ++i) { ah[i] = ahn[i]; al[i] = aln[i]; ph[i] = phn[i]; pl[i] = pln[i]; }
#pragma unroll
      for (int j = 0; j < RB; ++j) { yh[j] = yhn[j]; yl[j] = yln[j]; uh[j] = uhn[j]; ul[j] = uln[j]; }
    }
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        dacc[i][j] += accB[i][j] * accC[i][j];
        accB[i][j] = zero4<float>();
        accC[i][j] = zero4<float>();
      }
  }

  float* Db = p.D + t * p.d_tstride;
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int j = 0; j < RB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int P = P0 + 16 * i + 4 * g + r;
        const int R = R0 + 16 * j + li;
        const long off = (long)P * p.NP + R;
        Db[off] = p.accumulate ? Db[off] + dacc[i][j][r] : dacc[i][j][r];
      }
}

template <int WP, int WR>
inline hipError_t launch_fused_bf16x3(const FusedSplitArgs& a, hipStream_t s) {
  const int nb = a.tiles_p * a.tiles_r * a.n_tau;
  if (nb <= 0) return hipSuccess;
  if (a.nP % 32 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fused_bcd_bf16x3_kernel<WP, WR>), dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

// LDS-staged variant with a 128 x 128 block of D per workgroup (four
// wavefronts of 64 x 64) and k stages of 32.  For every stage (v, k chunk)
// the workgroup copies the hi and lo planes of its four row panels -- A^v
// and G_wP^T over its P rows, Y and U2^v over its R rows, 128 rows x 32
// bf16 each, 64 KB in all -- straight from global memory into one of two
// LDS buffers (16-byte global-to-LDS loads, no registers in between); each
// panel row is then read from LDS by the two wavefronts that share it, so
// the operand traffic through the vector cache is that of the workgroup
// tile, not of four wave tiles.  The copy for stage s+1 is issued before
// the MFMAs of stage s; one barrier per stage suffices, since a buffer is
// rewritten only after every wavefront has passed the barrier that follows
// its last read of it, and every wavefront waits for its own copies before
// that barrier.
//
// LDS rows are 64 bytes (four 16-byte segments); segment c of row r sits at
// position c ^ ((r >> 1) & 3), so the 16-byte reads of eight consecutive
// rows at one k group cover all banks once.  The Hadamard epilogue of v is
// folded into the first stage of v + 1: the first MFMA of each B and C tile
// starts from zero, and the products of the previous v are added to D just
// before, tile by tile, so the vector ALU work overlaps the matrix pipe.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kLdsTile = 128;                 // rows of each staged panel
constexpr int kLdsPieces = kLdsTile * 4;      // 16-byte pieces per panel plane

template <bool FIRST>
__device__ __forceinline__ void lds_bf16x3_stage(const u32x4 (*buf)[kLdsPieces], const int* sa,
                                                 const int* sy, f32x4 (*accB)[4],
                                                 f32x4 (*accC)[4], f32x4 (*dacc)[4]) {
  bf16x8 ah[4], al[4], yh[4], yl[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ah[i] = __builtin_bit_cast(bf16x8, buf[0][sa[i]]);
    al[i] = __builtin_bit_cast(bf16x8, buf[1][sa[i]]);
    yh[i] = __builtin_bit_cast(bf16x8, buf[2][sy[i]]);
    yl[i] = __builtin_bit_cast(bf16x8, buf[3][sy[i]]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (FIRST) {
        dacc[i][j] += accB[i][j] * accC[i][j];
        accB[i][j] = mfma16x16x32bf16(ah[i], yh[j], zero4<float>());
      } else {
        accB[i][j] = mfma16x16x32bf16(ah[i], yh[j], accB[i][j]);
      }
      accB[i][j] = mfma16x16x32bf16(ah[i], yl[j], accB[i][j]);
      accB[i][j] = mfma16x16x32bf16(al[i], yh[j], accB[i][j]);
    }
  bf16x8 ph[4], pl[4], uh[4], ul[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ph[i] = __builtin_bit_cast(bf16x8, buf[4][sa[i]]);
    pl[i] = __builtin_bit_cast(bf16x8, buf[5][sa[i]]);
    uh[i] = __builtin_bit_cast(bf16x8, buf[6][sy[i]]);
    ul[i] = __builtin_bit_cast(bf16x8, buf[7][sy[i]]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (FIRST) accC[i][j] = mfma16x16x32bf16(ph[i], uh[j], zero4<float>());
      else accC[i][j] = mfma16x16x32bf16(ph[i], uh[j], accC[i][j]);
      accC[i][j] = mfma16x16x32bf16(ph[i], ul[j], accC[i][j]);
      accC[i][j] = mfma16x16x32bf16(pl[i], uh[j], accC[i][j]);
    }
}

__global__ __launch_bounds__(256) void fused_bcd_lds_bf16x3_kernel(const FusedSplitArgs p) {
  // [buffer][panel plane: Ah Al Yh Yl Ph Pl Uh Ul][row * 4 + swizzled segment]
  __shared__ u32x4 lds[2][8][kLdsPieces];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int rt = bid % p.tiles_r;
  int rest = bid / p.tiles_r;
  const int pt = rest % p.tiles_p;
  rest /= p.tiles_p;
  const int t = rest % p.n_tau;
  const int sp = rest / p.n_tau;
  const int v_begin = sp * p.vchunk;
  const int v_end = v_begin + p.vchunk < p.n ? v_begin + p.vchunk : p.n;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15;
  const int g = lane >> 4;
  const int P0 = pt * kLdsTile, R0 = rt * kLdsTile;
  const long ld = p.nP;

  // Copies: instruction h of wavefront w fills LDS pieces 64 c .. 64 c + 63
  // (c = w + 4 h) of a plane, one 16-byte piece per lane at position 64 c +
  // lane, i.e. row 16 c + lane / 4 and swizzled segment lane % 4.
  long oa[2], oy[2], op[2], ou[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = wave + 4 * h;
    const int row = 16 * c + (lane >> 2);
    const int seg = (lane & 3) ^ ((row >> 1) & 3);
    oa[h] = (long)t * p.a_tstride + (long)(P0 + row) * ld + 8 * seg;
    oy[h] = (long)t * p.y_tstride + (long)(R0 + row) * ld + 8 * seg;
    op[h] = (long)t * p.p_tstride + (long)(P0 + row) * ld + 8 * seg;
    ou[h] = (long)(R0 + row) * p.u_rstride + 8 * seg;
  }
  // fragment positions: P rows (wave >> 1) 64 + 16 i + li, R rows (wave & 1) 64 + 16 j + li
  int sa[4], sy[4];
  const int sw = g ^ ((li >> 1) & 3);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sa[i] = ((wave >> 1) * 64 + 16 * i + li) * 4 + sw;
    sy[i] = ((wave & 1) * 64 + 16 * i + li) * 4 + sw;
  }

  f32x4 accB[4][4], accC[4][4], dacc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      accB[i][j] = zero4<float>();
      accC[i][j] = zero4<float>();
      dacc[i][j] = zero4<float>();
    }

  auto load_stage = [&](int v, int kc, int b) {
    const long ko = (long)kc * 32;
    const long av = (long)v * p.a_vstride + ko, uv = (long)v * p.u_vstride + ko;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = 64 * (wave + 4 * h);
      global_to_lds16(p.Ah + oa[h] + av, &lds[b][0][c]);
      global_to_lds16(p.Al + oa[h] + av, &lds[b][1][c]);
      global_to_lds16(p.Yh + oy[h] + ko, &lds[b][2][c]);
      global_to_lds16(p.Yl + oy[h] + ko, &lds[b][3][c]);
      global_to_lds16(p.Ph + op[h] + ko, &lds[b][4][c]);
      global_to_lds16(p.Pl + op[h] + ko, &lds[b][5][c]);
      global_to_lds16(p.Uh + ou[h] + uv, &lds[b][6][c]);
      global_to_lds16(p.Ul + ou[h] + uv, &lds[b][7][c]);
    }
  };

  const int KC = p.nP >> 5;
  const int nst = v_end > v_begin ? (v_end - v_begin) * KC : 0;
  if (nst > 0) load_stage(v_begin, 0, 0);
  wait_vm_all();
  __syncthreads();
  int v = v_begin, kc = 0;
  for (int s = 0; s < nst; ++s) {
    int vn = v, kn = kc + 1;
    if (kn == KC) {
      kn = 0;
      ++vn;
    }
    if (s + 1 < nst) load_stage(vn, kn, (s & 1) ^ 1);
    if (kc == 0) lds_bf16x3_stage<true>(lds[s & 1], sa, sy, accB, accC, dacc);
    else lds_bf16x3_stage<false>(lds[s & 1], sa, sy, accB, accC, dacc);
    wait_vm_all();
    __syncthreads();
    v = vn;
    kc = kn;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) dacc[i][j] += accB[i][j] * accC[i][j];

  float* Db = p.D + (long)sp * p.d_sstride + (long)t * p.d_tstride;
  const int Pw = P0 + (wave >> 1) * 64, Rw = R0 + (wave & 1) * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long off = (long)(Pw + 16 * i + 4 * g + r) * p.NP + Rw + 16 * j + li;
        Db[off] = p.accumulate ? Db[off] + dacc[i][j][r] : dacc[i][j][r];
      }
}

// Grid: (R tile, P tile, tau, v split), R tiles fastest.
inline hipError_t launch_fused_lds_bf16x3(const FusedSplitArgs& a, hipStream_t s) {
  if (a.nP % 32 != 0 || a.NP % kLdsTile != 0 || a.tiles_p * kLdsTile != a.NP ||
      a.tiles_r * kLdsTile != a.NP || a.vsplit < 1)
    return hipErrorInvalidValue;
  const long nb = (long)a.tiles_p * a.tiles_r * a.n_tau * a.vsplit;
  if (nb <= 0) return hipSuccess;
  if (nb > (1L << 31) - 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fused_bcd_lds_bf16x3_kernel, dim3((unsigned)nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace sox
