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

#include <type_traits>

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
// wavefronts of 64 x 64).  The v sum runs in stages of one v and 32 k, and
// each stage in two halves: the B half needs the hi and lo planes of A^v
// (the workgroup's P rows) and Y (its R rows), the C half those of G_wP^T
// (P rows) and U2^v (R rows), 128 rows x 32 bf16 per plane, 32 KB per half.
// The halves are copied straight from global memory into a ring of five
// LDS buffers (16-byte global-to-LDS loads, no registers in between), four
// halves ahead of the MFMAs, so the copies have about two stages of matrix
// work to land.  Each panel row is read from LDS by the two wavefronts that
// share it, so the operand traffic through the vector cache is that of the
// workgroup tile, not of four wave tiles, and the fragments of half h + 1
// are read into a second register set while the MFMAs of half h run.
//
// One barrier per half h, after the wavefront has waited for its own copies
// of half h + 2 (copies of halves h + 3 and h + 4 stay in flight; the
// barrier carries no memory fence, which would wait for them too): the
// copy issued in half h overwrites the buffer of half h - 1, whose
// fragments every wavefront consumed before the barrier that ends half
// h - 1.
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
constexpr int kLdsBufs = 5;                   // ring of half-stage buffers (160 KB)
constexpr int kLdsAhead = kLdsBufs - 1;       // halves copied ahead of the MFMAs

// s_waitcnt vmcnt(8 (kLdsAhead - 2)): the copies of the kLdsAhead - 2
// newest halves (eight loads per wavefront each) may still be in flight
constexpr int kLdsWaitAhead = 8 * (kLdsAhead - 2);
static_assert(kLdsWaitAhead < 64, "vmcnt holds six bits");
__device__ __forceinline__ void wait_vm_ahead() {
  __builtin_amdgcn_s_waitcnt((kLdsWaitAhead & 15) | ((kLdsWaitAhead >> 4) << 14) | 0x0F70);
}

struct Bf16x3Frags {
  bf16x8 ah[4], al[4], bh[4], bl[4];  // P-row panel hi/lo, R-row panel hi/lo
};

__device__ __forceinline__ void lds_read_frags(const u32x4 (*buf)[kLdsPieces], const int* sa,
                                               const int* sy, Bf16x3Frags& f) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    f.ah[i] = __builtin_bit_cast(bf16x8, buf[0][sa[i]]);
    f.al[i] = __builtin_bit_cast(bf16x8, buf[1][sa[i]]);
    f.bh[i] = __builtin_bit_cast(bf16x8, buf[2][sy[i]]);
    f.bl[i] = __builtin_bit_cast(bf16x8, buf[3][sy[i]]);
  }
}

// acc (+)= hi hi + hi lo + lo hi over one 32-deep k chunk; FIRST starts from zero
template <bool FIRST>
__device__ __forceinline__ void bf16x3_half(const Bf16x3Frags& f, f32x4 (*acc)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = mfma16x16x32bf16(f.ah[i], f.bh[j], FIRST ? zero4<float>() : acc[i][j]);
      acc[i][j] = mfma16x16x32bf16(f.ah[i], f.bl[j], acc[i][j]);
      acc[i][j] = mfma16x16x32bf16(f.al[i], f.bh[j], acc[i][j]);
    }
}

__global__ __launch_bounds__(256) void fused_bcd_lds_bf16x3_kernel(const FusedSplitArgs p) {
  // [buffer][plane: P-row hi, P-row lo, R-row hi, R-row lo][row * 4 + swizzled segment]
  __shared__ u32x4 lds[kLdsBufs][4][kLdsPieces];
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
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15;
  const int g = lane >> 4;
  const int P0 = pt * kLdsTile, R0 = rt * kLdsTile;
  const int ld = p.nP;

  // Copies: instruction h of wavefront w fills LDS pieces 64 c .. 64 c + 63
  // (c = w + 4 h) of a plane, one 16-byte piece per lane at position 64 c +
  // lane, i.e. row 16 c + lane / 4 and swizzled segment lane % 4.  Sources
  // are a wave-uniform base (tau, v, k chunk) plus a 32-bit lane offset
  // (the launcher checks the panels' extents).
  unsigned orow_p[2], orow_r[2], orow_u[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = wave + 4 * h;
    const int row = 16 * c + (lane >> 2);
    const int seg = (lane & 3) ^ ((row >> 1) & 3);
    orow_p[h] = (unsigned)((P0 + row) * ld + 8 * seg);
    orow_r[h] = (unsigned)((R0 + row) * ld + 8 * seg);
    orow_u[h] = (unsigned)((R0 + row) * p.u_rstride + 8 * seg);
  }
  const long ot_a = (long)t * p.a_tstride, ot_y = (long)t * p.y_tstride;
  const long ot_p = (long)t * p.p_tstride;
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

  const int KC = p.nP >> 5;
  const int nst = v_end > v_begin ? (v_end - v_begin) * KC : 0;
  // Copy cursor: the stage whose halves are copied next, held at the last
  // stage once every stage is under way, so that the halves past the end
  // repeat it into buffers nobody reads again.  Every half then issues
  // exactly eight copies per wavefront and the wait below stays exact.
  int cv = v_begin, ckc = 0, cs = 0;
  const int c0 = 64 * wave, c1 = 64 * (wave + 4);
  auto copy_b = [&](int b) {
    const long ko = (long)ckc * 32;
    const bf16_t* ah = p.Ah + ot_a + (long)cv * p.a_vstride + ko;
    const bf16_t* al = p.Al + ot_a + (long)cv * p.a_vstride + ko;
    const bf16_t* yh = p.Yh + ot_y + ko;
    const bf16_t* yl = p.Yl + ot_y + ko;
    global_to_lds16(ah + orow_p[0], &lds[b][0][c0]);
    global_to_lds16(ah + orow_p[1], &lds[b][0][c1]);
    global_to_lds16(al + orow_p[0], &lds[b][1][c0]);
    global_to_lds16(al + orow_p[1], &lds[b][1][c1]);
    global_to_lds16(yh + orow_r[0], &lds[b][2][c0]);
    global_to_lds16(yh + orow_r[1], &lds[b][2][c1]);
    global_to_lds16(yl + orow_r[0], &lds[b][3][c0]);
    global_to_lds16(yl + orow_r[1], &lds[b][3][c1]);
  };
  auto copy_c = [&](int b) {
    const long ko = (long)ckc * 32;
    const bf16_t* ph = p.Ph + ot_p + ko;
    const bf16_t* pl = p.Pl + ot_p + ko;
    const bf16_t* uh = p.Uh + (long)cv * p.u_vstride + ko;
    const bf16_t* ul = p.Ul + (long)cv * p.u_vstride + ko;
    global_to_lds16(ph + orow_p[0], &lds[b][0][c0]);
    global_to_lds16(ph + orow_p[1], &lds[b][0][c1]);
    global_to_lds16(pl + orow_p[0], &lds[b][1][c0]);
    global_to_lds16(pl + orow_p[1], &lds[b][1][c1]);
    global_to_lds16(uh + orow_u[0], &lds[b][2][c0]);
    global_to_lds16(uh + orow_u[1], &lds[b][2][c1]);
    global_to_lds16(ul + orow_u[0], &lds[b][3][c0]);
    global_to_lds16(ul + orow_u[1], &lds[b][3][c1]);
    const int adv = cs + 1 < nst ? 1 : 0;  // selects, no branch: one block per half
    cs += adv;
    ckc += adv;
    const int wrap = ckc == KC ? 1 : 0;
    ckc = wrap ? 0 : ckc;
    cv += wrap;
  };
  if (nst > 0) {
    Bf16x3Frags f0, f1;
    // halves 0..3 (stages 0 and 1) in flight, then halves 0 and 1 landed
    copy_b(0);
    copy_c(1);
    copy_b(2);
    copy_c(3);
    wait_vm_ahead();
    barrier_nofence();
    lds_read_frags(lds[0], sa, sy, f0);
    int b1 = 1;  // buffer of half 2 s + 1
    // B half of stage s: copy half 2 s + 4 into the buffer of half 2 s - 1,
    // read the C-half fragments, MFMAs from f0.  C half: copy half 2 s + 5
    // into the buffer of half 2 s, read the next B-half fragments, MFMAs
    // from f1.  Each half is one basic block (no branch between its copies,
    // fragment reads and MFMAs), which leaves the compiler free to overlap
    // them.
    auto half_b = [&](auto first, int bcopy) {
      constexpr bool F = decltype(first)::value;
      copy_b(bcopy);
      lds_read_frags(lds[b1], sa, sy, f1);
      if constexpr (F) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) dacc[i][j] += accB[i][j] * accC[i][j];
      }
      bf16x3_half<F>(f0, accB);
      wait_vm_ahead();
      barrier_nofence();
    };
    auto half_c = [&](auto first, int bcopy, int bread) {
      constexpr bool F = decltype(first)::value;
      copy_c(bcopy);
      lds_read_frags(lds[bread], sa, sy, f0);
      bf16x3_half<F>(f1, accC);
      wait_vm_ahead();
      barrier_nofence();
    };
    for (int v = v_begin; v < v_end; ++v) {
      for (int kc = 0; kc < KC; ++kc) {
        const int b0 = b1 == 0 ? kLdsBufs - 1 : b1 - 1;  // half 2 s
        const int b2 = b1 + 1 == kLdsBufs ? 0 : b1 + 1;  // half 2 s + 2
        const int b3 = b2 + 1 == kLdsBufs ? 0 : b2 + 1;  // half 2 s + 3
        const int b4 = b3 + 1 == kLdsBufs ? 0 : b3 + 1;  // half 2 s + 4
        if (kc == 0) {
          half_b(std::true_type{}, b4);
          half_c(std::true_type{}, b0, b2);
        } else {
          half_b(std::false_type{}, b4);
          half_c(std::false_type{}, b0, b2);
        }
        b1 = b3;
      }
    }
    wait_vm_all();  // the repeated copies past the end
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
