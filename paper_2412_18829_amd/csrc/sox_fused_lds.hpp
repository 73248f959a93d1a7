// LDS-staged fused B, C -> D contraction (the same products as
// fused_bcd_kernel in sox_fused.hpp), for float32 operands on the 16x16x4
// float32 MFMA and for split-precision operands (x = hi + lo in bf16,
// hi hi + hi lo + lo hi on the 16x16x32 bf16 MFMA, float32 accumulation).
//
// A workgroup owns a 128 x 128 block of D for one tau and one range of v,
// split over four wavefronts of 64 x 64 (PB = 4: 4 x 4 MFMA tiles each, one
// wavefront per SIMD) or eight of 32 x 64 (PB = 2: 2 x 4 tiles, two per
// SIMD, so one wavefront's MFMAs cover the other's LDS reads).  The v
// sum runs in stages of one v and one 64-byte k chunk (16 float32 or 32
// bf16 values), and each stage in two halves: the B half needs the P-row
// panel of A^v and the R-row panel of Y, the C half the P-row panel of
// G_wP^T and the R-row panel of U2^v, 128 rows x 64 bytes per panel and
// plane (hi and lo are separate planes).  The halves are copied straight
// from global memory into a ring of five LDS buffers (16-byte global-to-LDS
// loads, no registers in between), four halves ahead of the MFMAs.  Each
// panel row is read from LDS by the wavefronts that share it, so the
// operand traffic through the vector cache is that of the workgroup tile,
// not of the wave tiles, and the fragments of half h + 1 are read into a
// second register set while the MFMAs of half h run.
//
// One barrier per half h, after the wavefront has waited for its own copies
// of half h + 2 (copies of halves h + 3 and h + 4 stay in flight; the
// barrier carries no memory fence, which would wait for them too): the copy
// issued in half h overwrites the buffer of half h - 1, whose fragments
// every wavefront consumed before the barrier that ends half h - 1.  Past
// the last stage the copy cursor repeats the last stage, so every half
// issues the same number of copies and the wait stays exact; the kernel
// drains them before it ends.
//
// LDS rows are 64 bytes (four 16-byte segments); segment c of row r sits at
// position c ^ ((r >> 1) & 3), so the 16-byte reads of eight consecutive
// rows at one k group cover all banks once.  Lane (li, g) reads segment g of
// row li: k = 4g..4g+3 for float32 (MFMA step m takes k = 4g + m in both
// operands) and k = 8g..8g+7 for bf16.  The Hadamard epilogue of v is folded
// into the first stage of v + 1: the first MFMA of each B and C tile starts
// from zero, and the products of the previous v are added to D just before.
#pragma once

#include <type_traits>

#include "sox_common.hpp"

namespace sox {

enum { kLdsBf16x3 = 0, kLdsFp32 = 1 };

struct LdsFusedArgs {
  // panel planes (hi then lo in split precision; one plane in float32)
  const char* bp[2];  // B half, P rows: A^v      [tau][v][P][k]
  const char* br[2];  // B half, R rows: Y        [tau][R][k]
  const char* cp[2];  // C half, P rows: G_wP^T   [tau][P][k]
  const char* cr[2];  // C half, R rows: U2^v     R stride u_rstride, v stride u_vstride
  long a_tstride, a_vstride, y_tstride, p_tstride, u_rstride, u_vstride;  // elements
  long d_tstride, d_sstride;  // float32 D: tau and v-split strides
  float* D;
  int accumulate;
  int n, nP, NP;      // v range, k depth (64-byte chunks), padded THC extent
  int tiles_p, tiles_r, n_tau;
  int vsplit, vchunk;  // split s sums v in [s vchunk, (s+1) vchunk)
};

// Fragments of one half stage: PB 16-row blocks of the P rows (first MFMA
// operand) and four of the R rows.
template <int MODE, int PB> struct LdsFrags;
template <int PB> struct LdsFrags<kLdsBf16x3, PB> {
  bf16x8 ah[PB], al[PB], bh[4], bl[4];
};
template <int PB> struct LdsFrags<kLdsFp32, PB> {
  f32x4 a[PB], b[4];
};

template <int MODE> struct LdsMode;
template <> struct LdsMode<kLdsBf16x3> {
  static constexpr int kPlanes = 2;  // hi, lo
  static constexpr int kEsize = 2;
  typedef LdsFrags<kLdsBf16x3, 4> Frags;
};
template <> struct LdsMode<kLdsFp32> {
  static constexpr int kPlanes = 1;
  static constexpr int kEsize = 4;
  typedef LdsFrags<kLdsFp32, 4> Frags;
};

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kLdsTile = 128;             // rows of each staged panel
constexpr int kLdsPieces = kLdsTile * 4;  // 16-byte pieces per panel plane
constexpr int kLdsBufs = 5;               // ring of half-stage buffers
constexpr int kLdsAhead = kLdsBufs - 1;   // halves copied ahead of the MFMAs

template <int MODE, int NPL, int PB = 4>
__device__ __forceinline__ void lds_frags(const u32x4 (*buf)[kLdsPieces], const int* sa,
                                          const int* sy, LdsFrags<MODE, PB>& f) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (MODE == kLdsBf16x3) {
      if (i < PB) {
        f.ah[i] = __builtin_bit_cast(bf16x8, buf[0][sa[i]]);
        f.al[i] = __builtin_bit_cast(bf16x8, buf[1][sa[i]]);
      }
      f.bh[i] = __builtin_bit_cast(bf16x8, buf[NPL][sy[i]]);
      f.bl[i] = __builtin_bit_cast(bf16x8, buf[NPL + 1][sy[i]]);
    } else {
      if (i < PB) f.a[i] = __builtin_bit_cast(f32x4, buf[0][sa[i]]);
      f.b[i] = __builtin_bit_cast(f32x4, buf[NPL][sy[i]]);
    }
  }
}

// the same from separate plane sets: P rows from pp[0 .. NPL), R rows from
// rp[0 .. NPL)
template <int MODE, int NPL, int PB = 4>
__device__ __forceinline__ void lds_frags2(const u32x4 (*pp)[kLdsPieces],
                                           const u32x4 (*rp)[kLdsPieces], const int* sa,
                                           const int* sy, LdsFrags<MODE, PB>& f) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (MODE == kLdsBf16x3) {
      if (i < PB) {
        f.ah[i] = __builtin_bit_cast(bf16x8, pp[0][sa[i]]);
        f.al[i] = __builtin_bit_cast(bf16x8, pp[1][sa[i]]);
      }
      f.bh[i] = __builtin_bit_cast(bf16x8, rp[0][sy[i]]);
      f.bl[i] = __builtin_bit_cast(bf16x8, rp[1][sy[i]]);
    } else {
      if (i < PB) f.a[i] = __builtin_bit_cast(f32x4, pp[0][sa[i]]);
      f.b[i] = __builtin_bit_cast(f32x4, rp[0][sy[i]]);
    }
  }
}

// acc (+)= one 64-byte k chunk of the product; FIRST starts from zero
template <int MODE, bool FIRST, int PB = 4>
__device__ __forceinline__ void lds_half_mfma(const LdsFrags<MODE, PB>& f, f32x4 (*acc)[4]) {
  if constexpr (MODE == kLdsBf16x3) {
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = mfma16x16x32bf16(f.ah[i], f.bh[j], FIRST ? zero4<float>() : acc[i][j]);
        acc[i][j] = mfma16x16x32bf16(f.ah[i], f.bl[j], acc[i][j]);
        acc[i][j] = mfma16x16x32bf16(f.al[i], f.bh[j], acc[i][j]);
      }
  } else {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int i = 0; i < PB; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = mfma16x16x4(f.a[i][m], f.b[j][m],
                                  (FIRST && m == 0) ? zero4<float>() : acc[i][j]);
  }
}

// PB = 4: four wavefronts of 64 x 64; PB = 2: eight wavefronts of 32 x 64
// (the P rows of the workgroup tile split four ways), two per SIMD.
//
// RES: the two v-independent panels (Y for the B half, G_wP^T for the C
// half) are copied into LDS once, for every k chunk, when the workgroup
// starts, and stay resident for the whole v sum; the ring then carries only
// the v-dependent panels (A^v, U2^v), half the copies and LDS writes per
// half.  For K up to lds_res_chunks 64-byte chunks (nP <= 64: 144 KB of
// LDS in bf16 x 3).
template <int MODE> constexpr int lds_res_chunks() { return MODE == kLdsBf16x3 ? 2 : 1; }

template <int MODE, int PB = 4, bool RES = false>
__global__ __launch_bounds__(1024 / PB) void fused_bcd_lds_kernel(const LdsFusedArgs p) {
  static_assert(PB == 2 || PB == 4, "32 or 64 P rows per wavefront");
  constexpr int NPL = LdsMode<MODE>::kPlanes;
  constexpr int ES = LdsMode<MODE>::kEsize;
  constexpr int NW = 16 / PB;           // wavefronts
  constexpr int CP = PB / 2;            // copies per wavefront, panel and plane
  constexpr int RPL = RES ? NPL : 2 * NPL;  // ring planes per half
  constexpr int kCopies = RPL * CP;        // copies per wavefront and half
  constexpr int RC = RES ? lds_res_chunks<MODE>() : 1;
  // ring: [buffer][plane: P rows (hi, lo), then R rows (hi, lo); RES: the
  // half's v-dependent panel only][row * 4 + swizzled segment]
  __shared__ u32x4 lds[kLdsBufs][RPL][kLdsPieces];
  // RES: [k chunk][plane: Y rows (hi, lo), then G_wP^T rows (hi, lo)][...]
  __shared__ u32x4 res[RC][RES ? 2 * NPL : 1][RES ? kLdsPieces : 1];
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

  // Copies: instruction h of wavefront w fills LDS pieces 64 c .. 64 c + 63
  // (c = w + NW h) of a plane, one 16-byte piece per lane at position 64 c +
  // lane, i.e. row 16 c + lane / 4 and swizzled segment lane % 4.  Sources
  // are a wave-uniform base (tau, v, k chunk) plus a 32-bit byte offset per
  // lane (the launcher checks the panels' extents).
  unsigned orow_p[CP], orow_r[CP], orow_u[CP];
#pragma unroll
  for (int h = 0; h < CP; ++h) {
    const int c = wave + NW * h;
    const int row = 16 * c + (lane >> 2);
    const unsigned seg = (unsigned)((lane & 3) ^ ((row >> 1) & 3));
    orow_p[h] = (unsigned)(P0 + row) * (unsigned)(p.nP * ES) + 16u * seg;
    orow_r[h] = (unsigned)(R0 + row) * (unsigned)(p.nP * ES) + 16u * seg;
    orow_u[h] = (unsigned)(R0 + row) * (unsigned)(p.u_rstride * ES) + 16u * seg;
  }
  const long ot_a = (long)t * p.a_tstride * ES, ot_y = (long)t * p.y_tstride * ES;
  const long ot_p = (long)t * p.p_tstride * ES;
  // fragment positions: P rows (wave >> 1) 16 PB + 16 i + li, R rows (wave & 1) 64 + 16 j + li
  int sa[4], sy[4];
  const int sw = g ^ ((li >> 1) & 3);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sa[i] = ((wave >> 1) * 16 * PB + 16 * (i < PB ? i : 0) + li) * 4 + sw;
    sy[i] = ((wave & 1) * 64 + 16 * i + li) * 4 + sw;
  }

  f32x4 accB[PB][4], accC[PB][4], dacc[PB][4];
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      accB[i][j] = zero4<float>();
      accC[i][j] = zero4<float>();
      dacc[i][j] = zero4<float>();
    }

  const int KC = p.nP * ES / 64;
  const int nst = v_end > v_begin ? (v_end - v_begin) * KC : 0;
  // copy cursor: the stage whose halves are copied next, held at the last
  // stage once every stage is under way
  int cv = v_begin, ckc = 0, cs = 0;
  auto copy_panels = [&](u32x4 (*buf)[kLdsPieces], const char* const* srcp, long offp,
                         const char* const* srcr, long offr, const unsigned* orr) {
#pragma unroll
    for (int q = 0; q < NPL; ++q)
#pragma unroll
      for (int h = 0; h < CP; ++h) {
        const int ch = 64 * (wave + NW * h);
        global_to_lds16(srcp[q] + offp + orow_p[h], &buf[q][ch]);
        global_to_lds16(srcr[q] + offr + orr[h], &buf[NPL + q][ch]);
      }
  };
  // one panel's planes (RES)
  auto copy_one = [&](u32x4 (*buf)[kLdsPieces], const char* const* src, long off,
                      const unsigned* orr) {
#pragma unroll
    for (int q = 0; q < NPL; ++q)
#pragma unroll
      for (int h = 0; h < CP; ++h)
        global_to_lds16(src[q] + off + orr[h], &buf[q][64 * (wave + NW * h)]);
  };
  auto copy_b = [&](int b) {
    const long ko = (long)ckc * 64;
    if constexpr (RES)
      copy_one(lds[b], p.bp, ot_a + (long)cv * p.a_vstride * ES + ko, orow_p);
    else
      copy_panels(lds[b], p.bp, ot_a + (long)cv * p.a_vstride * ES + ko, p.br, ot_y + ko,
                  orow_r);
  };
  auto copy_c = [&](int b) {
    const long ko = (long)ckc * 64;
    if constexpr (RES)
      copy_one(lds[b], p.cr, (long)cv * p.u_vstride * ES + ko, orow_u);
    else
      copy_panels(lds[b], p.cp, ot_p + ko, p.cr, (long)cv * p.u_vstride * ES + ko, orow_u);
    const int adv = cs + 1 < nst ? 1 : 0;  // selects, no branch: one block per half
    cs += adv;
    ckc += adv;
    const int wrap = ckc == KC ? 1 : 0;
    ckc = wrap ? 0 : ckc;
    cv += wrap;
  };

  // fragments of the B half of stage (v, kc) in buffer b, and of its C half
  auto frags_b = [&](int b, int kc, LdsFrags<MODE, PB>& f) {
    if constexpr (RES) lds_frags2<MODE, NPL, PB>(lds[b], res[kc], sa, sy, f);
    else lds_frags<MODE, NPL, PB>(lds[b], sa, sy, f);
  };
  auto frags_c = [&](int b, int kc, LdsFrags<MODE, PB>& f) {
    if constexpr (RES) lds_frags2<MODE, NPL, PB>(res[kc] + NPL, lds[b], sa, sy, f);
    else lds_frags<MODE, NPL, PB>(lds[b], sa, sy, f);
  };

  if (nst > 0) {
    LdsFrags<MODE, PB> f0, f1;
    if constexpr (RES) {
      // the resident panels of every k chunk first (they complete before
      // any ring copy, so the ring's counted waits cover them)
      for (int kc = 0; kc < KC; ++kc) {
        copy_one(res[kc], p.br, ot_y + (long)kc * 64, orow_r);
        copy_one(res[kc] + NPL, p.cp, ot_p + (long)kc * 64, orow_p);
      }
    }
    // halves 0..3 (stages 0 and 1) in flight, then halves 0 and 1 landed
    copy_b(0);
    copy_c(1);
    copy_b(2);
    copy_c(3);
    wait_vm<kCopies * (kLdsAhead - 2)>();
    barrier_nofence();
    frags_b(0, 0, f0);
    int b1 = 1;  // buffer of half 2 s + 1
    // B half of stage s: copy half 2 s + 4 into the buffer of half 2 s - 1,
    // read the C-half fragments, MFMAs from f0.  C half: copy half 2 s + 5
    // into the buffer of half 2 s, read the next B-half fragments, MFMAs
    // from f1.  Each half is one basic block (no branch between its copies,
    // fragment reads and MFMAs), which leaves the compiler free to overlap
    // them.
    auto half_b = [&](auto first, int bcopy, int kc) {
      constexpr bool F = decltype(first)::value;
      copy_b(bcopy);
      frags_c(b1, kc, f1);
      if constexpr (F) {
#pragma unroll
        for (int i = 0; i < PB; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) dacc[i][j] += accB[i][j] * accC[i][j];
      }
      lds_half_mfma<MODE, F, PB>(f0, accB);
      wait_vm<kCopies * (kLdsAhead - 2)>();
      barrier_nofence();
    };
    auto half_c = [&](auto first, int bcopy, int bread, int kcn) {
      constexpr bool F = decltype(first)::value;
      copy_c(bcopy);
      frags_b(bread, kcn, f0);
      lds_half_mfma<MODE, F, PB>(f1, accC);
      wait_vm<kCopies * (kLdsAhead - 2)>();
      barrier_nofence();
    };
    for (int v = v_begin; v < v_end; ++v) {
      for (int kc = 0; kc < KC; ++kc) {
        const int b0 = b1 == 0 ? kLdsBufs - 1 : b1 - 1;  // half 2 s
        const int b2 = b1 + 1 == kLdsBufs ? 0 : b1 + 1;  // half 2 s + 2
        const int b3 = b2 + 1 == kLdsBufs ? 0 : b2 + 1;  // half 2 s + 3
        const int b4 = b3 + 1 == kLdsBufs ? 0 : b3 + 1;  // half 2 s + 4
        const int kcn = kc + 1 == KC ? 0 : kc + 1;  // k chunk of the next stage
        if (kc == 0) {
          half_b(std::true_type{}, b4, kc);
          half_c(std::true_type{}, b0, b2, kcn);
        } else {
          half_b(std::false_type{}, b4, kc);
          half_c(std::false_type{}, b0, b2, kcn);
        }
        b1 = b3;
      }
    }
    wait_vm<0>();  // the repeated copies past the end
  }
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) dacc[i][j] += accB[i][j] * accC[i][j];

  float* Db = p.D + (long)sp * p.d_sstride + (long)t * p.d_tstride;
  const int Pw = P0 + (wave >> 1) * 16 * PB, Rw = R0 + (wave & 1) * 64;
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long off = (long)(Pw + 16 * i + 4 * g + r) * p.NP + Rw + 16 * j + li;
        Db[off] = p.accumulate ? Db[off] + dacc[i][j][r] : dacc[i][j][r];
      }
}

// the resident-panel form applies: split precision (in float32 it measured
// slower, 1.16 -> 1.24 ms per fused launch at n = 64, N = 384, 64 nodes:
// its single-plane ring halves are already small) and every k chunk's Y and
// G_wP^T panels fit (bf16 x 3 at n = 64, N = 384: 0.496 -> 0.472 ms)
template <int MODE> inline bool fused_lds_resident(int nP) {
  return MODE == kLdsBf16x3 && nP * LdsMode<MODE>::kEsize / 64 <= lds_res_chunks<MODE>();
}

// Grid: (R tile, P tile, tau, v split), R tiles fastest; 1024 / PB threads.
template <int MODE, int PB = 4>
inline hipError_t launch_fused_lds(const LdsFusedArgs& a, hipStream_t s) {
  constexpr long ES = LdsMode<MODE>::kEsize;
  if ((a.nP * ES) % 64 != 0 || a.NP % kLdsTile != 0 || a.tiles_p * kLdsTile != a.NP ||
      a.tiles_r * kLdsTile != a.NP || a.vsplit < 1 || a.vchunk < 1)
    return hipErrorInvalidValue;
  // lane offsets within one (tau, v) panel set are 32-bit
  if ((long)a.NP * a.nP * ES >= (1L << 32) || (long)a.NP * a.u_rstride * ES >= (1L << 32))
    return hipErrorInvalidValue;
  const long nb = (long)a.tiles_p * a.tiles_r * a.n_tau * a.vsplit;
  if (nb <= 0) return hipSuccess;
  if (!grid_fits(nb, 1024 / PB)) return hipErrorInvalidValue;
  if (fused_lds_resident<MODE>(a.nP))
    hipLaunchKernelGGL((fused_bcd_lds_kernel<MODE, PB, true>), dim3((unsigned)nb), dim3(1024 / PB),
                       0, s, a);
  else
    hipLaunchKernelGGL((fused_bcd_lds_kernel<MODE, PB, false>), dim3((unsigned)nb),
                       dim3(1024 / PB), 0, s, a);
  return hipGetLastError();
}

}  // namespace sox
