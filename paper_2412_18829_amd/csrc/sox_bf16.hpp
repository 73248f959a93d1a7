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
  const long nb = (long)a.tiles_p * a.tiles_r * a.n_tau;
  if (nb <= 0) return hipSuccess;
  if (a.nP % 32 != 0 || !grid_fits(nb, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fused_bcd_bf16x3_kernel<WP, WR>), dim3((unsigned)nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace sox
