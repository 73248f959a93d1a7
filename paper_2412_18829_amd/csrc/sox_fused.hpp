// Fused B, C -> D contraction over the auxiliary indices (the paper's B, C
// and D steps, the N^2 n^2 n_tau regime that dominates the SOX cost):
//
//   B^v[P,R] = sum_q A[P,q,v] Y[q,R]            (static: Y = G_Rq^T,
//                                                dynamic: Y = X, B_PRv = sum_u X_uR A_Puv)
//   C^v[R,P] = sum_w U2[R,v,w] G_wP
//   D[P,R]   = sum_v B^v[P,R] C^v[R,P]
//
// Both products of one v are MFMA tiles over the same [P, R] output block,
// so D is accumulated in registers by a Hadamard epilogue and B, C never
// reach memory.  Operands (all zero padded, K contiguous, 16-byte aligned):
//
//   A   [tau][v][P][q]   row stride nP   (the A step output)
//   Y   [tau][R][q]      row stride nP   (y_tstride = 0 shares one Y)
//   P2T [tau][P][w]      row stride nP   (G_wP transposed)
//   U2  R stride u_rstride, v stride u_vstride, w contiguous
//   D   [tau][P][R]      row stride NP
//
// One workgroup = 4 wavefronts (2 x 2) owns a (2 WP) x (2 WR) block of D for
// one tau and one range of v (the v sum may be split over several
// workgroups so that a launch fills whole rounds of the chip; the partial D
// blocks are summed ahead of the back-transform, by dsplit_sum_kernel in
// float64 and while D is widened to float64 in float32).  The loops run over v and
// 16-deep k chunks with the next chunk's operands loaded before the current
// chunk's MFMAs are issued; the Hadamard epilogue closes each v.
#pragma once

#include "sox_common.hpp"

namespace sox {

template <typename T> struct FusedArgs {
  const T* A;
  const T* Y;
  const T* P2T;
  const T* U2;
  T* D;
  long a_tstride, a_vstride;
  long y_tstride;
  long p_tstride;
  long u_rstride, u_vstride;
  long d_tstride;
  int accumulate;  // D += result (v processed in slabs)
  int n;      // orbitals: the v range
  int nP;     // padded k depth (multiple of 16)
  int NP;     // padded THC extent (multiple of the tile)
  int tiles_p, tiles_r, n_tau;
  // the v sum split over vsplit workgroups per tile (vchunk orbitals each,
  // every split non-empty); split s writes its partial D at D + s d_sstride
  int vsplit = 1;
  int vchunk = 0;
  long d_sstride = 0;
};

template <typename T, int WP, int WR>
__global__ __launch_bounds__(256) void fused_bcd_kernel(const FusedArgs<T> p) {
  using V4 = vec4_t<T>;
  constexpr int PB = WP / 16;
  constexpr int RB = WR / 16;
  const int nblocks = gridDim.x;
  const int bid0 = xcd_remap(blockIdx.x, nblocks);
  const int per_split = p.tiles_r * p.tiles_p * p.n_tau;
  const int sidx = bid0 / per_split;
  const int bid = bid0 - sidx * per_split;
  const int rt = bid % p.tiles_r;
  const int tmp = bid / p.tiles_r;
  const int pt = tmp % p.tiles_p;
  const int t = tmp / p.tiles_p;
  const int vbeg = p.vsplit > 1 ? sidx * p.vchunk : 0;
  const int vend = p.vsplit > 1 ? (vbeg + p.vchunk < p.n ? vbeg + p.vchunk : p.n) : p.n;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15;
  const int g = lane >> 4;
  const int P0 = pt * (2 * WP) + (wave >> 1) * WP;
  const int R0 = rt * (2 * WR) + (wave & 1) * WR;

  const long ld = p.nP;
  const T* Ab = p.A + t * p.a_tstride + (long)vbeg * p.a_vstride + (long)(P0 + li) * ld + 4 * g;
  const T* Yb = p.Y + t * p.y_tstride + (long)(R0 + li) * ld + 4 * g;
  const T* Pb = p.P2T + t * p.p_tstride + (long)(P0 + li) * ld + 4 * g;
  const T* Ub = p.U2 + (long)vbeg * p.u_vstride + (long)(R0 + li) * p.u_rstride + 4 * g;

  V4 accB[PB][RB], accC[PB][RB], dacc[PB][RB];
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      accB[i][j] = zero4<T>();
      accC[i][j] = zero4<T>();
      dacc[i][j] = zero4<T>();
    }

  const int KC = p.nP >> 4;
  const int nv = vend - vbeg;

  // Operands of the current chunk.  The next chunk is always loaded (the
  // last iteration re-loads chunk (n-1, KC-1), which stays in bounds) so the
  // loop body has no control flow around the loads and the wait for them
  // lands after this chunk's MFMAs have been issued.
  V4 a[PB], y[RB], pp[PB], u[RB];
#pragma unroll
  for (int i = 0; i < PB; ++i) {
    a[i] = *(const V4*)(Ab + (long)(16 * i) * ld);
    pp[i] = *(const V4*)(Pb + (long)(16 * i) * ld);
  }
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    y[j] = *(const V4*)(Yb + (long)(16 * j) * ld);
    u[j] = *(const V4*)(Ub + (long)(16 * j) * p.u_rstride);
  }

  for (int v = 0; v < nv; ++v) {
    for (int kc = 0; kc < KC; ++kc) {
      const bool wrap = (kc + 1 == KC);
      int vn = wrap ? v + 1 : v;
      int kn = wrap ? 0 : kc + 1;
      const bool last = vn >= nv;
      vn = last ? nv - 1 : vn;
      kn = last ? KC - 1 : kn;
      const long ko = (long)kn * 16;
      const T* Av = Ab + (long)vn * p.a_vstride + ko;
      const T* Uv = Ub + (long)vn * p.u_vstride + ko;
      V4 an[PB], yn[RB], pn[PB], un[RB];
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        an[i] = *(const V4*)(Av + (long)(16 * i) * ld);
        pn[i] = *(const V4*)(Pb + ko + (long)(16 * i) * ld);
      }
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        yn[j] = *(const V4*)(Yb + ko + (long)(16 * j) * ld);
        un[j] = *(const V4*)(Uv + (long)(16 * j) * p.u_rstride);
      }
      // keep the prefetch ahead of the MFMA block (and in its own registers)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < PB; ++i)
#pragma unroll
          for (int j = 0; j < RB; ++j) {
            accB[i][j] = mfma16x16x4(a[i][m], y[j][m], accB[i][j]);
            accC[i][j] = mfma16x16x4(pp[i][m], u[j][m], accC[i][j]);
          }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < PB; ++i) { a[i] = an[i]; pp[i] = pn[i]; }
#pragma unroll
      for (int j = 0; j < RB; ++j) { y[j] = yn[j]; u[j] = un[j]; }
    }
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        dacc[i][j] += accB[i][j] * accC[i][j];
        accB[i][j] = zero4<T>();
        accC[i][j] = zero4<T>();
      }
  }

  T* Db = p.D + t * p.d_tstride + (long)sidx * p.d_sstride;
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int j = 0; j < RB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int P = P0 + 16 * i + acc_row<T>(g, r);
        const int R = R0 + 16 * j + li;
        const long off = (long)P * p.NP + R;
        Db[off] = p.accumulate ? Db[off] + dacc[i][j][r] : dacc[i][j][r];
      }
}

template <typename T, int WP, int WR>
inline hipError_t launch_fused(const FusedArgs<T>& a, hipStream_t s) {
  const long nb = (long)a.tiles_p * a.tiles_r * a.n_tau * (a.vsplit > 1 ? a.vsplit : 1);
  if (nb <= 0) return hipSuccess;
  if (!grid_fits(nb, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fused_bcd_kernel<T, WP, WR>), dim3((unsigned)nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

// D[i] (+)= sum_{s=1}^{ns-1} D[s stride + i]: adds the partial D blocks of
// the v splits into the first one.
template <typename T>
__global__ __launch_bounds__(256) void dsplit_sum_kernel(T* D, long count, long stride, int ns) {
  SOX_FOR_FLAT(i, count) {
    T acc = D[i];
    for (int s = 1; s < ns; ++s) acc += D[(long)s * stride + i];
    D[i] = acc;
  }
}

}  // namespace sox
