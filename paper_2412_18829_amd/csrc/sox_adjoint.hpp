// Adjoint (vector-Jacobian product) kernels of the SOX step chain.
//
// With the cotangent of D, dD[P,R] = -(X^T R X)^T per tau, the loss
// L = sum_{P,R,v} dD[P,R] B[P,R,v] C[R,v,P] has four gradients that each
// contract a recomputed B or C tile, weighted by dD, over one of P or R:
//
//   dA[P,q,v]  = sum_R   dD[P,R] C[R,v,P] G_Rq[R,q]
//   dG_Rq[R,q] = sum_P,v dD[P,R] C[R,v,P] A[P,q,v]
//   dU2[R,v,w] = sum_P   dD[P,R] B[P,R,v] G_wP[w,P]     (summed over tau)
//   dG_wP[w,P] = sum_R,v dD[P,R] B[P,R,v] U2[R,v,w]
//
// hc_kernel evaluates all four ("Hadamard-contract"):
//   stage 1  M[z][x] = sum_k L[z][k] Rm[x][k]       (MFMA, k over nP)
//   stage 2  H = Wt[z][x] * M[z][x]                 (Wt = dD or dD^T)
//   stage 3  Out[x][y] += sum_z H[z][x] F[z][y]     (MFMA, F given as FT[y][z])
// The accumulator of stage 1 holds M[z = 16 i + acc_row(g, r)][x = li] in
// element r of lane (li, g); MFMA m of stage 3 takes that element r = m as
// its A operand A[x][k] with k = z.  The B operand then has to supply
// F[z][y] at the same z = 16 i + acc_row(g, m), i.e. FT[y0 + li][...], which
// is contiguous for float32 (4g..4g+3).  No LDS round trip is needed.
//
// Each wavefront owns 16 XB rows x of Out and all ny columns y; a
// workgroup (4 wavefronts) owns 64 XB rows.  The loops over inner tau / v
// accumulate in registers; outer tau / v come from the grid.
#pragma once

#include "sox_common.hpp"

namespace sox {

template <typename T, typename TC> struct HcArgs {
  const T* L;  long l_ld, l_ts, l_vs;
  const T* Rm; long r_ld, r_ts, r_vs;
  const T* W;  long w_ld, w_ts;
  const T* FT; long f_ld, f_ts, f_vs;
  TC* Out;     long o_ld, o_ts, o_vs;
  int nz, nk, ny;       // nz multiple of 32, nk and ny multiples of 16
  int tiles_x;
  int n_ot, n_ov, n_it, n_iv;
  int accumulate;
};

template <typename T>
__device__ __forceinline__ vec4_t<T> load_perm4(const T* row, int base, int g) {
  vec4_t<T> v;
#pragma unroll
  for (int m = 0; m < 4; ++m) v[m] = row[base + acc_row<T>(g, m)];
  return v;
}
template <>
__device__ __forceinline__ f32x4 load_perm4<float>(const float* row, int base, int g) {
  return *(const f32x4*)(row + base + 4 * g);
}

template <typename T, typename TC, int XB, int YB>
__global__ __launch_bounds__(256) void hc_kernel(const HcArgs<T, TC> p) {
  using V4 = vec4_t<T>;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = bid % p.tiles_x;
  const int rest = bid / p.tiles_x;
  const int ov = rest % p.n_ov;
  const int ot = rest / p.n_ov;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15;
  const int g = lane >> 4;
  const int x0 = tx * (64 * XB) + wave * (16 * XB);
  const int nyb = p.ny >> 4;

  V4 acc[XB][YB];
#pragma unroll
  for (int j = 0; j < XB; ++j)
#pragma unroll
    for (int yb = 0; yb < YB; ++yb) acc[j][yb] = zero4<T>();

  for (int it = 0; it < p.n_it; ++it) {
    for (int iv = 0; iv < p.n_iv; ++iv) {
      const long tau = (long)ot * p.n_it + it;
      const long v = (long)ov * p.n_iv + iv;
      const T* Lp = p.L + tau * p.l_ts + v * p.l_vs + 4 * g;
      const T* Rp = p.Rm + tau * p.r_ts + v * p.r_vs + 4 * g;
      const T* Wp = p.W + tau * p.w_ts;
      const T* Fp = p.FT + tau * p.f_ts + v * p.f_vs;
      for (int z0 = 0; z0 < p.nz; z0 += 32) {
        // cotangent weights of this z chunk, loaded ahead of stage 1
        T wt[2][XB][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < XB; ++j)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
              const int z = z0 + 16 * i + acc_row<T>(g, rr);
              wt[i][j][rr] = Wp[(long)z * p.w_ld + x0 + 16 * j + li];
            }
        V4 M[2][XB];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < XB; ++j) M[i][j] = zero4<T>();
        // stage 1, software-pipelined: the next k chunk's operands are
        // loaded before the current chunk's MFMAs
        V4 l[2], r[XB];
#pragma unroll
        for (int i = 0; i < 2; ++i) l[i] = *(const V4*)(Lp + (long)(z0 + 16 * i + li) * p.l_ld);
#pragma unroll
        for (int j = 0; j < XB; ++j) r[j] = *(const V4*)(Rp + (long)(x0 + 16 * j + li) * p.r_ld);
        for (int k0 = 0; k0 < p.nk; k0 += 16) {
          const int kn = k0 + 16 < p.nk ? k0 + 16 : k0;
          V4 ln[2], rn[XB];
#pragma unroll
          for (int i = 0; i < 2; ++i)
            ln[i] = *(const V4*)(Lp + (long)(z0 + 16 * i + li) * p.l_ld + kn);
#pragma unroll
          for (int j = 0; j < XB; ++j)
            rn[j] = *(const V4*)(Rp + (long)(x0 + 16 * j + li) * p.r_ld + kn);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < XB; ++j) M[i][j] = mfma16x16x4(l[i][m], r[j][m], M[i][j]);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < 2; ++i) l[i] = ln[i];
#pragma unroll
          for (int j = 0; j < XB; ++j) r[j] = rn[j];
        }
        // Hadamard with the cotangent tile
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < XB; ++j)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) M[i][j][rr] *= wt[i][j][rr];
        // contract over z: Out[x][y] += sum_z H[z][x] F[z][y], in groups of
        // four y blocks so that eight independent accumulators sit between
        // two MFMAs into the same one; the F rows of the next group are
        // loaded before the current group's MFMAs
        constexpr int YG = 4;
        V4 f[YG][2], fn[YG][2];
#pragma unroll
        for (int q = 0; q < YG; ++q) {
          const int yq = q < nyb ? q : nyb - 1;
          const T* frow = Fp + (long)(16 * yq + li) * p.f_ld;
#pragma unroll
          for (int i = 0; i < 2; ++i) f[q][i] = load_perm4<T>(frow, z0 + 16 * i, g);
        }
#pragma unroll
        for (int y0 = 0; y0 < YB; y0 += YG) {
          if (y0 < nyb) {
#pragma unroll
            for (int q = 0; q < YG; ++q) {
              int yq = y0 + YG + q;
              yq = yq < nyb ? yq : nyb - 1;
              const T* frow = Fp + (long)(16 * yq + li) * p.f_ld;
#pragma unroll
              for (int i = 0; i < 2; ++i) fn[q][i] = load_perm4<T>(frow, z0 + 16 * i, g);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int q = 0; q < YG; ++q)
#pragma unroll
                  for (int j = 0; j < XB; ++j)
                    if (y0 + q < YB && y0 + q < nyb)
                      acc[j][y0 + q] = mfma16x16x4(M[i][j][m], f[q][i][m], acc[j][y0 + q]);
#pragma unroll
            for (int q = 0; q < YG; ++q)
#pragma unroll
              for (int i = 0; i < 2; ++i) f[q][i] = fn[q][i];
          }
        }
      }
    }
  }

  TC* Ob = p.Out + (long)ot * p.o_ts + (long)ov * p.o_vs;
#pragma unroll
  for (int j = 0; j < XB; ++j)
#pragma unroll
    for (int yb = 0; yb < YB; ++yb) {
      if (yb < nyb) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const long off = (long)(x0 + 16 * j + acc_row<T>(g, rr)) * p.o_ld + 16 * yb + li;
          const TC val = TC(acc[j][yb][rr]);
          Ob[off] = p.accumulate ? Ob[off] + val : val;
        }
      }
    }
}

template <typename T, typename TC, int XB, int YB>
inline hipError_t launch_hc(HcArgs<T, TC> a, int nx, hipStream_t s) {
  if (nx % (64 * XB) != 0 || a.nz % 32 != 0 || a.nk % 16 != 0 || a.ny % 16 != 0 ||
      a.ny > 16 * YB)
    return hipErrorInvalidValue;
  a.tiles_x = nx / (64 * XB);
  const long nb = (long)a.tiles_x * a.n_ot * a.n_ov;
  if (nb <= 0) return hipSuccess;
  if (!grid_fits(nb, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((hc_kernel<T, TC, XB, YB>), dim3((unsigned)nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

// -----------------------------------------------------------------------------
// Layout helpers
//   out[b][c][r] = in[b][r][c]   (rows x cols per batch entry)
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* in, T* out, int rows, int cols,
                                                        long batch) {
  __shared__ T tile[32][33];
  const long b = blockIdx.z;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const T* ib = in + b * (long)rows * cols;
  T* ob = out + b * (long)rows * cols;
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = ib[(long)r * cols + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) ob[(long)c * rows + r] = tile[tx][k];
  }
}

template <typename T>
__global__ void fill_kernel(T* p, long count, T value) {
  SOX_FOR_FLAT(idx, count) p[idx] = value;
}

// dX[q][Q] += sum_s (M[Q][q][s] + M[Q][s][q]) X[s][Q]   (U-contraction adjoint)
__global__ void ut_adjoint_x_kernel(const double* M, const double* X, double* dX, int n, int Nthc,
                                    int nP) {
  SOX_FOR_FLAT(idx, (long)n * Nthc) {
    const int q = (int)(idx / Nthc), Q = (int)(idx - (idx / Nthc) * Nthc);
    const double* MQ = M + (long)Q * nP * nP;
    double acc = 0.0;
    for (int s = 0; s < n; ++s)
      acc += (MQ[(long)q * nP + s] + MQ[(long)s * nP + q]) * X[(long)s * Nthc + Q];
    dX[idx] += acc;
  }
}

}  // namespace sox
