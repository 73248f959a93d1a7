// THC-GW direct term: the GW self-energy of fig:diag (its dynamic part, the
// screened line W_d between the same two points as the propagator),
//
//   Sigma_ij(tau) = - sum_kl (ik|lj)_{W_d(tau)} G_kl(tau),
//
// on the same THC factors as the SOX chain (section "THC-SOX and THC-SOSEX"):
// with (ik|lj) = sum_PQ X_iP X_kP W_PQ X_lQ X_jQ the sum factorises into the
// chain's half projection G_Rl = sum_k X_kR G_kl, one more projection, an
// elementwise product with W_d(tau) and the back-transform,
//
//   molecule:  Gt[R][Q] = sum_l G_Rl X_lQ
//              M[R][Q]  = -Gt[R][Q] W[R][Q]
//              Sigma    = X M X^T
//   mesh:      Gt^{k'}[R][Q] = sum_l G^{k'}_Rl conj(X^{k'}_lQ)
//              M^k[R][Q]     = -(1/N_k) sum_{k'} W^{k-k'}[R][Q] Gt^{k'}[R][Q]
//              Sigma^k       = conj(X^k) M^k X^k^T
//
// O(n_tau N^2 n) per momentum pair: a factor n below the SOX chain's
// contractions, so every step runs in float64 (MFMA for the products).  The
// molecular products are problem structs of the generic GEMM (sox_gemm.hpp);
// the mesh products use the batched complex product (sox_complex.hpp); the
// momentum convolution is its own kernel below.
#pragma once

#include "sox_common.hpp"
#include "sox_complex.hpp"
#include "sox_gemm.hpp"

namespace sox {

// M[t][R][Q] = -W[t0 + t][R][Q] sum_l P1[t][R][l] X[l][Q]   (rows R, columns Q)
struct GwHadProb {
  const double* P1;  // [slab][N][n]   G_Rl
  const double* X;   // [n][N]
  const double* W;   // [n_tau][N][N]
  double* out;       // [slab][N][N]
  int n, Nthc, t0;
  int M, N, K;       // M = N = Nthc, K = n
  __device__ f64x4 loadA4(int b, int R, int l) const {
    if (R >= Nthc) return zero4<double>();
    return load4_strided<double>(P1 + ((long)b * Nthc + R) * n, 1, l, n);
  }
  __device__ f64x4 loadB4(int, int Q, int l) const {
    if (Q >= Nthc) return zero4<double>();
    return load4_strided<double>(X + Q, Nthc, l, n);
  }
  __device__ void store(int b, int R, int Q, double v) const {
    const long e = (long)R * Nthc + Q;
    out[(long)b * Nthc * Nthc + e] = -v * W[(long)(t0 + b) * Nthc * Nthc + e];
  }
};

// Y[t][i][Q] = sum_R X[i][R] M[t][R][Q]   (rows i, columns Q, depth R)
struct GwLeftProb {
  const double* X;   // [n][N]
  const double* Mt;  // [slab][N][N]
  double* out;       // [slab][n][N]
  int n, Nthc;
  int M, N, K;       // M = n, N = K = Nthc
  __device__ f64x4 loadA4(int, int i, int R) const {
    if (i >= n) return zero4<double>();
    return load4_strided<double>(X + (long)i * Nthc, 1, R, Nthc);
  }
  __device__ f64x4 loadB4(int b, int Q, int R) const {
    if (Q >= Nthc) return zero4<double>();
    return load4_strided<double>(Mt + (long)b * Nthc * Nthc + Q, Nthc, R, Nthc);
  }
  __device__ void store(int b, int i, int Q, double v) const {
    out[((long)b * n + i) * Nthc + Q] = v;
  }
};

// Sigma[t0 + t][i][j] = sum_Q Y[t][i][Q] X[j][Q]   (rows i, columns j, depth Q)
struct GwRightProb {
  const double* Y;   // [slab][n][N]
  const double* X;   // [n][N]
  double* out;       // [n_tau][n][n]
  int n, Nthc, t0;
  int M, N, K;       // M = N = n, K = Nthc
  __device__ f64x4 loadA4(int b, int i, int Q) const {
    if (i >= n) return zero4<double>();
    return load4_strided<double>(Y + ((long)b * n + i) * Nthc, 1, Q, Nthc);
  }
  __device__ f64x4 loadB4(int, int j, int Q) const {
    if (j >= n) return zero4<double>();
    return load4_strided<double>(X + (long)j * Nthc, 1, Q, Nthc);
  }
  __device__ void store(int b, int i, int j, double v) const {
    out[((long)(t0 + b) * n + i) * n + j] = v;
  }
};

// Momentum convolution of the mesh term, interleaved complex float64:
//   M[k][t][e] = alpha * sum_{k'} W[kdiff[k][k']][t0 + t][e] Gt[k'][t][e],
// e = R * N + Q.  A workgroup takes E consecutive elements of one node t
// (workgroup index = t * nblk_e + element block), copies every momentum's
// Gt and W values of them into LDS (nk * E <= kGwLdsC each, coalesced over
// e), then thread (e, g) forms outputs k = g, g + 256 / E, ... from LDS.
// Each Gt and W value is read from memory once and each M value written once.
constexpr int kGwLdsC = 2048;

__global__ __launch_bounds__(256) void gw_conv_kernel(const double* __restrict__ W,
                                                      const double* __restrict__ Gt,
                                                      double* __restrict__ Mo,
                                                      const int* __restrict__ kdiff, int nk,
                                                      int E, long NN, int slab, int t0, int n_tau,
                                                      double alpha, long nblk_e) {
  __shared__ f64x2 sg[kGwLdsC];
  __shared__ f64x2 sw[kGwLdsC];
  const long blk = blockIdx.x;
  const int t = (int)(blk / nblk_e);
  const long e0 = (blk - (long)t * nblk_e) * E;
  for (int idx = threadIdx.x; idx < nk * E; idx += 256) {
    const int kk = idx / E, e = idx - kk * E;
    const long ee = e0 + e;
    f64x2 g = {0.0, 0.0}, w = {0.0, 0.0};
    if (ee < NN) {
      g = *(const f64x2*)(Gt + 2 * (((long)kk * slab + t) * NN + ee));
      w = *(const f64x2*)(W + 2 * (((long)kk * n_tau + t0 + t) * NN + ee));
    }
    sg[idx] = g;
    sw[idx] = w;
  }
  __syncthreads();
  const int e = threadIdx.x % E, g0 = threadIdx.x / E, ng = 256 / E;
  const long ee = e0 + e;
  if (ee >= NN) return;
  for (int k = g0; k < nk; k += ng) {
    const int* kd = kdiff + (long)k * nk;
    double re = 0.0, im = 0.0;
    for (int kp = 0; kp < nk; ++kp) {
      const f64x2 w = sw[kd[kp] * E + e], g = sg[kp * E + e];
      re += w.x * g.x - w.y * g.y;
      im += w.x * g.y + w.y * g.x;
    }
    f64x2 o;
    o.x = alpha * re;
    o.y = alpha * im;
    *(f64x2*)(Mo + 2 * (((long)k * slab + t) * NN + ee)) = o;
  }
}

// The same convolution for a mesh known at compile time (M1 x M2 x M3
// momenta, index (a * M2 + b) * M3 + c, axes of length 1, 2 or 3), by the
// convolution theorem on the momentum group: with F[f](xi) = sum_k f[k]
// w^(xi.k), F[M] = alpha F[W] F[Gt] and M = F^-1[F[M]] (the D step's
// in-register butterflies, mesh_dft).  One work-item per (t, e) loads every
// momentum's W and Gt value (all loads issued before any arithmetic), so each
// value is read from memory once and each M value written once; the
// arithmetic is n_k log n_k per element instead of n_k^2.
template <int M1, int M2, int M3>
__global__ __launch_bounds__(256) void gw_conv_mesh_kernel(const double* __restrict__ W,
                                                           const double* __restrict__ Gt,
                                                           double* __restrict__ Mo, long NN,
                                                           int slab, int t0, int n_tau,
                                                           double alpha, long count) {
  constexpr int NK = M1 * M2 * M3;
  SOX_FOR_FLAT(idx, count) {
    const long t = idx / NN, e = idx - t * NN;
    double wr[NK], wi[NK], gr[NK], gi[NK];
#pragma unroll
    for (int q = 0; q < NK; ++q) {
      const f64x2 w = *(const f64x2*)(W + 2 * (((long)q * n_tau + t0 + t) * NN + e));
      wr[q] = w.x;
      wi[q] = w.y;
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const f64x2 g = *(const f64x2*)(Gt + 2 * (((long)k * slab + t) * NN + e));
      gr[k] = g.x;
      gi[k] = g.y;
    }
    mesh_dft<double, +1, M1, M2, M3>(wr, wi);
    mesh_dft<double, +1, M1, M2, M3>(gr, gi);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const double r = wr[k] * gr[k] - wi[k] * gi[k];
      wi[k] = wr[k] * gi[k] + wi[k] * gr[k];
      wr[k] = r;
    }
    mesh_dft<double, -1, M1, M2, M3>(wr, wi);
    const double f = alpha / NK;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      f64x2 o;
      o.x = f * wr[k];
      o.y = f * wi[k];
      *(f64x2*)(Mo + 2 * (((long)k * slab + t) * NN + e)) = o;
    }
  }
}

// Element-block width of gw_conv_kernel: the largest power of two <= 64
// with nk * E <= kGwLdsC (nk <= 256 gives E >= 8); it divides 256.
inline int gw_conv_width(int nk) {
  int E = 64;
  while (E > 8 && nk * E > kGwLdsC) E >>= 1;
  return E;
}

}  // namespace sox
