// Operand-access structs for the smaller contractions of the adjoint chain
// (float64 on the generic MFMA GEMM).  Notation as in sox_adjoint.hpp; b is
// the tau index inside the current slab, t0 the slab's first node, and
// G(beta - tau) is node n_tau - 1 - tau.
#pragma once

#include "sox_common.hpp"
#include "sox_gemm.hpp"

namespace sox {

// E[b][t][P] = sum_r R[t0+b][t][r] X[r][P]   (trans = 0: R X)
// E[b][t][P] = sum_r R[t0+b][r][t] X[r][P]   (trans = 1: R^T X)
struct RXProb {
  const double* R;  // [n_tau][n][n]
  const double* X;  // [n][N]
  double* E;        // [slab][n][NP]
  int n, Nthc, NP, t0, trans;
  int M, N, K;      // n, Nthc, n
  __device__ f64x4 loadA4(int b, int t, int r) const {
    if (t >= n) return zero4<double>();
    const double* Rb = R + (long)(t0 + b) * n * n;
    return trans ? load4_strided<double>(Rb + t, n, r, n) : load4_strided<double>(Rb + (long)t * n, 1, r, n);
  }
  __device__ f64x4 loadB4(int, int P, int r) const {
    if (P >= Nthc) return zero4<double>();
    return load4_strided<double>(X + P, Nthc, r, n);
  }
  __device__ void store(int b, int t, int P, double v) const { E[((long)b * n + t) * NP + P] = v; }
};

// Cotangent of D:  dD[P][R] = -(X^T R X)[R][P], stored as dD and dD^T:
//   dDT[b][R][P] = dD[b][P][R] = -sum_t X[t][R] E[b][t][P]
template <typename T> struct DDProb {
  const double* X;
  const double* E;  // [slab][n][NP]  (R X)
  T* dD;            // [slab][NP][NP]
  T* dDT;           // [slab][NP][NP]
  int n, Nthc, NP;
  int M, N, K;      // NP, NP, n
  __device__ f64x4 loadA4(int, int Rr, int t) const {
    if (Rr >= Nthc) return zero4<double>();
    return load4_strided<double>(X + Rr, Nthc, t, n);
  }
  __device__ f64x4 loadB4(int b, int P, int t) const {
    if (P >= Nthc) return zero4<double>();
    return load4_strided<double>(E + (long)b * n * NP + P, NP, t, n);
  }
  __device__ void store(int b, int Rr, int P, double v) const {
    const long base = (long)b * NP * NP;
    dDT[base + (long)Rr * NP + P] = T(-v);
    dD[base + (long)P * NP + Rr] = T(-v);
  }
};

// dU1t[(P,q)][s] += sum_{b,v} dA[b][v][(P,q)] G_sv(beta - tau_b)
struct DU1tProb {
  const double* dA;  // [slab][n][NP*nP]
  const double* G;
  double* dU1t;      // [NP*nP][nP]
  int n, nP, NP, n_tau, t0;
  int M, N, K;       // NP*nP, nP, slab*n
  __device__ f64x4 loadA4(int, int row, int k) const {
    return load4_strided<double>(dA + row, (long)NP * nP, k, K);
  }
  __device__ f64x4 loadB4(int, int sI, int k) const {
    f64x4 r;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int kk = k + m;
      const int b = kk / n, v = kk - (kk / n) * n;
      r[m] = (kk < K && sI < n) ? G[(long)(n_tau - 1 - (t0 + b)) * n * n + (long)sI * n + v] : 0.0;
    }
    return r;
  }
  __device__ void store(int, int row, int sI, double v) const { dU1t[(long)row * nP + sI] += v; }
};

// dG[n_tau-1-(t0+b)][s][v] += sum_(P,q) U1t[(P,q)][s] dA[b][v][(P,q)]
template <typename T> struct DGbProb {
  const T* U1t;       // [NP*nP][nP]
  const double* dA;   // [slab][n][NP*nP]
  double* dG;
  int n, nP, NP, n_tau, t0;
  int M, N, K;        // n, n, NP*nP
  __device__ f64x4 loadA4(int, int sI, int k) const {
    if (sI >= n) return zero4<double>();
    return load4_strided<double>(U1t + sI, nP, k, K);
  }
  __device__ f64x4 loadB4(int b, int v, int k) const {
    if (v >= n) return zero4<double>();
    return load4_strided<double>(dA + ((long)b * n + v) * NP * nP, 1, k, K);
  }
  __device__ void store(int b, int sI, int v, double val) const {
    dG[(long)(n_tau - 1 - (t0 + b)) * n * n + (long)sI * n + v] += val;
  }
};

// dG[t0+b][u][q] += sum_R X[u][R] dP1[b][R][q]            (which = 0)
// dG[t0+b][w][p] += sum_P dP2T[b][P][w] X[p][P]            (which = 1)
struct DGProjProb {
  const double* X;
  const double* dP;   // [slab][NP][nP]
  double* dG;
  int n, Nthc, nP, NP, t0, which;
  int M, N, K;        // n, n, Nthc
  __device__ f64x4 loadA4(int b, int row, int k) const {
    if (row >= n) return zero4<double>();
    if (which == 0) return load4_strided<double>(X + (long)row * Nthc, 1, k, Nthc);
    return load4_strided<double>(dP + (long)b * NP * nP + row, nP, k, Nthc);
  }
  __device__ f64x4 loadB4(int b, int col, int k) const {
    if (col >= n) return zero4<double>();
    if (which == 0) return load4_strided<double>(dP + (long)b * NP * nP + col, nP, k, Nthc);
    return load4_strided<double>(X + (long)col * Nthc, 1, k, Nthc);
  }
  __device__ void store(int b, int row, int col, double v) const {
    dG[(long)(t0 + b) * n * n + (long)row * n + col] += v;
  }
};

// dX[u][R] += sum_{b,q} G[t0+b][u][q] dP1[b][R][q]          (which = 0)
// dX[p][P] += sum_{b,w} G[t0+b][w][p] dP2T[b][P][w]         (which = 1)
struct DXProjProb {
  const double* G;
  const double* dP;   // [slab][NP][nP]
  double* dX;
  int n, Nthc, nP, NP, t0;
  int which;
  int M, N, K;        // n, Nthc, slab*nP  (k = b*nP + q)
  __device__ f64x4 loadA4(int, int u, int k) const {
    f64x4 r;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int kk = k + m;
      const int b = kk / nP, q = kk - (kk / nP) * nP;
      double v = 0.0;
      if (kk < K && q < n && u < n) {
        const double* Gb = G + (long)(t0 + b) * n * n;
        v = which == 0 ? Gb[(long)u * n + q] : Gb[(long)q * n + u];
      }
      r[m] = v;
    }
    return r;
  }
  __device__ f64x4 loadB4(int, int Rr, int k) const {
    if (Rr >= Nthc) return zero4<double>();
    f64x4 r;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int kk = k + m;
      const int b = kk / nP, q = kk - (kk / nP) * nP;
      r[m] = (kk < K) ? dP[(long)b * NP * nP + (long)Rr * nP + q] : 0.0;
    }
    return r;
  }
  __device__ void store(int, int u, int Rr, double v) const { dX[(long)u * Nthc + Rr] += v; }
};

// back-transform adjoint:
//   dX[a][R] -= sum_{b,P} E[b][a][P] D[b][P][R]     (trans = 0, E = R X)
//   dX[a][R] -= sum_{b,P} E[b][a][P] D[b][R][P]     (trans = 1, E = R^T X)
template <typename Td> struct DXBackProb {
  const double* E;   // [slab][n][NP]
  const Td* D;       // [slab][NP][NP]
  double* dX;
  int n, Nthc, NP, trans;
  int M, N, K;       // n, Nthc, slab*NP  (k = b*NP + P)
  __device__ f64x4 loadA4(int, int a, int k) const {
    f64x4 r;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int kk = k + m;
      const int b = kk / NP, P = kk - (kk / NP) * NP;
      r[m] = (kk < K && P < Nthc && a < n) ? E[((long)b * n + a) * NP + P] : 0.0;
    }
    return r;
  }
  __device__ f64x4 loadB4(int, int Rr, int k) const {
    if (Rr >= Nthc) return zero4<double>();
    f64x4 r;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int kk = k + m;
      const int b = kk / NP, P = kk - (kk / NP) * NP;
      double v = 0.0;
      if (kk < K && P < Nthc) {
        const Td* Db = D + (long)b * NP * NP;
        v = trans ? double(Db[(long)Rr * NP + P]) : double(Db[(long)P * NP + Rr]);
      }
      r[m] = v;
    }
    return r;
  }
  __device__ void store(int, int a, int Rr, double v) const { dX[(long)a * Nthc + Rr] -= v; }
};

// U-contraction adjoint.  dUt(P, (q,s)) is read from
//   layout 0: dUt[P][q][s]  (NP x nP x nP)      layout 1: dUt[q][P][s] (nP x NP x nP)
//   dU[P][Q] (+)= sum_(q,s) dUt(P,(q,s)) X[q][Q] X[s][Q]
struct DUProb {
  const double* dUt;
  const double* X;
  double* dU;        // [N][N]
  int n, Nthc, nP, NP, layout, accumulate;
  int M, N, K;       // Nthc, Nthc, nP*nP
  __device__ double at(int P, int k) const {
    const int q = k / nP, sI = k - (k / nP) * nP;
    return layout == 0 ? dUt[((long)P * nP + q) * nP + sI] : dUt[((long)q * NP + P) * nP + sI];
  }
  __device__ f64x4 loadA4(int, int P, int k) const {
    f64x4 r;
#pragma unroll
    for (int m = 0; m < 4; ++m) r[m] = (P < Nthc && k + m < K) ? at(P, k + m) : 0.0;
    return r;
  }
  __device__ f64x4 loadB4(int, int Q, int k) const {
    f64x4 r;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int kk = k + m;
      const int q = kk / nP, sI = kk - (kk / nP) * nP;
      r[m] = (Q < Nthc && kk < K && q < n && sI < n) ? X[(long)q * Nthc + Q] * X[(long)sI * Nthc + Q] : 0.0;
    }
    return r;
  }
  __device__ void store(int, int P, int Q, double v) const {
    const long off = (long)P * Nthc + Q;
    dU[off] = accumulate ? dU[off] + v : v;
  }
};

//   Mq[Q][(q,s)] = sum_P U[P][Q] dUt(P,(q,s))      (feeds the dX term of the U-contraction)
struct DUMProb {
  const double* U;
  const double* dUt;
  double* Mq;        // [NP][nP*nP]
  int n, Nthc, nP, NP, layout;
  int M, N, K;       // Nthc, nP*nP, Nthc
  __device__ f64x4 loadA4(int, int Q, int P) const {
    if (Q >= Nthc) return zero4<double>();
    return load4_strided<double>(U + Q, Nthc, P, Nthc);
  }
  __device__ f64x4 loadB4(int, int k, int P) const {
    const int q = k / nP, sI = k - (k / nP) * nP;
    f64x4 r;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int PP = P + m;
      double v = 0.0;
      if (PP < Nthc && k < N)
        v = layout == 0 ? dUt[((long)PP * nP + q) * nP + sI] : dUt[((long)q * NP + PP) * nP + sI];
      r[m] = v;
    }
    return r;
  }
  __device__ void store(int, int Q, int k, double v) const { Mq[(long)Q * nP * nP + k] = v; }
};

}  // namespace sox

namespace sox {

// ---------------------------------------------------------------------------
// Dynamic-path adjoints (transforms in float64).
//
// IFT adjoint for the v-slab:  dAW[m][c NP + P][vl n + u] = sum_tau Tb2[tau][k] dAdyn[tau][vl][P][u]
// (k = c n_omega + m), stored twice: dAW (rows (c,P), ld ldk) and dAWT
// (rows (vl,u), ld 2NP).
template <typename T> struct IFTAdjProb {
  const double* Tb2;    // [n_tau][2 n_omega]
  const double* dAdyn;  // [n_tau][vc][NP][nP]
  T* dAW;               // [n_omega][2NP][ldk]
  T* dAWT;              // [n_omega][vc*n][2NP]
  int n, nP, NP, n_omega, n_tau, vc, ldk;
  int M, N, K;          // M = 2 n_omega, N = NP*vc*n, K = n_tau
  __device__ f64x4 loadA4(int, int row, int t) const {
    if (row >= M) return zero4<double>();
    return load4_strided<double>(Tb2 + row, 2L * n_omega, t, n_tau);
  }
  __device__ f64x4 loadB4(int, int col, int t) const {
    if (col >= N) return zero4<double>();
    const int u = col % n, pv = col / n;
    const int vl = pv % vc, P = pv / vc;
    return load4_strided<double>(dAdyn + ((long)vl * NP + P) * nP + u, (long)vc * NP * nP, t, n_tau);
  }
  __device__ void store(int, int row, int col, double v) const {
    const int c = row / n_omega, m = row - (row / n_omega) * n_omega;
    const int u = col % n, pv = col / n;
    const int vl = pv % vc, P = pv / vc;
    const long vu = (long)vl * n + u;
    dAW[((long)m * 2 * NP + (long)c * NP + P) * ldk + vu] = T(v);
    dAWT[((long)m * vc * n + vu) * (2L * NP) + (long)c * NP + P] = T(v);
  }
};

// FT adjoint:  dGG[tau][(vl,u)][Q] = sum_k Tf2[k][tau] dGG2[m][(vl,u)][c NP + Q]
struct FTAdjProb {
  const double* Tf2;    // [2 n_omega][n_tau]
  const double* dGG2;   // [n_omega][vc*n][2NP]
  double* dGG;          // [n_tau][vc*n][NP]
  int n, NP, n_omega, n_tau, vc;
  int M, N, K;          // M = n_tau, N = vc*n*NP, K = 2 n_omega
  __device__ f64x4 loadA4(int, int t, int k) const {
    if (t >= M) return zero4<double>();
    return load4_strided<double>(Tf2 + t, n_tau, k, 2 * n_omega);
  }
  __device__ f64x4 loadB4(int, int col, int k) const {
    if (col >= N) return zero4<double>();
    const int Q = col % NP, vu = col / NP;
    f64x4 r;
#pragma unroll
    for (int mm = 0; mm < 4; ++mm) {
      const int kk = k + mm;
      if (kk < 2 * n_omega) {
        const int c = kk / n_omega, m = kk - (kk / n_omega) * n_omega;
        r[mm] = dGG2[((long)m * vc * n + vu) * (2L * NP) + (long)c * NP + Q];
      } else {
        r[mm] = 0.0;
      }
    }
    return r;
  }
  __device__ void store(int, int t, int col, double v) const { dGG[(long)t * N + col] = v; }
};

// dW_tau[j][P][Q] = sum_k Tf2[k][j] dWc[m](P,Q) with dWr = dW2[00] + dW2[11],
// dWi = dW2[10] - dW2[01] (blocks of the real 2NP x 2NP form)
struct DWtauProb {
  const double* Tf2;   // [2 n_omega][n_tau]
  const double* dW2;   // [n_omega][2NP][2NP]
  double* dW;          // [n_tau][N][N]
  int Nthc, NP, n_omega, n_tau;
  int M, N, K;         // M = n_tau, N = Nthc*Nthc, K = 2 n_omega
  __device__ f64x4 loadA4(int, int j, int k) const {
    if (j >= M) return zero4<double>();
    return load4_strided<double>(Tf2 + j, n_tau, k, 2 * n_omega);
  }
  __device__ f64x4 loadB4(int, int col, int k) const {
    if (col >= N) return zero4<double>();
    const int P = col / Nthc, Q = col - (col / Nthc) * Nthc;
    const long ld = 2L * NP;
    f64x4 r;
#pragma unroll
    for (int mm = 0; mm < 4; ++mm) {
      const int kk = k + mm;
      double v = 0.0;
      if (kk < 2 * n_omega) {
        const int c = kk / n_omega, m = kk - (kk / n_omega) * n_omega;
        const double* W = dW2 + (long)m * ld * ld;
        v = c == 0 ? W[(long)P * ld + Q] + W[(long)(NP + P) * ld + NP + Q]
                   : W[(long)(NP + P) * ld + Q] - W[(long)P * ld + NP + Q];
      }
      r[mm] = v;
    }
    return r;
  }
  __device__ void store(int, int j, int col, double v) const { dW[(long)j * N + col] = v; }
};

// eq:GG product rule for the v-slab:
//   dP2T[tau][Q][u]           += sum_vl dGG[tau][(vl,u)][Q] P1[n_tau-1-tau][Q][v0+vl]
//   dP1[n_tau-1-tau][Q][v0+vl] += sum_u  dGG[tau][(vl,u)][Q] P2T[tau][Q][u]
__global__ void gg_adjoint_p2_kernel(const double* dGG, const double* P1, double* dP2T, int n,
                                     int nP, int NP, int Nthc, int n_tau, int v0, int vc) {
  SOX_FOR_FLAT(idx, (long)n_tau * Nthc * n) {
    const int t = (int)(idx / ((long)Nthc * n));
    const int rem = (int)(idx - (long)t * Nthc * n);
    const int Q = rem / n, u = rem - (rem / n) * n;
    const double* p1 = P1 + ((long)(n_tau - 1 - t) * NP + Q) * nP + v0;
    const double* g = dGG + (long)t * vc * n * NP + (long)u * NP + Q;
    double acc = 0.0;
    for (int vl = 0; vl < vc; ++vl) acc += g[(long)vl * n * NP] * p1[vl];
    dP2T[((long)t * NP + Q) * nP + u] += acc;
  }
}

__global__ void gg_adjoint_p1_kernel(const double* dGG, const double* P2T, double* dP1, int n,
                                     int nP, int NP, int Nthc, int n_tau, int v0, int vc) {
  SOX_FOR_FLAT(idx, (long)n_tau * Nthc * vc) {
    const int t = (int)(idx / ((long)Nthc * vc));
    const int rem = (int)(idx - (long)t * Nthc * vc);
    const int Q = rem / vc, vl = rem - (rem / vc) * vc;
    const double* p2 = P2T + ((long)t * NP + Q) * nP;
    const double* g = dGG + ((long)t * vc * n + (long)vl * n) * NP + Q;
    double acc = 0.0;
    for (int u = 0; u < n; ++u) acc += g[(long)u * NP] * p2[u];
    dP1[((long)(n_tau - 1 - t) * NP + Q) * nP + v0 + vl] += acc;
  }
}

// XP[u][R] = X[u][R] zero padded to nP x NP;  dX[u][R] += dXT[R][u]
template <typename T>
__global__ void xpad_kernel(const double* X, T* out, int n, int Nthc, int nP, int NP) {
  SOX_FOR_FLAT(idx, (long)nP * NP) {
    const int u = (int)(idx / NP), R = (int)(idx - (idx / NP) * NP);
    out[idx] = (u < n && R < Nthc) ? T(X[(long)u * Nthc + R]) : T(0);
  }
}

__global__ void add_transposed_kernel(const double* dXT, double* dX, int n, int Nthc, int nP) {
  SOX_FOR_FLAT(idx, (long)n * Nthc) {
    const int u = (int)(idx / Nthc), R = (int)(idx - (idx / Nthc) * Nthc);
    dX[idx] += dXT[(long)R * nP + u];
  }
}

}  // namespace sox
