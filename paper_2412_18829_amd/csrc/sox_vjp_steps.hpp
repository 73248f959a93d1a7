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
