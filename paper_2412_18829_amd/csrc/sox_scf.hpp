// Device kernels of the minimal self-consistent Dyson loop (section
// "Definitions": eq:Dyson, eq:G0 with S = I, eq:E1b), one spin channel of a
// molecule, float64 throughout:
//
//   gamma_pq = -G_qp(beta^-) = -sum_i t_beta[i] G_qp(tau_i)
//   Sigma^HF = J - K: J_ij = sum_P X_iP X_jP (V rho)_P, rho_Q = sum_kl X_kQ gamma_lk X_lQ
//              (K comes from the GW chain with W = V and G = gamma)
//   Sigma(i nu_m) = sum_j T_fwd[m][j] Sigma(tau_j)
//   G(i nu_m) = [(i nu_m + mu) I - h - Sigma^HF - Sigma(i nu_m)]^-1
//   G(tau_i) = Re sum_m T_bwd[i][m] G(i nu_m),  N = -sum_i t_beta[i] Tr G(tau_i)
//   (mu: the root of N(mu) = n_elec, found on the host by a bracketing search)
//   G <- (1 - a) G + a G_new,  delta = max |G_new - G|
//   E_inf = sum_pq (h + Sigma^HF / 2)_pq gamma_pq
//
// The Dyson inversions are batched Gauss-Jordan eliminations with partial
// pivoting, one workgroup per frequency, on the matrices in device memory.
#pragma once

#include "sox_common.hpp"

namespace sox {

constexpr int kScfMaxN = 1024;    // orbitals at most (LDS column of the Dyson kernel)
constexpr int kScfThreads = 1024;  // threads of a Dyson workgroup (one frequency each)

// gamma[p][q] = -sum_i tb[i] G[i][q][p]
__global__ void scf_density_kernel(const double* G, const double* tb, int n, int nt, double* gam) {
  const long nn = (long)n * n;
  SOX_FOR_FLAT(e, nn) {
    const int p = (int)(e / n), q = (int)(e - (long)p * n);
    double acc = 0.0;
    for (int i = 0; i < nt; ++i) acc += tb[i] * G[(long)i * nn + (long)q * n + p];
    gam[e] = -acc;
  }
}

// rho[Q] = sum_kl X[k][Q] gamma[l][k] X[l][Q]
__global__ void scf_rho_kernel(const double* X, const double* gam, int n, int N, double* rho) {
  SOX_FOR_FLAT(Q, N) {
    double acc = 0.0;
    for (int k = 0; k < n; ++k) {
      double t = 0.0;
      for (int l = 0; l < n; ++l) t += gam[(long)l * n + k] * X[(long)l * N + Q];
      acc += X[(long)k * N + Q] * t;
    }
    rho[Q] = acc;
  }
}

// v[P] = sum_Q V[P][Q] rho[Q]
__global__ void scf_matvec_kernel(const double* V, const double* rho, int N, double* v) {
  SOX_FOR_FLAT(P, N) {
    double acc = 0.0;
    for (int Q = 0; Q < N; ++Q) acc += V[(long)P * N + Q] * rho[Q];
    v[P] = acc;
  }
}

// shf = exch + J, J[i][j] = sum_P X[i][P] X[j][P] v[P]; heff = h + shf
__global__ void scf_hartree_kernel(const double* X, const double* v, const double* exch,
                                   const double* h, int n, int N, double* shf, double* heff) {
  const long nn = (long)n * n;
  SOX_FOR_FLAT(e, nn) {
    const int i = (int)(e / n), j = (int)(e - (long)i * n);
    double acc = 0.0;
    for (int P = 0; P < N; ++P) acc += X[(long)i * N + P] * X[(long)j * N + P] * v[P];
    shf[e] = exch[e] + acc;
    heff[e] = h[e] + shf[e];
  }
}

// out[m][e] = sum_j Tf[m][j] S[j][e] (Tf complex [nm][nt], S real, out complex)
__global__ void scf_ft_kernel(const double* Tf, const double* S, int nt, int nm, long nn,
                              double* out) {
  SOX_FOR_FLAT(idx, (long)nm * nn) {
    const long m = idx / nn, e = idx - m * nn;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < nt; ++j) {
      const double s = S[(long)j * nn + e];
      re += Tf[2 * (m * nt + j)] * s;
      im += Tf[2 * (m * nt + j) + 1] * s;
    }
    out[2 * idx] = re;
    out[2 * idx + 1] = im;
  }
}

// Ginv[m] = [(i nu_m + mu) I - heff - Snu[m]]^-1, one workgroup of
// kScfThreads per m (the widest workgroup: each elimination step is one pass
// over the matrix in memory, so more waves keep more of it in flight)
__global__ __launch_bounds__(kScfThreads) void scf_dyson_kernel(const double* heff,
                                                                const double* Snu,
                                                                const double* nu, double mu,
                                                                int n, double* Aw, double* Gi) {
  const int m = blockIdx.x;
  const int tid = threadIdx.x;
  const long nn = (long)n * n;
  double* A = Aw + 2 * (long)m * nn;
  double* R = Gi + 2 * (long)m * nn;
  const double* S = Snu + 2 * (long)m * nn;
  const double w = nu[m];
  for (long e = tid; e < nn; e += kScfThreads) {
    const int i = (int)(e / n), j = (int)(e - (long)i * n);
    double re = -heff[e] - S[2 * e], im = -S[2 * e + 1];
    if (i == j) {
      re += mu;
      im += w;
    }
    A[2 * e] = re;
    A[2 * e + 1] = im;
    R[2 * e] = i == j ? 1.0 : 0.0;
    R[2 * e + 1] = 0.0;
  }
  __shared__ double fr[kScfMaxN], fi[kScfMaxN];
  __shared__ double pv[kScfThreads];
  __shared__ int pix[kScfThreads];
  __shared__ double inv_r, inv_i;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot: the largest |A[i][k]|, i >= k
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < n; i += kScfThreads) {
      const double ar = A[2 * ((long)i * n + k)], ai = A[2 * ((long)i * n + k) + 1];
      const double a = ar * ar + ai * ai;
      if (a > best) {
        best = a;
        bi = i;
      }
    }
    pv[tid] = best;
    pix[tid] = bi;
    __syncthreads();
    for (int s = kScfThreads / 2; s > 0; s >>= 1) {
      if (tid < s && pv[tid + s] > pv[tid]) {
        pv[tid] = pv[tid + s];
        pix[tid] = pix[tid + s];
      }
      __syncthreads();
    }
    int r = pix[0];
    r = r < k ? k : (r > n - 1 ? n - 1 : r);
    if (r != k) {
      for (int j = tid; j < n; j += kScfThreads) {
        for (int c = 0; c < 2; ++c) {
          double* a1 = A + 2 * ((long)k * n + j) + c;
          double* a2 = A + 2 * ((long)r * n + j) + c;
          const double t = *a1;
          *a1 = *a2;
          *a2 = t;
          double* b1 = R + 2 * ((long)k * n + j) + c;
          double* b2 = R + 2 * ((long)r * n + j) + c;
          const double u = *b1;
          *b1 = *b2;
          *b2 = u;
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      const double pr = A[2 * ((long)k * n + k)], pi = A[2 * ((long)k * n + k) + 1];
      const double d = pr * pr + pi * pi;
      inv_r = pr / d;
      inv_i = -pi / d;
    }
    __syncthreads();
    const double ir = inv_r, ii = inv_i;
    for (int j = tid; j < n; j += kScfThreads) {
      double* a = A + 2 * ((long)k * n + j);
      double* b = R + 2 * ((long)k * n + j);
      const double ar = a[0], ai = a[1], br = b[0], bi2 = b[1];
      a[0] = ar * ir - ai * ii;
      a[1] = ar * ii + ai * ir;
      b[0] = br * ir - bi2 * ii;
      b[1] = br * ii + bi2 * ir;
    }
    __syncthreads();
    for (int i = tid; i < n; i += kScfThreads) {
      fr[i] = A[2 * ((long)i * n + k)];
      fi[i] = A[2 * ((long)i * n + k) + 1];
    }
    __syncthreads();
    for (long e = tid; e < nn; e += kScfThreads) {
      const int i = (int)(e / n);
      if (i == k) continue;
      const int j = (int)(e - (long)i * n);
      const double f_r = fr[i], f_i = fi[i];
      if (j > k) {  // columns <= k of A are not read again
        const double* ak = A + 2 * ((long)k * n + j);
        double* a = A + 2 * e;
        a[0] -= f_r * ak[0] - f_i * ak[1];
        a[1] -= f_r * ak[1] + f_i * ak[0];
      }
      const double* bk = R + 2 * ((long)k * n + j);
      double* b = R + 2 * e;
      b[0] -= f_r * bk[0] - f_i * bk[1];
      b[1] -= f_r * bk[1] + f_i * bk[0];
    }
    __syncthreads();
  }
}

// G[i][e] = Re sum_m Tb[i][m] Gi[m][e] (Tb complex [nt][nm])
__global__ void scf_ift_kernel(const double* Tb, const double* Gi, int nt, int nm, long nn,
                               double* G) {
  SOX_FOR_FLAT(idx, (long)nt * nn) {
    const long i = idx / nn, e = idx - i * nn;
    double acc = 0.0;
    for (int m = 0; m < nm; ++m)
      acc += Tb[2 * (i * nm + m)] * Gi[2 * ((long)m * nn + e)] -
             Tb[2 * (i * nm + m) + 1] * Gi[2 * ((long)m * nn + e) + 1];
    G[idx] = acc;
  }
}

// out[0] = -sum_i tb[i] Tr G[i]   (one workgroup of 256)
__global__ __launch_bounds__(256) void scf_count_kernel(const double* G, const double* tb, int n,
                                                        int nt, double* out) {
  double acc = 0.0;
  const long nn = (long)n * n;
  for (long idx = threadIdx.x; idx < (long)nt * n; idx += 256) {
    const long i = idx / n, p = idx - i * n;
    acc += tb[i] * G[i * nn + p * n + p];
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = -red[0];
}

// G = (1 - a) G + a Gn; bmax[block] = max |Gn - G| over the block's elements
__global__ __launch_bounds__(256) void scf_mix_kernel(double* G, const double* Gn, double a,
                                                      long count, double* bmax) {
  double mx = 0.0;
  SOX_FOR_FLAT(e, count) {
    const double g = G[e], gn = Gn[e];
    mx = fmax(mx, fabs(gn - g));
    G[e] = (1.0 - a) * g + a * gn;
  }
  __shared__ double red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) bmax[blockIdx.x] = red[0];
}

// out[0] = max of bmax[0 .. nb); out[1] = sum (h + shf / 2) * gamma (one workgroup)
__global__ __launch_bounds__(256) void scf_reduce_kernel(const double* bmax, int nb,
                                                         const double* h, const double* shf,
                                                         const double* gam, long nn,
                                                         double* out) {
  double mx = 0.0, acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) mx = fmax(mx, bmax[b]);
  for (long e = threadIdx.x; e < nn; e += 256) acc += (h[e] + 0.5 * shf[e]) * gam[e];
  __shared__ double rm[256], ra[256];
  rm[threadIdx.x] = mx;
  ra[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + s]);
      ra[threadIdx.x] += ra[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = rm[0];
    out[1] = ra[0];
  }
}

__global__ void scf_add_kernel(double* a, const double* b, long count) {
  SOX_FOR_FLAT(e, count) a[e] += b[e];
}

}  // namespace sox
