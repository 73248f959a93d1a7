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
// The Dyson inversions are batched Gauss-Jordan inversions in place with
// partial pivoting, one workgroup per frequency, the matrix in LDS when it
// fits.
#pragma once

#include "sox_common.hpp"

namespace sox {

constexpr int kScfMaxN = 1024;    // orbitals at most (LDS row and column of the Dyson kernel)
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

// rho[Q] = sum_kl X[k][Q] gamma[l][k] X[l][Q]: one workgroup of kScfThreads
// per 64 columns Q (one per lane), the k sum split over the wavefronts
__global__ __launch_bounds__(kScfThreads) void scf_rho_kernel(const double* X, const double* gam,
                                                              int n, int N, double* rho) {
  constexpr int NW = kScfThreads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int Q = blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (Q < N)
    for (int k = wave; k < n; k += NW) {
      double t = 0.0;
      for (int l = 0; l < n; ++l) t += gam[(long)l * n + k] * X[(long)l * N + Q];
      acc += X[(long)k * N + Q] * t;
    }
  __shared__ double part[NW][64];
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && Q < N) {
    double r = 0.0;
    for (int w = 0; w < NW; ++w) r += part[w][lane];
    rho[Q] = r;
  }
}

// v[P] = sum_Q V[P][Q] rho[Q]: one wavefront per row P (256 threads)
__global__ __launch_bounds__(256) void scf_matvec_kernel(const double* V, const double* rho, int N,
                                                         double* v) {
  const int lane = threadIdx.x & 63;
  const int P = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (P >= N) return;
  double acc = 0.0;
  for (int Q = lane; Q < N; Q += 64) acc += V[(long)P * N + Q] * rho[Q];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) v[P] = acc;
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
// kScfThreads per m: Gauss-Jordan inversion in place with partial pivoting.
// Step k: the pivot row r >= k of largest |A[r][k]| (a wavefront max
// reduction, then one over the wavefronts), rows k and r exchanged, row k
// scaled by 1 / p with its own column-k entry taken as 1 (so A[k][k] becomes
// 1 / p), then every other row i loses f_i times row k with its column-k
// entry taken as 0 (f_i = A[i][k] before the step), which leaves -f_i / p
// there.  After the last step the inverse of the row-exchanged matrix is in
// place; exchanging columns k and r_k for k = n - 1 down to 0 undoes the
// row exchanges.  Three barriers per step.  LDS: the matrix is held in
// LDS (n <= kScfLdsN) and written out at the end; otherwise it is
// eliminated in place in Gi (2 n^2 doubles per frequency, read through the
// cache).
constexpr int kScfLdsN = 96;  // largest n held in LDS (147 KB)

struct __attribute__((aligned(16))) ScfC {  // one complex double (16-byte loads)
  double x, y;
  __host__ __device__ ScfC() = default;
  __host__ __device__ constexpr ScfC(double a, double b) : x(a), y(b) {}
};

template <bool LDS>
__global__ __launch_bounds__(kScfThreads) void scf_dyson_kernel(const double* heff,
                                                                const double* Snu,
                                                                const double* nu, double mu,
                                                                int n, double* Gi) {
  constexpr int NW = kScfThreads / 64;
  constexpr int NR = LDS ? kScfLdsN : kScfMaxN;
  const int m = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const long nn = (long)n * n;
  ScfC* R = reinterpret_cast<ScfC*>(Gi) + (long)m * nn;
  const ScfC* S = reinterpret_cast<const ScfC*>(Snu) + (long)m * nn;
  __shared__ ScfC lmat[LDS ? kScfLdsN * kScfLdsN : 1];
  __shared__ ScfC row[NR], col[NR];
  __shared__ int perm[NR];
  __shared__ unsigned long long wkey[NW];
  __shared__ ScfC wval[NW];
  ScfC* A = LDS ? lmat : R;
  // the elements e = tid + kScfThreads t as (row, column): stepped without
  // divisions (the stride in columns is below n)
  const int nn32 = n * n;
  const int di = kScfThreads / n, dj = kScfThreads - di * n;
  const int i0 = tid / n, j0 = tid - i0 * n;
  const double w = nu[m];
  for (int e = tid, i = i0, j = j0; e < nn32; e += kScfThreads) {
    const ScfC sv = S[e];
    ScfC a = ScfC(-heff[e] - sv.x, -sv.y);
    if (i == j) {
      a.x += mu;
      a.y += w;
    }
    A[e] = a;
    i += di;
    j += dj;
    if (j >= n) {
      j -= n;
      ++i;
    }
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot: the largest |A[i][k]| over i >= k, as the largest key
    // bits(|A[i][k]|^2) with its low 10 bits replaced by 1023 - i (non-negative
    // doubles order as their bit patterns; among values equal to 2^-42
    // relative the smaller i wins); 0: no row.  n <= 128: wavefront 0 alone,
    // else every wavefront and then a pass over their winners.
    const bool one = n <= 128;
    if (!one || wave == 0) {
      unsigned long long key = 0;
      ScfC bv = ScfC(0.0, 0.0);
      const int i_begin = k + (one ? lane : tid), i_step = one ? 64 : kScfThreads;
      for (int i = i_begin; i < n; i += i_step) {
        const ScfC a = A[(long)i * n + k];
        const double q = a.x * a.x + a.y * a.y;
        const unsigned long long kk =
            (__builtin_bit_cast(unsigned long long, q) & ~1023ull) | (unsigned)(1023 - i);
        if (kk > key) {
          key = kk;
          bv = a;
        }
      }
      unsigned long long wmax = key;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long ok = __shfl_xor(wmax, o);
        wmax = ok > wmax ? ok : wmax;
      }
      if (key == wmax && wmax != 0) wval[wave] = bv;  // the row is unique
      if (lane == 0) wkey[wave] = wmax;
    }
    __syncthreads();
    int wbest = 0;
    if (!one)
      for (int q = 1; q < NW; ++q)
        if (wkey[q] > wkey[wbest]) wbest = q;
    const unsigned long long kbest = wkey[wbest];
    int r = 1023 - (int)(kbest & 1023ull);
    const ScfC p = kbest != 0 ? wval[wbest] : ScfC(0.0, 0.0);
    r = kbest == 0 || r < k ? k : (r > n - 1 ? n - 1 : r);
    const double d = p.x * p.x + p.y * p.y;
    const double ir = p.x / d, ii = -p.y / d;
    // exchange rows k and r, scale row k (each column j by one thread); the
    // column of multipliers (rows k and r by the owner of column k)
    for (int j = tid; j < n; j += kScfThreads) {
      const ScfC ak = A[(long)k * n + j];
      const ScfC ar = r != k ? A[(long)r * n + j] : ak;
      if (r != k) A[(long)r * n + j] = ak;
      const ScfC x = j == k ? ScfC(1.0, 0.0) : ar;
      const ScfC y = ScfC(x.x * ir - x.y * ii, x.x * ii + x.y * ir);
      A[(long)k * n + j] = y;
      row[j] = y;
      if (j == k) {
        col[k] = ScfC(0.0, 0.0);
        if (r != k) col[r] = ak;
      }
    }
    for (int i = tid; i < n; i += kScfThreads)
      if (i != k && i != r) col[i] = A[(long)i * n + k];
    if (tid == 0) perm[k] = r;
    __syncthreads();
    for (int e = tid, i = i0, j = j0; e < nn32; e += kScfThreads) {
      if (i != k) {
        const ScfC f = col[i], y = row[j];
        ScfC a = j == k ? ScfC(0.0, 0.0) : A[e];
        a.x -= f.x * y.x - f.y * y.y;
        a.y -= f.x * y.y + f.y * y.x;
        A[e] = a;
      }
      i += di;
      j += dj;
      if (j >= n) {
        j -= n;
        ++i;
      }
    }
    __syncthreads();
  }
  // undo the row exchanges: column exchanges in reverse order, each row by
  // one thread
  for (int i = tid; i < n; i += kScfThreads)
    for (int k = n - 1; k >= 0; --k) {
      const int r = perm[k];
      if (r != k) {
        const ScfC t = A[(long)i * n + k];
        A[(long)i * n + k] = A[(long)i * n + r];
        A[(long)i * n + r] = t;
      }
    }
  if constexpr (LDS) {
    __syncthreads();
    for (int e = tid; e < nn32; e += kScfThreads) R[e] = A[e];
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
