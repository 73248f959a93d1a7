// Operand-access structs that map each step of the SOX chain onto the
// generic MFMA GEMM (sox_gemm.hpp), plus the elementwise kernels.
//
// Padded extents: nP = n rounded up to 16 (the MFMA k chunk), NP = N rounded
// up to the fused kernel's workgroup tile.  Every intermediate the fused
// kernel reads is stored with these extents and zeros in the padding, which
// the producers below write by masking their loads to the true extents.
#pragma once

#include "sox_common.hpp"
#include "sox_gemm.hpp"

namespace sox {

// ---------------------------------------------------------------------------
// U-contraction (eq:U_contraction, molecule):
//   Ut[P][q][s] = sum_Q U[P][Q] X[q][Q] X[s][Q]       (float64 MFMA)
// GEMM rows P, columns (q, s) flattened over nP x nP, depth Q.
template <typename Tout> struct UTensorProb {
  const double* U;  // [N][N]
  const double* X;  // [n][N]
  Tout* out;        // layout 0: [NP][nP][nP];  layout 1: [nP][nP][NP] (P fastest)
  int n, Nthc, nP;
  int M, N, K;      // M = NP, N = nP*nP, K = Nthc
  int layout;
  int NPld;         // P extent of layout 1
  __device__ f64x4 loadA4(int, int P, int Q) const {
    if (P >= Nthc) return zero4<double>();
    return load4_strided<double>(U + (long)P * Nthc, 1, Q, Nthc);
  }
  __device__ f64x4 loadB4(int, int j, int Q) const {
    const int q = j / nP, s = j - (j / nP) * nP;
    if (q >= n || s >= n) return zero4<double>();
    f64x4 a = load4_strided<double>(X + (long)q * Nthc, 1, Q, Nthc);
    f64x4 b = load4_strided<double>(X + (long)s * Nthc, 1, Q, Nthc);
    return a * b;
  }
  __device__ void store(int, int P, int j, double v) const {
    if (layout == 0) out[(long)P * nP * nP + j] = Tout(v);
    else out[(long)j * NPld + P] = Tout(v);
  }
};

// ---------------------------------------------------------------------------
// Half projections onto the THC grid (float64 MFMA, stored in Tout):
//   P1[t][R][q]  = sum_u X[u][R] G[tau][u][q]        (the paper's G_Rq)
//   P2T[t][P][w] = sum_p X[p][P] G[tau][w][p]        (G_wP, transposed)
template <typename Tout> struct ProjP1Prob {
  const double* X;  // [n][N]
  const double* G;  // [n_tau][n][n]
  Tout* out;        // [slab][NP][nP]
  int n, Nthc, nP, NP, t0;
  int M, N, K;      // M = NP, N = nP, K = n
  __device__ f64x4 loadA4(int, int R, int u) const {
    if (R >= Nthc) return zero4<double>();
    return load4_strided<double>(X + R, Nthc, u, n);
  }
  __device__ f64x4 loadB4(int b, int q, int u) const {
    if (q >= n) return zero4<double>();
    return load4_strided<double>(G + (long)(t0 + b) * n * n + q, n, u, n);
  }
  __device__ void store(int b, int R, int q, double v) const {
    out[(long)b * NP * nP + (long)R * nP + q] = Tout(v);
  }
};

template <typename Tout> struct ProjP2TProb {
  const double* X;
  const double* G;
  Tout* out;        // [slab][NP][nP]
  int n, Nthc, nP, NP, t0;
  int M, N, K;      // M = NP, N = nP, K = n
  __device__ f64x4 loadA4(int, int P, int p) const {
    if (P >= Nthc) return zero4<double>();
    return load4_strided<double>(X + P, Nthc, p, n);
  }
  __device__ f64x4 loadB4(int b, int w, int p) const {
    if (w >= n) return zero4<double>();
    return load4_strided<double>(G + (long)(t0 + b) * n * n + (long)w * n, 1, p, n);
  }
  __device__ void store(int b, int P, int w, double v) const {
    out[(long)b * NP * nP + (long)P * nP + w] = Tout(v);
  }
};

// ---------------------------------------------------------------------------
// A step:  A[t][v][P][q] = sum_s U1t[P][q][s] G_sv(beta - tau)
// GEMM rows v, columns (P, q) flattened over NP x nP, depth s; G(beta-tau)
// is node n_tau - 1 - tau.  Runs in the contraction precision T.
template <typename T> struct AStepProb {
  const double* G;  // [n_tau][n][n]
  const T* U1t;     // [NP][nP][nP]
  T* out;           // [slab][n][NP][nP]
  int n, nP, NP, n_tau, t0;
  int M, N, K;      // M = n, N = NP*nP, K = nP
  __device__ vec4_t<T> loadA4(int b, int v, int s) const {
    if (v >= n) return zero4<T>();
    const double* Gb = G + (long)(n_tau - 1 - (t0 + b)) * n * n + v;
    return load4_strided<T>(Gb, n, s, n);
  }
  __device__ vec4_t<T> loadB4(int, int j, int s) const {
    if (j >= N) return zero4<T>();
    return *(const vec4_t<T>*)(U1t + (long)j * nP + s);
  }
  __device__ void store(int b, int v, int j, T val) const {
    out[((long)b * n + v) * ((long)NP * nP) + j] = val;
  }
};

// ---------------------------------------------------------------------------
// Elementwise layout kernels.
//   GbT[b][v][s] = G[n_tau-1-(t0+b)][s][v]  (A step operand, zero padded to nP)
//   XT[R][u]     = X[u][R]                  (zero padded to NP x nP)
//   dst = src converted (float64 -> contraction precision)
template <typename T>
__global__ void gbar_t_kernel(const double* G, T* out, int n, int nP, int n_tau, int t0, int cnt) {
  const long per = (long)nP * nP;
  SOX_FOR_FLAT(idx, per * cnt) {
    const int b = (int)(idx / per);
    const int rem = (int)(idx - (long)b * per);
    const int v = rem / nP, s = rem - (rem / nP) * nP;
    T val = T(0);
    if (v < n && s < n) val = T(G[(long)(n_tau - 1 - (t0 + b)) * n * n + (long)s * n + v]);
    out[idx] = val;
  }
}

template <typename T>
__global__ void xt_kernel(const double* X, T* out, int n, int Nthc, int nP, int NP) {
  SOX_FOR_FLAT(idx, (long)NP * nP) {
    const int R = (int)(idx / nP), u = (int)(idx - (idx / nP) * nP);
    out[idx] = (R < Nthc && u < n) ? T(X[(long)u * Nthc + R]) : T(0);
  }
}

// float32 operands of the U-contraction on the LDS-staged GEMM (zero
// padded so the GEMM runs without masks):
//   KR[(q nP + s)][Q] = X_qQ X_sQ   ([nP*nP][NP], the Khatri-Rao factor)
//   V32[P][Q] = U_PQ                ([NP][NP])
__global__ void kr_kernel(const double* X, float* KR, int n, int Nthc, int nP, int NP) {
  SOX_FOR_FLAT(idx, (long)nP * nP * NP) {
    const long j = idx / NP;
    const int Q = (int)(idx - j * NP);
    const int q = (int)(j / nP), s = (int)(j - (long)q * nP);
    float v = 0.0f;
    if (q < n && s < n && Q < Nthc) v = (float)(X[(long)q * Nthc + Q] * X[(long)s * Nthc + Q]);
    KR[idx] = v;
  }
}

__global__ void pad_cast_kernel(const double* src, float* dst, int rows, int cols, int rows_pad,
                                int cols_pad) {
  SOX_FOR_FLAT(idx, (long)rows_pad * cols_pad) {
    const int r = (int)(idx / cols_pad), c = (int)(idx - (long)r * cols_pad);
    dst[idx] = (r < rows && c < cols) ? (float)src[(long)r * cols + c] : 0.0f;
  }
}

// X zero padded to [n][NP] float64 (the back-transform operand)
__global__ void xpad64_kernel(const double* X, double* XP, int n, int Nthc, int NP) {
  SOX_FOR_FLAT(idx, (long)n * NP) {
    const int u = (int)(idx / NP), R = (int)(idx - (long)u * NP);
    XP[idx] = R < Nthc ? X[(long)u * Nthc + R] : 0.0;
  }
}

__global__ void widen_kernel(const float* src, double* dst, long count) {
  SOX_FOR_FLAT(idx, count) dst[idx] = (double)src[idx];
}

// dst = sum over ns float32 blocks src + s stride (split-K partial products)
__global__ void sum_blocks_kernel(const float* src, float* dst, long count, long stride, int ns) {
  SOX_FOR_FLAT(idx, count) {
    float acc = src[idx];
    for (int s = 1; s < ns; ++s) acc += src[idx + s * stride];
    dst[idx] = acc;
  }
}

// dst = sum over ns float32 blocks src + s stride, formed in float64 (the
// partial D blocks of a split v sum, summed and widened in one pass)
__global__ void widen_sum_kernel(const float* src, double* dst, long count, long stride, int ns) {
  SOX_FOR_FLAT(idx, count) {
    double acc = (double)src[idx];
    for (int s = 1; s < ns; ++s) acc += (double)src[idx + s * stride];
    dst[idx] = acc;
  }
}

// widen_sum_kernel on four consecutive elements per work-item: count and
// stride multiples of 4, src and dst 16- and 32-byte aligned.  The ns blocks
// (at most 8) are all loaded before the float64 sum, taken in block order as
// in widen_sum_kernel, so both give the same bits.
__global__ void widen_sum4_kernel(const float* src, double* dst, long count4, long stride, int ns) {
  SOX_FOR_FLAT(i, count4) {
    f32x4 v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s)
      if (s < ns) v[s] = *(const f32x4*)(src + s * stride + 4 * i);
    f64x4 acc = __builtin_convertvector(v[0], f64x4);
#pragma unroll
    for (int s = 1; s < 8; ++s)
      if (s < ns) acc += __builtin_convertvector(v[s], f64x4);
    *(f64x4*)(dst + 4 * i) = acc;
  }
}

template <typename T>
__global__ void cast_kernel(const double* src, T* dst, long count) {
  SOX_FOR_FLAT(idx, count) dst[idx] = T(src[idx]);
}

// ---------------------------------------------------------------------------
// Dynamic interaction (eq:GG scheme), transforms in float64.
//
// Tf2 [2 n_omega][n_tau]: rows 0..n_omega-1 = Re T_fwd, then Im T_fwd.
// Tb2 [n_tau][2 n_omega]: [Re T_bwd | -Im T_bwd], so that
//   Re sum_m T_bwd[i,m] f_m = sum_k Tb2[i,k] (Re f | Im f)_k.
//
// W(Omega_m) = sum_j T_fwd[m,j] W_tau[j] is stored as the real block matrix
//   W2[m] = [[Re W, -Im W], [Im W, Re W]]   (2 NP x 2 NP)
// so that one real GEMM W2[m] (Re GG; Im GG) gives (Re A; Im A).
template <typename T> struct WOmegaProb {
  const double* Tf2;   // [2 n_omega][n_tau]
  const double* Wtau;  // [n_tau][N][N]
  T* W2;               // [n_omega][2NP][2NP]
  int n_omega, n_tau, Nthc, NP;
  int M, N, K;         // M = 2 n_omega, N = NP*NP, K = n_tau
  T* W2T;              // optional transposed copy (adjoint), may be null
  __device__ f64x4 loadA4(int, int row, int j) const {
    if (row >= M) return zero4<double>();
    return load4_strided<double>(Tf2 + (long)row * n_tau, 1, j, n_tau);
  }
  __device__ f64x4 loadB4(int, int col, int j) const {
    if (col >= N) return zero4<double>();
    const int P = col / NP, Q = col - (col / NP) * NP;
    if (P >= Nthc || Q >= Nthc) return zero4<double>();
    return load4_strided<double>(Wtau + (long)P * Nthc + Q, (long)Nthc * Nthc, j, n_tau);
  }
  __device__ void store(int, int row, int col, double v) const {
    const int c = row / n_omega, m = row - (row / n_omega) * n_omega;
    const int P = col / NP, Q = col - (col / NP) * NP;
    const long ld = 2L * NP;
    T* W = W2 + (long)m * ld * ld;
    if (c == 0) {
      W[(long)P * ld + Q] = T(v);
      W[(long)(NP + P) * ld + NP + Q] = T(v);
    } else {
      W[(long)(NP + P) * ld + Q] = T(v);
      W[(long)P * ld + NP + Q] = T(-v);
    }
    if (W2T) {
      T* Wt = W2T + (long)m * ld * ld;
      if (c == 0) {
        Wt[(long)Q * ld + P] = T(v);
        Wt[(long)(NP + Q) * ld + NP + P] = T(v);
      } else {
        Wt[(long)Q * ld + NP + P] = T(v);
        Wt[(long)(NP + Q) * ld + P] = T(-v);
      }
    }
  }
};

// GG formation fused into the forward transform, for the v-slab [v0, v0+vc):
//   GG2[m][(vl,u)][c NP + Q] = sum_j Tf_c[m,j] G_uQ(tau_j) G_Qv(beta - tau_j)
// with G_uQ(tau_j) = P2T[j][Q][u] and G_Qv(beta - tau_j) = P1[n_tau-1-j][Q][v]
// (eq:GG; the third line read at beta - tau).
template <typename T> struct FTProb {
  const double* Tf2;   // [2 n_omega][n_tau]
  const double* P1;    // [n_tau][NP][nP]  float64
  const double* P2T;   // [n_tau][NP][nP]  float64
  T* GG2;              // [n_omega][vc*n][2NP]
  int n, nP, NP, Nthc, n_omega, n_tau, v0, vc;
  int M, N, K;         // M = 2 n_omega, N = vc*n*NP, K = n_tau
  T* GG2T;             // optional [n_omega][2NP][ldt] copy (adjoint), may be null
  int ldt;
  // qmajor = 1: P1 and P2T hold the transposed copies [n_tau][nP][NP] (Q
  // contiguous), so the lanes of a load instruction, which run over Q, read
  // consecutive addresses
  int qmajor = 0;
  // split precision: GG2 stored as bf16 hi and lo planes (same layout)
  bf16_t* GGhi = nullptr;
  bf16_t* GGlo = nullptr;
  __device__ void put(long o, double v) const {
    if (GGhi) {
      const float x = (float)v;
      const bf16_t h = f32_to_bf16(x);
      GGhi[o] = h;
      GGlo[o] = f32_to_bf16(x - bf16_to_f32(h));
    } else {
      GG2[o] = T(v);
    }
  }
  __device__ f64x4 loadA4(int, int row, int j) const {
    if (row >= M) return zero4<double>();
    return load4_strided<double>(Tf2 + (long)row * n_tau, 1, j, n_tau);
  }
  __device__ f64x4 loadB4(int, int col, int j) const {
    if (col >= N) return zero4<double>();
    const int Q = col % NP;
    const int vu = col / NP;
    const int vl = vu / n, u = vu - (vu / n) * n;
    const int v = v0 + vl;
    if (Q >= Nthc || v >= n) return zero4<double>();
    const long st = (long)NP * nP;
    f64x4 r;
    if (qmajor) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int jj = j + m;
        r[m] = (jj < n_tau) ? P2T[jj * st + (long)u * NP + Q] *
                                  P1[(long)(n_tau - 1 - jj) * st + (long)v * NP + Q]
                            : 0.0;
      }
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int jj = j + m;
        r[m] = (jj < n_tau) ? P2T[jj * st + (long)Q * nP + u] *
                                  P1[(long)(n_tau - 1 - jj) * st + (long)Q * nP + v]
                            : 0.0;
      }
    }
    return r;
  }
  __device__ void store(int, int row, int col, double v) const {
    const int c = row / n_omega, m = row - (row / n_omega) * n_omega;
    const int Q = col % NP, vu = col / NP;
    put(((long)m * vc * n + vu) * (2L * NP) + (long)c * NP + Q, v);
    if (GG2T) GG2T[((long)m * 2 * NP + (long)c * NP + Q) * ldt + vu] = T(v);
  }
};

// Forward transform with the transform matrix held stationary (the
// qmajor layout; the adjoint's transposed copy GG2T too when set): the rows of Tf2 (2 n_omega <= 80) over
// K = n_tau <= kFtKmax nodes (zero padded to a multiple of 16) sit in LDS
// for the whole launch.  A wavefront owns all rows of kFtJB column blocks
// that share u and the 16 THC points Q = 16 qb + lane % 16 and differ in v,
// so each G_uQ(tau_j) value is loaded once for the kFtJB blocks; groups run
// with v fastest, then qb, then u, so the wavefronts resident at one time
// reuse the same G_uQ and G_Qv rows from the cache.  The GG column values
// are formed in registers (two float64 loads and a product), float64 MFMA
// and accumulation, 16 k per chunk, the next chunk's loads in flight.
constexpr int kFtKmax = 128;
constexpr int kFtJB = 1;

template <typename T>
__global__ __launch_bounds__(512) void ft_kernel(const FTProb<T> q, long ngroups) {
  __shared__ double tf[80][kFtKmax + 2];
  const int K = q.n_tau, Kp = (K + 15) & ~15;
  for (int e = threadIdx.x; e < 80 * Kp; e += blockDim.x) {
    const int r = e / Kp, k = e - (e / Kp) * Kp;
    tf[r][k] = (r < q.M && k < K) ? q.Tf2[(long)r * K + k] : 0.0;
  }
  __syncthreads();
  constexpr int JB = kFtJB;
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int wave = threadIdx.x >> 6;
  const int nqb = q.NP / 16;
  const int nvp = (q.vc + JB - 1) / JB;
  const long st = (long)q.NP * q.nP;
  const int nch = Kp / 16;
  const int nwaves = blockDim.x >> 6;
  for (long grp = (long)blockIdx.x * nwaves + wave; grp < ngroups;
       grp += (long)gridDim.x * nwaves) {
    const int vp = (int)(grp % nvp);
    const long rest = grp / nvp;
    const int qb = (int)(rest % nqb);
    const int u = (int)(rest / nqb);
    const int Q = 16 * qb + li;
    const bool qok = Q < q.Nthc;
    int vl[JB];
    bool vok[JB];
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      vl[j] = JB * vp + j;
      vok[j] = qok && vl[j] < q.vc && q.v0 + vl[j] < q.n;
    }
    // G_uQ(tau_k) and G_Qv(beta - tau_k) of chunk ch (zero past K or outside)
    auto load = [&](int ch, double* gu, double (*gv)[4]) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k = 16 * ch + 4 * g + m;
        const bool kok = ch < nch && k < K;
        gu[m] = (qok && kok) ? q.P2T[k * st + (long)u * q.NP + Q] : 0.0;
#pragma unroll
        for (int j = 0; j < JB; ++j)
          gv[j][m] = (vok[j] && kok)
                         ? q.P1[(long)(K - 1 - k) * st + (long)(q.v0 + vl[j]) * q.NP + Q]
                         : 0.0;
      }
    };
    f64x4 acc[5][JB];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
      for (int j = 0; j < JB; ++j) acc[i][j] = zero4<double>();
    double u0[4], u1[4], w0[JB][4], w1[JB][4];
    load(0, u0, w0);
    for (int ch = 0; ch < nch; ++ch) {
      load(ch + 1, u1, w1);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        double a[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) a[i] = tf[16 * i + li][16 * ch + 4 * g + m];
#pragma unroll
        for (int j = 0; j < JB; ++j) {
          const double b = u0[m] * w0[j][m];
#pragma unroll
          for (int i = 0; i < 5; ++i) acc[i][j] = mfma16x16x4(a[i], b, acc[i][j]);
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        u0[m] = u1[m];
#pragma unroll
        for (int j = 0; j < JB; ++j) w0[j][m] = w1[j][m];
      }
    }
    // GG2[m][vl n + u][c NP + Q], rows r = c n_omega + m (padded Q stored as 0)
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      if (vl[j] >= q.vc) continue;
      const long vu = (long)vl[j] * q.n + u;
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * i + acc_row<double>(g, r);
          if (row >= q.M) continue;
          const int c = row / q.n_omega, mm = row - (row / q.n_omega) * q.n_omega;
          q.put(((long)mm * q.vc * q.n + vu) * (2L * q.NP) + (long)c * q.NP + Q, acc[i][j][r]);
          if (q.GG2T)
            q.GG2T[((long)mm * 2 * q.NP + (long)c * q.NP + Q) * q.ldt + vu] = T(acc[i][j][r]);
        }
    }
  }
}

// The forward transform: the stationary kernel above for the qmajor layout
// when 2 n_omega <= 80 and n_tau <= kFtKmax, else the generic product with
// 80-row tiles.
template <typename T>
inline hipError_t launch_ft(const FTProb<T>& q, int n_cu, hipStream_t s) {
  if (q.qmajor && q.M <= 80 && q.n_tau <= kFtKmax && q.NP % 16 == 0) {
    const long ngroups = (long)q.n * (q.NP / 16) * ((q.vc + kFtJB - 1) / kFtJB);
    long nwg = (ngroups + 7) / 8;
    if (nwg > 4L * n_cu) nwg = 4L * n_cu;
    if (nwg < 1) return hipSuccess;
    hipLaunchKernelGGL(ft_kernel<T>, dim3((unsigned)nwg), dim3(512), 0, s, q, ngroups);
    return hipGetLastError();
  }
  return launch_gemm<FTProb<T>, double, 1, 4, 5, 1>(q, 1, s);
}

// Inverse transform into the fused kernel's A layout for the v-slab:
//   Adyn[tau][vl][P][u] = sum_k Tb2[tau][k] AW[m][c NP + P][vl n + u],  k = c n_omega + m
// (u >= n is padding and written as zero).
template <typename T> struct IFTProb {
  const double* Tb2;   // [n_tau][2 n_omega]
  const T* AW;         // [n_omega][2NP][vc*n]
  T* Adyn;             // [n_tau][vc][NP][nP]
  int n, nP, NP, n_omega, n_tau, vc;
  int M, N, K;         // M = n_tau, N = NP*vc*nP, K = 2 n_omega
  // split precision: A(tau) stored as bf16 hi and lo planes (same layout)
  // instead of Adyn
  bf16_t* Ahi = nullptr;
  bf16_t* Alo = nullptr;
  __device__ f64x4 loadA4(int, int t, int k) const {
    if (t >= M) return zero4<double>();
    return load4_strided<double>(Tb2 + (long)t * 2 * n_omega, 1, k, 2 * n_omega);
  }
  __device__ f64x4 loadB4(int, int col, int k) const {
    if (col >= N) return zero4<double>();
    const int u = col % nP;
    const int pv = col / nP;
    const int vl = pv % vc, P = pv / vc;
    if (u >= n) return zero4<double>();
    const long vcn = (long)vc * n;
    f64x4 r;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int kk = k + m;
      if (kk < 2 * n_omega) {
        const int c = kk / n_omega, mm = kk - (kk / n_omega) * n_omega;
        r[m] = double(AW[((long)mm * 2 * NP + (long)c * NP + P) * vcn + (long)vl * n + u]);
      } else {
        r[m] = 0.0;
      }
    }
    return r;
  }
  __device__ void store(int, int t, int col, double v) const {
    const int u = col % nP;
    const int pv = col / nP;
    const int vl = pv % vc, P = pv / vc;
    const long o = (((long)t * vc + vl) * NP + P) * nP + u;
    if (Ahi) {
      const float x = (float)v;
      const bf16_t h = f32_to_bf16(x);
      Ahi[o] = h;
      Alo[o] = f32_to_bf16(x - bf16_to_f32(h));
    } else {
      Adyn[o] = T(v);
    }
  }
};

// Inverse transform with the transform matrix held stationary: the rows
// tau < 128 of Tb2 (K = 2 n_omega <= kIftKmax, zero padded to a multiple of
// 16) sit in LDS for the whole launch.  Wavefront w of a workgroup takes the
// 64-row slab w % 2 and walks column groups (32 output columns: two blocks
// of 16 consecutive u of one (P, v)) together with the other slab's
// wavefront, so each AW value is fetched from memory once.  float64 MFMA
// and accumulation as in the generic product, 16 k per chunk (lane g takes
// k = 16 s + 4 g + m in step m of both operands); the AW values of the next
// two chunks are in flight while a chunk's MFMAs run.
constexpr int kIftKmax = 96;
constexpr int kIftJB = 2;  // 16-column blocks per wavefront

template <typename T>
__global__ __launch_bounds__(512) void ift_kernel(const IFTProb<T> q, long ngroups) {
  __shared__ double tb[128][kIftKmax + 2];
  const int K = q.K, Kp = (K + 15) & ~15;
  for (int e = threadIdx.x; e < 128 * Kp; e += blockDim.x) {
    const int r = e / Kp, k = e - (e / Kp) * Kp;
    tb[r][k] = (r < q.M && k < K) ? q.Tb2[(long)r * K + k] : 0.0;
  }
  __syncthreads();
  constexpr int JB = kIftJB;
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int wave = threadIdx.x >> 6;
  const int r0 = 64 * (wave & 1);
  const int nP16 = q.nP / 16;
  const long nblk = (long)q.NP * q.vc * nP16;
  const long vcn = (long)q.vc * q.n;
  const int nch = Kp / 16;
  for (long grp = (long)blockIdx.x * 4 + (wave >> 1); grp < ngroups; grp += (long)gridDim.x * 4) {
    // the lane's column in block j: u = 16 ub + li of (P, vl)
    const T* src[JB];
    int ok[JB], vlj[JB], Pj[JB], uj[JB];
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      const long blk = grp * JB + j;
      const int ub = (int)(blk % nP16);
      const long pv = blk / nP16;
      vlj[j] = (int)(pv % q.vc);
      Pj[j] = (int)(pv / q.vc);
      uj[j] = 16 * ub + li;
      ok[j] = blk < nblk && uj[j] < q.n;
      src[j] = q.AW + (ok[j] ? (long)Pj[j] * vcn + (long)vlj[j] * q.n + uj[j] : 0);
    }
    auto load_b = [&](int ch, T (*b)[4]) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k = 16 * ch + 4 * g + m;
        const int c = k / q.n_omega, mm = k - (k / q.n_omega) * q.n_omega;
        const long koff = ((long)mm * 2 * q.NP + (long)c * q.NP) * vcn;
#pragma unroll
        for (int j = 0; j < JB; ++j)
          b[j][m] = (ok[j] && k < K && ch < nch) ? src[j][koff] : T(0);
      }
    };
    f64x4 acc[4][JB];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < JB; ++j) acc[i][j] = zero4<double>();
    T b0[JB][4], b1[JB][4], b2[JB][4];
    load_b(0, b0);
    load_b(1, b1);
    for (int ch = 0; ch < nch; ++ch) {
      load_b(ch + 2, b2);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        double a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = tb[r0 + 16 * i + li][16 * ch + 4 * g + m];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < JB; ++j) acc[i][j] = mfma16x16x4(a[i], double(b0[j][m]), acc[i][j]);
      }
#pragma unroll
      for (int j = 0; j < JB; ++j)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          b0[j][m] = b1[j][m];
          b1[j][m] = b2[j][m];
        }
    }
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      if (grp * JB + j >= nblk) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int t = r0 + 16 * i + acc_row<double>(g, r);
          if (t >= q.M) continue;
          const long o = (((long)t * q.vc + vlj[j]) * q.NP + Pj[j]) * q.nP + uj[j];
          const double v = acc[i][j][r];
          if (q.Ahi) {
            const float x = (float)v;
            const bf16_t h = f32_to_bf16(x);
            q.Ahi[o] = h;
            q.Alo[o] = f32_to_bf16(x - bf16_to_f32(h));
          } else {
            q.Adyn[o] = T(v);
          }
        }
    }
  }
}

// The inverse transform: the stationary kernel above when n_tau <= 128 and
// 2 n_omega <= kIftKmax, else the generic product.
template <typename T>
inline hipError_t launch_ift(const IFTProb<T>& q, int n_cu, hipStream_t s) {
  if (q.M <= 128 && q.K <= kIftKmax && q.nP % 16 == 0) {
    const long nblk = (long)q.NP * q.vc * (q.nP / 16);
    const long ngroups = (nblk + kIftJB - 1) / kIftJB;
    long nwg = (ngroups + 3) / 4;
    if (nwg > 4L * n_cu) nwg = 4L * n_cu;
    if (nwg < 1) return hipSuccess;
    hipLaunchKernelGGL(ift_kernel<T>, dim3((unsigned)nwg), dim3(512), 0, s, q, ngroups);
    return hipGetLastError();
  }
  return launch_gemm<IFTProb<T>, double, 2, 2, 2, 2>(q, 1, s);
}

// ---------------------------------------------------------------------------
// G(tau) synthesis (eq:G_def, one-body Hamiltonian), float64:
//   occ[k][a] = n(eps_a, tau_k);  G[k][p][q] = -sum_a Q[p][a] occ[k][a] Q[q][a]
__global__ void occupation_kernel(const double* eps, const double* tau, double mu, double beta,
                                  int n, int n_tau, double* occ) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n_tau) return;
  const int k = idx / n, a = idx - (idx / n) * n;
  const double x = eps[a] - mu;
  const double t = tau[k];
  double v;
  if (x >= 0.0) v = exp(-x * t) / (1.0 + exp(-beta * x));
  else v = exp((beta - t) * x) / (1.0 + exp(beta * x));
  occ[idx] = v;
}

struct GBuildProb {
  const double* Q;    // [n][n]
  const double* occ;  // [n_tau][n]
  double* G;          // [n_tau][n][n]
  int n;
  int M, N, K;        // n, n, n
  __device__ f64x4 loadA4(int b, int p, int a) const {
    if (p >= n) return zero4<double>();
    f64x4 q = load4_strided<double>(Q + (long)p * n, 1, a, n);
    f64x4 o = load4_strided<double>(occ + (long)b * n, 1, a, n);
    return q * o;
  }
  __device__ f64x4 loadB4(int, int qq, int a) const {
    if (qq >= n) return zero4<double>();
    return load4_strided<double>(Q + (long)qq * n, 1, a, n);
  }
  __device__ void store(int b, int p, int qq, double v) const { G[((long)b * n + p) * n + qq] = -v; }
};

// ---------------------------------------------------------------------------
// Galitskii-Migdal energy (eq:E2b in imaginary time), float64:
//   tr[k] = sum_tr Sigma[k][t][r] G[n_tau-1-k][r][t]; E = -1/2 sum_k w_k tr[k]
__global__ __launch_bounds__(256) void energy_trace_kernel(const double* Sigma, const double* G,
                                                           int n, int n_tau, double* tr) {
  const int k = blockIdx.x;
  const double* S = Sigma + (long)k * n * n;
  const double* Gb = G + (long)(n_tau - 1 - k) * n * n;
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int t = idx / n, r = idx - (idx / n) * n;
    acc += S[idx] * Gb[(long)r * n + t];
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) tr[k] = red[0];
}

__global__ __launch_bounds__(256) void energy_reduce_kernel(const double* tr, const double* w,
                                                            int n_tau, double* E) {
  double acc = 0.0;
  for (int k = threadIdx.x; k < n_tau; k += blockDim.x) acc += w[k] * tr[k];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) E[0] = -0.5 * red[0];
}

}  // namespace sox
