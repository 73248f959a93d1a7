// Complex kernels of the k-point (periodic solid) SOX path.
//
// Storage is interleaved complex (re, im) in the compute type T.  Every
// complex contraction of the chain is one batched NT product
//
//   C[z][i][j] (+)= alpha * sum_k opA(A[z])[i][k] * opB(B[z])[j][k]
//
// run on the real 16x16x4 MFMA: each complex product is four real products
// into a real and an imaginary accumulator (re += ar br - ai bi,
// im += ar bi + ai br).  opA / opB optionally conjugate; opB optionally
// multiplies element k by a per-batch vector S[k] (or conj S[k]), which fuses
// the Khatri-Rao factor of the U-contraction into the load.
//
// Batch z = zo * nzi + zi; every operand offset (in complex elements) is
// (idx ? idx[zo] : zo) * so + zi * si, so momentum-indexed gathers (k_v - q1,
// k_w, q) come from small device tables.  Row r of A or B sits at
// (r / split) * hi + (r % split) * ld, which lets one kernel read the
// U-tensor [a][P][b] as rows (P, a).
//
// K runs in 16-deep chunks (lane group g holds k = 4g + m, m = 0..3, four
// consecutive complex values) with the next chunk's loads issued ahead of
// the current chunk's MFMAs; a K tail below 16 runs in 4-deep steps (lane
// group g holds k = 4m + g).  Rows past M or N read the last valid row and
// are zeroed; k past K is zeroed; nothing is read out of range.
#pragma once

#include "sox_common.hpp"

namespace sox {

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct vec2;
template <> struct vec2<float> { typedef f32x2 type; };
template <> struct vec2<double> { typedef f64x2 type; };
template <typename T> using vec2_t = typename vec2<T>::type;

template <typename T, typename TC> struct CgArgs {
  const T* A;
  const T* B;
  const T* S;  // optional per-k factor of opB
  TC* C;
  const int* idxA;
  const int* idxB;
  const int* idxS;
  const int* idxC;
  long soA, soB, soS, soC;
  long siA, siB, siS, siC;
  int nzi, nz;
  int splitA, splitB;
  long ldA, hiA, ldB, hiB, ldc;
  int M, N, K;
  int tiles_m, tiles_n;
  T alpha;
  int conjA, conjB, conjS;
  int accumulate;
};

template <typename T>
__device__ __forceinline__ long cg_off(const int* idx, long so, long si, int zo, int zi) {
  return (long)(idx ? idx[zo] : zo) * so + (long)zi * si;
}

template <typename T, typename TC, int WGR, int WGC, int RB, int CB>
__global__ __launch_bounds__(256) void cgemm_nt_kernel(const CgArgs<T, TC> p) {
  static_assert(WGR * WGC == 4, "four wavefronts per workgroup");
  using V2 = vec2_t<T>;
  using V4 = vec4_t<T>;
  const int z = blockIdx.y + blockIdx.z * gridDim.y;
  if (z >= p.nz) return;
  const int zo = z / p.nzi;
  const int zi = z - zo * p.nzi;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int tn = bid % p.tiles_n;
  const int tm = bid / p.tiles_n;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15;
  const int g = lane >> 4;
  const int row0 = tm * (WGR * RB * 16) + (wave / WGC) * (RB * 16);
  const int col0 = tn * (WGC * CB * 16) + (wave % WGC) * (CB * 16);

  const V2* Ab = (const V2*)p.A + cg_off<T>(p.idxA, p.soA, p.siA, zo, zi);
  const V2* Bb = (const V2*)p.B + cg_off<T>(p.idxB, p.soB, p.siB, zo, zi);
  const V2* Sb = p.S ? (const V2*)p.S + cg_off<T>(p.idxS, p.soS, p.siS, zo, zi) : nullptr;
  const V2* arow[RB];
  const V2* brow[CB];
  bool aok[RB], bok[CB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int r0 = row0 + 16 * i + li;
    aok[i] = r0 < p.M;
    const int r = aok[i] ? r0 : p.M - 1;
    arow[i] = Ab + (long)(r / p.splitA) * p.hiA + (long)(r % p.splitA) * p.ldA;
  }
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int c0 = col0 + 16 * j + li;
    bok[j] = c0 < p.N;
    const int c = bok[j] ? c0 : p.N - 1;
    brow[j] = Bb + (long)(c / p.splitB) * p.hiB + (long)(c % p.splitB) * p.ldB;
  }
  const T sa = p.conjA ? T(-1) : T(1);
  const T sb = p.conjB ? T(-1) : T(1);
  const T ss = p.conjS ? T(-1) : T(1);

  V4 accr[RB][CB], acci[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      accr[i][j] = zero4<T>();
      acci[i][j] = zero4<T>();
    }

  // operand registers of the current chunk: A as (re, im), B as (re, im, -im)
  T ar[RB][4], ai[RB][4], br[CB][4], bi[CB][4], nbi[CB][4];
  V2 ra[RB][4], rb[CB][4], rs[4];

  auto prep = [&](const V2 (&xa)[RB][4], const V2 (&xb)[CB][4], const V2 (&xs)[4]) {
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        ar[i][m] = aok[i] ? xa[i][m].x : T(0);
        ai[i][m] = aok[i] ? sa * xa[i][m].y : T(0);
      }
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        T re = bok[j] ? xb[j][m].x : T(0);
        T im = bok[j] ? sb * xb[j][m].y : T(0);
        if (Sb) {
          const T sr = xs[m].x, si = ss * xs[m].y;
          const T r2 = re * sr - im * si;
          im = re * si + im * sr;
          re = r2;
        }
        br[j][m] = re;
        bi[j][m] = im;
        nbi[j][m] = -im;
      }
  };
  auto mma = [&](int m) {
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        accr[i][j] = mfma16x16x4(ar[i][m], br[j][m], accr[i][j]);
        accr[i][j] = mfma16x16x4(ai[i][m], nbi[j][m], accr[i][j]);
        acci[i][j] = mfma16x16x4(ar[i][m], bi[j][m], acci[i][j]);
        acci[i][j] = mfma16x16x4(ai[i][m], br[j][m], acci[i][j]);
      }
  };

  const int KC = p.K >> 4;
  if (KC > 0) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int i = 0; i < RB; ++i) ra[i][m] = arow[i][4 * g + m];
#pragma unroll
      for (int j = 0; j < CB; ++j) rb[j][m] = brow[j][4 * g + m];
      rs[m] = Sb ? Sb[4 * g + m] : V2{T(0), T(0)};
    }
    prep(ra, rb, rs);
  }
  for (int kc = 0; kc < KC; ++kc) {
    const int kn = (kc + 1 < KC) ? kc + 1 : kc;
    const int ko = kn * 16 + 4 * g;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int i = 0; i < RB; ++i) ra[i][m] = arow[i][ko + m];
#pragma unroll
      for (int j = 0; j < CB; ++j) rb[j][m] = brow[j][ko + m];
      rs[m] = Sb ? Sb[ko + m] : V2{T(0), T(0)};
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < 4; ++m) mma(m);
    __builtin_amdgcn_sched_barrier(0);
    prep(ra, rb, rs);
  }
  // K tail: 4-deep steps, lane group g holds k = base + 4m + g
  const int base = KC * 16;
  const int kr = p.K - base;
  for (int m = 0; 4 * m < kr; ++m) {
    const int k = base + 4 * m + g;
    const bool kin = k < p.K;
    const int kk = kin ? k : base;
    V2 xa[RB][4], xb[CB][4], xs[4];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      V2 v = arow[i][kk];
      if (!kin) v = V2{T(0), T(0)};
      xa[i][0] = v;
      xa[i][1] = xa[i][2] = xa[i][3] = v;
    }
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      V2 v = brow[j][kk];
      if (!kin) v = V2{T(0), T(0)};
      xb[j][0] = v;
      xb[j][1] = xb[j][2] = xb[j][3] = v;
    }
    V2 s = Sb ? Sb[kk] : V2{T(0), T(0)};
    xs[0] = xs[1] = xs[2] = xs[3] = s;
    prep(xa, xb, xs);
    mma(0);
  }

  TC* Cb = p.C + 2 * cg_off<T>(p.idxC, p.soC, p.siC, zo, zi);
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + 16 * i + acc_row<T>(g, r);
        const int col = col0 + 16 * j + li;
        if (row < p.M && col < p.N) {
          const long off = 2 * ((long)row * p.ldc + col);
          TC re = TC(p.alpha * accr[i][j][r]);
          TC im = TC(p.alpha * acci[i][j][r]);
          if (p.accumulate) {
            re += Cb[off];
            im += Cb[off + 1];
          }
          Cb[off] = re;
          Cb[off + 1] = im;
        }
      }
}

template <typename T, typename TC> inline CgArgs<T, TC> cg_args() {
  CgArgs<T, TC> a{};
  a.nzi = 1;
  a.splitA = a.splitB = 1 << 30;
  a.alpha = T(1);
  return a;
}

template <typename T, typename TC, int WGR, int WGC, int RB, int CB>
inline hipError_t launch_cgemm(CgArgs<T, TC> a, int nz, hipStream_t s) {
  constexpr int TM = WGR * RB * 16;
  constexpr int TN = WGC * CB * 16;
  if (a.M <= 0 || a.N <= 0 || nz <= 0) return hipSuccess;
  if (a.K < 0 || a.nzi <= 0 || a.splitA <= 0 || a.splitB <= 0) return hipErrorInvalidValue;
  a.nz = nz;
  a.tiles_m = (a.M + TM - 1) / TM;
  a.tiles_n = (a.N + TN - 1) / TN;
  const int gy = nz < 65535 ? nz : 65535;
  const int gz = (nz + gy - 1) / gy;
  dim3 grid(a.tiles_m * a.tiles_n, gy, gz);
  hipLaunchKernelGGL((cgemm_nt_kernel<T, TC, WGR, WGC, RB, CB>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The n_k^3 D step of a solid (section on solids: for every (P, R) pair,
// D^{k_t}_PR accumulates C^{q2,k_w}_RvP B^{q1,k_w-q2}_PRv over k_w, q2 and
// v with q1 = k_w - k_t).  B and C are stored [pair][v][P][R] with pair =
// q * n_k + k; with k_v = k_w - q2 the sum reads, per element e = (P, R),
//
//   D[k_t][e] += scale * sum_{k_v, v} sum_{k_w} C[(k_w - k_v, k_w)][v][e]
//                                              * B[(k_w - k_t, k_v)][v][e].
//
// One thread per element: for each (k_v, v) it loads the n_k values
// B[(., k_v)][v][e] and the n_k values C[(k_w - k_v, k_w)][v][e] once and
// forms all n_k^2 products in registers.  Pairs are sp elements apart, v
// slices NN apart; nv slices are summed.  The mesh is a template parameter so
// that every momentum difference is a compile-time register index.
// D is float64 (the cross-slab accumulation).
template <int M1, int M2, int M3>
__host__ __device__ constexpr int kdiff_of(int a, int b) {
  return ((((a / (M2 * M3)) - (b / (M2 * M3)) + M1) % M1) * M2 +
          (((a / M3) % M2 - (b / M3) % M2 + M2) % M2)) * M3 +
         ((a % M3 - b % M3 + M3) % M3);
}

template <typename T, int M1, int M2, int M3>
__global__ __launch_bounds__(256) void dstep_mesh_kernel(const T* __restrict__ B,
                                                         const T* __restrict__ C, double* D,
                                                         long NN, long sp, int nv, double scale,
                                                         int accumulate) {
  constexpr int NK = M1 * M2 * M3;
  using V2 = vec2_t<T>;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  const V2* Bp = (const V2*)B + e;
  const V2* Cp = (const V2*)C + e;
  double dr[NK], di[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) dr[k] = di[k] = 0.0;
  for (int kv = 0; kv < NK; ++kv) {
    for (int v = 0; v < nv; ++v) {
      const long ov = (long)v * NN;
      V2 b[NK], c[NK];
#pragma unroll
      for (int q1 = 0; q1 < NK; ++q1) b[q1] = Bp[(long)(q1 * NK + kv) * sp + ov];
#pragma unroll
      for (int kw = 0; kw < NK; ++kw) {
        const int q2 = kdiff_of<M1, M2, M3>(kw, kv);
        c[kw] = Cp[(long)(q2 * NK + kw) * sp + ov];
      }
      // n_k-term partial sums in T, accumulated across (k_v, v) in float64
#pragma unroll
      for (int kt = 0; kt < NK; ++kt) {
        T sr = T(0), si = T(0);
#pragma unroll
        for (int kw = 0; kw < NK; ++kw) {
          const int q1 = kdiff_of<M1, M2, M3>(kw, kt);
          sr += c[kw].x * b[q1].x - c[kw].y * b[q1].y;
          si += c[kw].x * b[q1].y + c[kw].y * b[q1].x;
        }
        dr[kt] += (double)sr;
        di[kt] += (double)si;
      }
    }
  }
#pragma unroll
  for (int kt = 0; kt < NK; ++kt) {
    double* o = D + 2 * ((long)kt * NN + e);
    double re = scale * dr[kt], im = scale * di[kt];
    if (accumulate) {
      re += o[0];
      im += o[1];
    }
    o[0] = re;
    o[1] = im;
  }
}

// Any mesh (runtime momentum-difference table kdiff[n_k][n_k]): one thread
// per (element, k_t), operands re-read per k_t.
template <typename T>
__global__ __launch_bounds__(256) void dstep_any_kernel(const T* __restrict__ B,
                                                        const T* __restrict__ C,
                                                        const int* __restrict__ kdiff, double* D,
                                                        long NN, int nk, long sp, int nv,
                                                        double scale, int accumulate) {
  using V2 = vec2_t<T>;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= NN * nk) return;
  const int kt = (int)(idx / NN);
  const long e = idx - (long)kt * NN;
  const V2* Bp = (const V2*)B + e;
  const V2* Cp = (const V2*)C + e;
  double re = 0.0, im = 0.0;
  for (int kw = 0; kw < nk; ++kw) {
    const int q1 = kdiff[kw * nk + kt];
    for (int kv = 0; kv < nk; ++kv) {
      const int q2 = kdiff[kw * nk + kv];
      for (int v = 0; v < nv; ++v) {
        const V2 c = Cp[(long)(q2 * nk + kw) * sp + (long)v * NN];
        const V2 b = Bp[(long)(q1 * nk + kv) * sp + (long)v * NN];
        re += (double)c.x * b.x - (double)c.y * b.y;
        im += (double)c.x * b.y + (double)c.y * b.x;
      }
    }
  }
  double* o = D + 2 * ((long)kt * NN + e);
  re *= scale;
  im *= scale;
  if (accumulate) {
    re += o[0];
    im += o[1];
  }
  o[0] = re;
  o[1] = im;
}

// ---------------------------------------------------------------------------
// Small complex helpers.

// out[b][j][i] = in[b][i][j] (rows x cols per batch), complex, with a type
// conversion; 32 x 32 tiles through LDS.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void ctranspose_kernel(const TI* in, TO* out, int rows, int cols) {
  __shared__ TI tr[32][33], ti[32][33];
  const long b = blockIdx.z;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const TI* ib = in + 2 * b * rows * cols;
  TO* ob = out + 2 * b * rows * cols;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int r = r0 + y, c = c0 + tx;
    if (r < rows && c < cols) {
      tr[y][tx] = ib[2 * ((long)r * cols + c)];
      ti[y][tx] = ib[2 * ((long)r * cols + c) + 1];
    }
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int c = c0 + y, r = r0 + tx;
    if (r < rows && c < cols) {
      ob[2 * ((long)c * rows + r)] = TO(tr[tx][y]);
      ob[2 * ((long)c * rows + r) + 1] = TO(ti[tx][y]);
    }
  }
}

// occ_c[i] = (occ[i], 0): the occupation factors as complex values.
__global__ void real_to_complex_kernel(const double* x, double* out, long count) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    out[2 * i] = x[i];
    out[2 * i + 1] = 0.0;
  }
}

// tr[k][t] = Re sum_{a,b} Sigma^k(tau_t)[a][b] G^k(beta - tau_t)[b][a].
__global__ __launch_bounds__(256) void energy_trace_c_kernel(const double* Sigma, const double* G,
                                                             int n, int n_tau, double* tr) {
  const int t = blockIdx.x, k = blockIdx.y;
  const double* S = Sigma + 2 * ((long)k * n_tau + t) * n * n;
  const double* Gb = G + 2 * ((long)k * n_tau + (n_tau - 1 - t)) * n * n;
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int a = idx / n, b = idx - (idx / n) * n;
    const long j = (long)b * n + a;
    acc += S[2 * idx] * Gb[2 * j] - S[2 * idx + 1] * Gb[2 * j + 1];
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) tr[(long)k * n_tau + t] = red[0];
}

// E = -1/2 (1/n_k) sum_k sum_t w_t tr[k][t]
__global__ __launch_bounds__(256) void energy_reduce_c_kernel(const double* tr, const double* w,
                                                              int n_tau, int nk, double* E) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n_tau * nk; i += blockDim.x) acc += w[i % n_tau] * tr[i];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) E[0] = -0.5 * red[0] / nk;
}

}  // namespace sox
