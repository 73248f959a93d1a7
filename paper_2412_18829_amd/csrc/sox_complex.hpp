// Complex kernels of the k-point (periodic solid) SOX path.
//
// Storage is interleaved complex (re, im) in the compute type T.  Every
// complex contraction of the chain is one batched NT product
//
//   C[z][v][i][j] (+)= alpha * sum_k opA(A[z][v])[i][k] * opB(B[z][v])[j][k]
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
// U-tensor [a][P][b] as rows (P, a); element k of a row is ks elements past
// element k - 1 (ks = 1 for K-contiguous rows, the row count of a K-major
// operand otherwise).  Inside a workgroup, v = 0 .. nv-1
// offsets A, B and C by v * vsA, v * vsB, v * vsC: one operand of the B and
// C steps is the same for every v (vs = 0) and stays in cache, and the
// software pipeline runs on across the v boundary.
//
// K runs in 16-deep chunks: in MFMA step m of a chunk, lane group g holds
// k = 16 kc + 4 m + g, so a final partial chunk costs only ceil(rest / 4)
// steps.  The loads of the next chunk (of this v or the next) are issued
// before the current chunk's MFMAs.  Rows past M or N read the last valid
// row and are zeroed; k past K reads the last valid k and is zeroed; nothing
// is read out of range.
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
  long vsA, vsB, vsC;
  long ksA, ksB;  // k strides of A and B (1: K-contiguous rows)
  int nzi, nz, nv;
  int splitA, splitB;
  int splitC;     // column c of C sits at (c / splitC) * hiC + c % splitC
  long hiC;
  long ldA, hiA, ldB, hiB, ldc;
  int M, N, K;
  int tiles_m, tiles_n;
  T alpha;
  int conjA, conjB, conjS;
  int accumulate;
};

__device__ __forceinline__ long cg_off(const int* idx, long so, long si, int zo, int zi) {
  return (long)(idx ? idx[zo] : zo) * so + (long)zi * si;
}

template <typename T, typename TC, int WGR, int WGC, int RB, int CB>
__global__ __launch_bounds__(64 * WGR * WGC) void cgemm_nt_kernel(const CgArgs<T, TC> p) {
  using V2 = vec2_t<T>;
  using V4 = vec4_t<T>;
  using C2 = vec2_t<TC>;
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

  const V2* Ab = (const V2*)p.A + cg_off(p.idxA, p.soA, p.siA, zo, zi);
  const V2* Bb = (const V2*)p.B + cg_off(p.idxB, p.soB, p.siB, zo, zi);
  const V2* Sb = p.S ? (const V2*)p.S + cg_off(p.idxS, p.soS, p.siS, zo, zi) : nullptr;
  TC* Cb = p.C + 2 * cg_off(p.idxC, p.soC, p.siC, zo, zi);
  long aoff[RB], boff[CB];
  bool aok[RB], bok[CB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int r0 = row0 + 16 * i + li;
    aok[i] = r0 < p.M;
    const int r = aok[i] ? r0 : p.M - 1;
    aoff[i] = (long)(r / p.splitA) * p.hiA + (long)(r % p.splitA) * p.ldA;
  }
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int c0 = col0 + 16 * j + li;
    bok[j] = c0 < p.N;
    const int c = bok[j] ? c0 : p.N - 1;
    boff[j] = (long)(c / p.splitB) * p.hiB + (long)(c % p.splitB) * p.ldB;
  }
  const T sa = p.conjA ? T(-1) : T(1);
  const T sb = p.conjB ? T(-1) : T(1);
  const T ss = p.conjS ? T(-1) : T(1);

  V4 accr[RB][CB], acci[RB][CB];
  auto zero_acc = [&]() {
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        accr[i][j] = zero4<T>();
        acci[i][j] = zero4<T>();
      }
  };
  auto store = [&](int v) {
    TC* Cv = Cb + 2 * (long)v * p.vsC;
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + 16 * i + acc_row<T>(g, r);
          const int col = col0 + 16 * j + li;
          if (row < p.M && col < p.N) {
            const long co = (long)(col / p.splitC) * p.hiC + (col % p.splitC);
            C2* o = (C2*)(Cv + 2 * ((long)row * p.ldc + co));
            C2 val;
            val.x = TC(p.alpha * accr[i][j][r]);
            val.y = TC(p.alpha * acci[i][j][r]);
            if (p.accumulate) val += *o;
            *o = val;
          }
        }
  };
  zero_acc();
  const int KC = (p.K + 15) >> 4;
  if (KC == 0) {
    for (int v = 0; v < p.nv; ++v) store(v);
    return;
  }
  const int T_ = p.nv * KC;

  // operand registers of the current step: (re, im) of both, plus the
  // negated imaginary part of the operand with fewer blocks
  constexpr bool NEG_A = RB <= CB;
  constexpr int NA = NEG_A ? RB : 1, NB = NEG_A ? 1 : CB;
  T ar[RB][4], ai[RB][4], br[CB][4], bi[CB][4], nai[NA][4], nbi[NB][4];
  V2 ra[RB][4], rb[CB][4], rs[4];

  auto load = [&](int t) {
    const int v = t / KC;
    const int kc = t - v * KC;
    const V2* Av = Ab + (long)v * p.vsA;
    const V2* Bv = Bb + (long)v * p.vsB;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      int k = kc * 16 + 4 * m + g;
      k = k < p.K ? k : p.K - 1;
      const long ka = (long)k * p.ksA, kb = (long)k * p.ksB;
#pragma unroll
      for (int i = 0; i < RB; ++i) ra[i][m] = Av[aoff[i] + ka];
#pragma unroll
      for (int j = 0; j < CB; ++j) rb[j][m] = Bv[boff[j] + kb];
      rs[m] = Sb ? Sb[k] : V2{T(0), T(0)};
    }
  };
  auto prep = [&](int t) {
    const int kc = t % KC;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const bool kin = kc * 16 + 4 * m + g < p.K;
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const bool ok = aok[i] && kin;
        ar[i][m] = ok ? ra[i][m].x : T(0);
        ai[i][m] = ok ? sa * ra[i][m].y : T(0);
        if constexpr (NEG_A) nai[i][m] = -ai[i][m];
      }
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const bool ok = bok[j] && kin;
        T re = ok ? rb[j][m].x : T(0);
        T im = ok ? sb * rb[j][m].y : T(0);
        if (Sb) {
          const T sr = rs[m].x, si = ss * rs[m].y;
          const T r2 = re * sr - im * si;
          im = re * si + im * sr;
          re = r2;
        }
        br[j][m] = re;
        bi[j][m] = im;
        if constexpr (!NEG_A) nbi[j][m] = -im;
      }
    }
  };
  auto mma = [&](int m) {
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        accr[i][j] = mfma16x16x4(ar[i][m], br[j][m], accr[i][j]);
        if constexpr (NEG_A) accr[i][j] = mfma16x16x4(nai[i][m], bi[j][m], accr[i][j]);
        else accr[i][j] = mfma16x16x4(ai[i][m], nbi[j][m], accr[i][j]);
        acci[i][j] = mfma16x16x4(ar[i][m], bi[j][m], acci[i][j]);
        acci[i][j] = mfma16x16x4(ai[i][m], br[j][m], acci[i][j]);
      }
  };

  const int last_steps = (p.K - (KC - 1) * 16 + 3) >> 2;  // MFMA steps of the final chunk
  load(0);
  prep(0);
  for (int t = 0; t < T_; ++t) {
    load(t + 1 < T_ ? t + 1 : t);
    __builtin_amdgcn_sched_barrier(0);
    const int kc = t % KC;
    const int steps = kc == KC - 1 ? last_steps : 4;
    mma(0);
    if (steps > 1) mma(1);
    if (steps > 2) mma(2);
    if (steps > 3) mma(3);
    __builtin_amdgcn_sched_barrier(0);
    if (kc == KC - 1) {
      store(t / KC);
      zero_acc();
    }
    prep(t + 1 < T_ ? t + 1 : t);
  }
}

template <typename T, typename TC> inline CgArgs<T, TC> cg_args() {
  CgArgs<T, TC> a{};
  a.nzi = 1;
  a.nv = 1;
  a.ksA = a.ksB = 1;
  a.splitA = a.splitB = a.splitC = 1 << 30;
  a.alpha = T(1);
  return a;
}

template <typename T, typename TC, int WGR, int WGC, int RB, int CB>
inline hipError_t launch_cgemm(CgArgs<T, TC> a, int nz, hipStream_t s) {
  constexpr int TM = WGR * RB * 16;
  constexpr int TN = WGC * CB * 16;
  if (a.M <= 0 || a.N <= 0 || nz <= 0 || a.nv <= 0) return hipSuccess;
  if (a.K < 0 || a.nzi <= 0 || a.splitA <= 0 || a.splitB <= 0 || a.splitC <= 0)
    return hipErrorInvalidValue;
  a.nz = nz;
  a.tiles_m = (a.M + TM - 1) / TM;
  a.tiles_n = (a.N + TN - 1) / TN;
  const int gy = nz < 65535 ? nz : 65535;
  const int gz = (nz + gy - 1) / gy;
  const long gx = (long)a.tiles_m * a.tiles_n;
  if (!grid_fits(gx, 64 * WGR * WGC, gy, gz)) return hipErrorInvalidValue;
  dim3 grid((unsigned)gx, gy, gz);
  hipLaunchKernelGGL((cgemm_nt_kernel<T, TC, WGR, WGC, RB, CB>), grid, dim3(64 * WGR * WGC), 0, s,
                     a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The B and C steps of a solid: the same complex NT product as above, for
// nv orbitals v per workgroup, where one operand does not depend on v (the
// G_Rq panel of the B step, the G_wP^T panel of the C step).  A workgroup
// of NW wavefronts owns an (16 NW) x 80 output tile:
//   FIXA = false (B step): A varies with v; wavefront w owns rows
//     [16 w, 16 w + 16) and keeps them in registers; B (80 rows) is staged
//     once in LDS for every v.
//   FIXA = true (C step): B varies with v; wavefront w owns columns
//     [16 w, 16 w + 16); A (80 rows) is staged once in LDS.
// Four wavefronts let two workgroups share a CU (about 200 registers per
// lane), which keeps all four SIMDs busy; five would divide N = 400 exactly
// but leave one SIMD with twice the work.
// A wavefront's own rows for v + 1 are loaded while the MFMAs of v run
// (one lane holds k = 4 s + g for s < SM, the instantiated step count
// >= ceil(K / 4); steps past K multiply zeros), so the loads have a whole v
// of MFMAs to arrive.  K <= 64, no conjugation, no S factor,
// K-contiguous rows, float32 (the launcher checks and otherwise uses the
// kernel above).  The LDS row stride is K rounded up to 4, then to 4 mod 32
// complex, so the 16 rows a load instruction touches spread over the banks.
constexpr int kPanelRows = 80;
constexpr int kPanelSmax = 16;

__host__ __device__ constexpr int panel_ls(int K) {
  return ((K + 3) & ~3) + ((4 - ((K + 3) & ~3) % 32) + 32) % 32;
}
constexpr int kPanelLSMax = panel_ls(4 * kPanelSmax);  // 68 complex

template <typename T, bool FIXA, int SM, int NW>
__global__ __launch_bounds__(64 * NW) void cgemm_panel_kernel(const CgArgs<T, T> p) {
  static_assert(SM <= kPanelSmax, "panel holds at most 64 k");
  using V2 = vec2_t<T>;
  using V4 = vec4_t<T>;
  __shared__ V2 panel[kPanelRows * kPanelLSMax];
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
  const int row0 = tm * (FIXA ? kPanelRows : 16 * NW);
  const int col0 = tn * (FIXA ? 16 * NW : kPanelRows);
  const int LS = panel_ls(p.K);

  const V2* Ab = (const V2*)p.A + cg_off(p.idxA, p.soA, p.siA, zo, zi);
  const V2* Bb = (const V2*)p.B + cg_off(p.idxB, p.soB, p.siB, zo, zi);
  T* Cb = p.C + 2 * cg_off(p.idxC, p.soC, p.siC, zo, zi);

  // stage the fixed panel: 80 rows x LS complex, zero past K and past M / N
  {
    const V2* F = FIXA ? Ab : Bb;
    const long ldf = FIXA ? p.ldA : p.ldB;
    const int f0 = FIXA ? row0 : col0;
    const int fext = FIXA ? p.M : p.N;
    for (int idx = threadIdx.x; idx < kPanelRows * LS; idx += blockDim.x) {
      const int r = idx / LS, k = idx - (idx / LS) * LS;
      V2 v = V2{T(0), T(0)};
      if (f0 + r < fext && k < p.K) v = F[(long)(f0 + r) * ldf + k];
      panel[idx] = v;
    }
  }
  __syncthreads();

  // this wavefront's varying rows
  const int vr0 = (FIXA ? col0 : row0) + 16 * wave;
  const int vext = FIXA ? p.N : p.M;
  const bool vok = vr0 + li < vext;
  const V2* Vb = (FIXA ? Bb : Ab) + (long)(vok ? vr0 + li : vext - 1) * (FIXA ? p.ldB : p.ldA);
  const long vsv = FIXA ? p.vsB : p.vsA;
  V2 cur[SM], nxt[SM];
  auto load = [&](int v, V2 (&dst)[SM]) {
    const V2* src = Vb + (long)v * vsv;
#pragma unroll
    for (int s = 0; s < SM; ++s) {
      int k = 4 * s + g;
      k = k < p.K ? k : p.K - 1;
      dst[s] = src[k];
    }
  };
  auto mask = [&](V2 (&x)[SM]) {
#pragma unroll
    for (int s = 0; s < SM; ++s) {
      const bool ok = vok && 4 * s + g < p.K;
      x[s].x = ok ? x[s].x : T(0);
      x[s].y = ok ? x[s].y : T(0);
    }
  };

  const V2* P = panel + li * LS + g;  // row 16 b + li, column 4 s + g
  load(0, cur);
  mask(cur);
  for (int v = 0; v < p.nv; ++v) {
    load(v + 1 < p.nv ? v + 1 : v, nxt);
    V4 accr[5], acci[5];
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      accr[b] = zero4<T>();
      acci[b] = zero4<T>();
    }
    // panel operands one step ahead of the MFMAs that use them
    V2 fc[5], fn[5];
#pragma unroll
    for (int b = 0; b < 5; ++b) fc[b] = P[16 * b * LS];
#pragma unroll
    for (int s = 0; s < SM; ++s) {
      {
        if (s + 1 < SM) {
#pragma unroll
          for (int b = 0; b < 5; ++b) fn[b] = P[16 * b * LS + 4 * (s + 1)];
        }
        __builtin_amdgcn_sched_barrier(0);
        const T xr = cur[s].x, xi = cur[s].y, nxi = -cur[s].y;
#pragma unroll
        for (int b = 0; b < 5; ++b) {
          const V2 f = fc[b];
          if (FIXA) {  // A = panel (f), B = own rows (x)
            accr[b] = mfma16x16x4(f.x, xr, accr[b]);
            accr[b] = mfma16x16x4(f.y, nxi, accr[b]);
            acci[b] = mfma16x16x4(f.x, xi, acci[b]);
            acci[b] = mfma16x16x4(f.y, xr, acci[b]);
          } else {     // A = own rows (x), B = panel (f)
            accr[b] = mfma16x16x4(xr, f.x, accr[b]);
            accr[b] = mfma16x16x4(nxi, f.y, accr[b]);
            acci[b] = mfma16x16x4(xr, f.y, acci[b]);
            acci[b] = mfma16x16x4(xi, f.x, acci[b]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < 5; ++b) fc[b] = fn[b];
      }
    }
    T* Cv = Cb + 2 * (long)v * p.vsC;
#pragma unroll
    for (int b = 0; b < 5; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = FIXA ? row0 + 16 * b + acc_row<T>(g, r) : vr0 + acc_row<T>(g, r);
        const int col = FIXA ? vr0 + li : col0 + 16 * b + li;
        if (row < p.M && col < p.N) {
          V2 o;
          o.x = p.alpha * accr[b][r];
          o.y = p.alpha * acci[b][r];
          *(V2*)(Cv + 2 * ((long)row * p.ldc + col)) = o;
        }
      }
#pragma unroll
    for (int s = 0; s < SM; ++s) cur[s] = nxt[s];
    mask(cur);
  }
}

// The panel kernel for the B and C steps when its conditions hold (K <= 64,
// plain rows, no conjugation, no S factor, no accumulation, LDS within the
// per-workgroup limit); returns hipErrorNotSupported otherwise.
inline hipError_t launch_cgemm_panel(CgArgs<float, float> a, int nz, bool fixa, hipStream_t s) {
  if (a.K < 1 || a.K > 4 * kPanelSmax || a.conjA || a.conjB || a.S || a.accumulate ||
      a.splitA != (1 << 30) || a.splitB != (1 << 30) || a.splitC != (1 << 30) || a.ksA != 1 ||
      a.ksB != 1 ||
      (fixa ? a.vsA : a.vsB) != 0)
    return hipErrorNotSupported;
  if (a.M <= 0 || a.N <= 0 || nz <= 0 || a.nv <= 0) return hipSuccess;
  constexpr int NW = 4;
  a.nz = nz;
  a.tiles_m = (a.M + (fixa ? kPanelRows : 16 * NW) - 1) / (fixa ? kPanelRows : 16 * NW);
  a.tiles_n = (a.N + (fixa ? 16 * NW : kPanelRows) - 1) / (fixa ? 16 * NW : kPanelRows);
  const int gy = nz < 65535 ? nz : 65535;
  const int gz = (nz + gy - 1) / gy;
  const long gx = (long)a.tiles_m * a.tiles_n;
  if (!grid_fits(gx, 64 * NW, gy, gz)) return hipErrorInvalidValue;
  dim3 grid((unsigned)gx, gy, gz);
  const int S = (a.K + 3) / 4;
#define SOX_PANEL(SM_)                                                                     \
  if (S <= SM_) {                                                                          \
    if (fixa)                                                                              \
      hipLaunchKernelGGL((cgemm_panel_kernel<float, true, SM_, NW>), grid, dim3(64 * NW), 0, \
                         s, a);                                                            \
    else                                                                                   \
      hipLaunchKernelGGL((cgemm_panel_kernel<float, false, SM_, NW>), grid, dim3(64 * NW),  \
                         0, s, a);                                                         \
    return hipGetLastError();                                                              \
  }
  SOX_PANEL(4)
  SOX_PANEL(8)
  SOX_PANEL(13)
  SOX_PANEL(16)
#undef SOX_PANEL
  return hipErrorNotSupported;
}

// ---------------------------------------------------------------------------
// The same B and C products in split precision: every float32 operand x is
// written as hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest
// even), and each real product is hi*hi + hi*lo + lo*hi on the bf16 MFMA
// (v_mfma_f32_16x16x32_bf16) with float32 accumulation; a complex
// multiply-add is four real products, twelve MFMAs per 32-deep k chunk.
// The fixed panel is split while it is staged into LDS (four bf16 planes:
// hi and lo of the real and imaginary parts), the wavefront's own rows are
// split in registers, so no split copy ever reaches HBM.  Operand layout of
// the bf16 MFMA: lane (li, g) holds row li, k = 32 kc + 8 g + e, e < 8.
// K <= 64 (two chunks).
//
// The products are bound by their stores (N x N outputs per K = n inputs),
// so the kernel keeps the stores flowing: the own rows of the next v are
// copied by the wavefront straight into its LDS region (16-byte
// global_load_lds of the contiguous 16-row block, when the rows are K
// complex apart and K is even; per-lane register loads otherwise) while the
// MFMAs of v run, and the stores of v - 1 are issued between the MFMA steps
// of v instead of in one burst (measured at n_k = 27, N = 400, n = 52 with
// eight nodes per launch: 2.57 -> 2.34 ms; the stores alone take 1.36 ms,
// the MFMAs alone 0.67 ms).
constexpr int kSplitLS = 72;     // bf16 row stride of one LDS plane (K <= 64, padded)
constexpr int kOwnBytes = 8192;  // a wavefront's copy of its 16 own rows (K <= 64 complex)
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8 as_bf16x8(u16x8 x) { return __builtin_bit_cast(bf16x8, x); }

template <bool FIXA, int NW, bool DMA>
__global__ __launch_bounds__(64 * NW) void cgemm_panel_bf16x3_kernel(const CgArgs<float, float> p) {
  using V2 = f32x2;
  __shared__ __align__(16) bf16_t pl[4][kPanelRows * kSplitLS];  // hi re, hi im, lo re, lo im
  __shared__ __align__(16) char own_lds[DMA ? NW : 1][DMA ? kOwnBytes : 16];
  const int z = blockIdx.y + blockIdx.z * gridDim.y;
  if (z >= p.nz) return;
  const int zo = z / p.nzi;
  const int zi = z - zo * p.nzi;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int tn = bid % p.tiles_n;
  const int tm = bid / p.tiles_n;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15;
  const int g = lane >> 4;
  const int row0 = tm * (FIXA ? kPanelRows : 16 * NW);
  const int col0 = tn * (FIXA ? 16 * NW : kPanelRows);
  const int K = p.K;

  const V2* Ab = (const V2*)p.A + cg_off(p.idxA, p.soA, p.siA, zo, zi);
  const V2* Bb = (const V2*)p.B + cg_off(p.idxB, p.soB, p.siB, zo, zi);
  float* Cb = p.C + 2 * cg_off(p.idxC, p.soC, p.siC, zo, zi);

  const int vr0 = (FIXA ? col0 : row0) + 16 * wave;
  const int vext = FIXA ? p.N : p.M;
  const bool vok = vr0 + li < vext;
  const V2* Vb = FIXA ? Bb : Ab;
  const long vld = FIXA ? p.ldB : p.ldA;
  const long vsv = FIXA ? p.vsB : p.vsA;
  // every output of the wavefront in range: twenty unmasked stores per v
  const bool full = vr0 + 16 <= vext && (FIXA ? row0 + kPanelRows <= p.M
                                                : col0 + kPanelRows <= p.N);
  // the LDS copy of v's own rows: 16-byte piece q = 64 i + lane (two complex)
  char* my = own_lds[DMA ? wave : 0];
  auto dma = [&](int v) {
    if constexpr (DMA) {
      const V2* src = Vb + (long)v * vsv;
      const int half = K / 2, npieces = 8 * K;
#pragma unroll
      for (int i = 0; i < kOwnBytes / 1024; ++i) {
        if (64 * i >= npieces) break;
        int q = 64 * i + lane;
        q = q < npieces ? q : npieces - 1;
        const int r = q / half, c = q - r * half;
        const int row = vr0 + r < vext ? vr0 + r : vext - 1;
        global_to_lds16(src + (long)row * vld + 2 * c, my + 1024 * i);
      }
    }
  };
  if (DMA) dma(0);

  {
    const V2* F = FIXA ? Ab : Bb;
    const long ldf = FIXA ? p.ldA : p.ldB;
    const int f0 = FIXA ? row0 : col0;
    const int fext = FIXA ? p.M : p.N;
    for (int idx = threadIdx.x; idx < kPanelRows * 64; idx += blockDim.x) {
      const int r = idx >> 6, k = idx & 63;
      V2 v = V2{0.f, 0.f};
      if (f0 + r < fext && k < K) v = F[(long)(f0 + r) * ldf + k];
      const bf16_t hr = f32_to_bf16(v.x), hi = f32_to_bf16(v.y);
      const int o = r * kSplitLS + k;
      pl[0][o] = hr;
      pl[1][o] = hi;
      pl[2][o] = f32_to_bf16(v.x - bf16_to_f32(hr));
      pl[3][o] = f32_to_bf16(v.y - bf16_to_f32(hi));
    }
  }
  __syncthreads();

  const V2* Vrow = Vb + (long)(vok ? vr0 + li : vext - 1) * vld;
  V2 raw[16];  // own row, k = 32 kc + 8 g + e at raw[8 kc + e]
  auto load = [&](int v) {  // per-lane register loads (rows not contiguous)
    const V2* src = Vrow + (long)v * vsv;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      int k = 32 * (j >> 3) + 8 * g + (j & 7);
      k = k < K ? k : K - 1;
      raw[j] = src[k];
    }
  };
  auto fetch = [&]() {  // the lane's row from the LDS copy (k past K is masked in split)
    const char* b = my + li * 8 * K;
#pragma unroll
    for (int kc = 0; kc < 2; ++kc)
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const f32x4 q = *(const f32x4*)(b + 8 * (32 * kc + 8 * g + 2 * h));
        raw[8 * kc + 2 * h] = V2{q[0], q[1]};
        raw[8 * kc + 2 * h + 1] = V2{q[2], q[3]};
      }
  };
  // own operand planes: [kc][hi re, hi im, lo re, lo im, -hi im, -lo im]
  bf16x8 own[2][6];
  auto split = [&]() {
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      u16x8 hr, hm, lr, lm, nhm, nlm;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool ok = vok && 32 * kc + 8 * g + e < K;
        const float xr = ok ? raw[8 * kc + e].x : 0.f, xi = ok ? raw[8 * kc + e].y : 0.f;
        const bf16_t a = f32_to_bf16(xr), b = f32_to_bf16(xi);
        const bf16_t c = f32_to_bf16(xr - bf16_to_f32(a)), d = f32_to_bf16(xi - bf16_to_f32(b));
        hr[e] = a; hm[e] = b; lr[e] = c; lm[e] = d;
        nhm[e] = (bf16_t)(b ^ 0x8000u);
        nlm[e] = (bf16_t)(d ^ 0x8000u);
      }
      own[kc][0] = as_bf16x8(hr); own[kc][1] = as_bf16x8(hm);
      own[kc][2] = as_bf16x8(lr); own[kc][3] = as_bf16x8(lm);
      own[kc][4] = as_bf16x8(nhm); own[kc][5] = as_bf16x8(nlm);
    }
  };
  // x * y in split precision: xh yh + xh yl + xl yh
  auto prod3 = [](bf16x8 xh, bf16x8 xl, bf16x8 yh, bf16x8 yl, f32x4 acc) {
    acc = mfma16x16x32bf16(xh, yh, acc);
    acc = mfma16x16x32bf16(xh, yl, acc);
    acc = mfma16x16x32bf16(xl, yh, acc);
    return acc;
  };
  // column (row) block b of v's products
  auto store = [&](int v, int b, const f32x4& xr, const f32x4& xi) {
    float* Cv = Cb + 2 * (long)v * p.vsC;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = FIXA ? row0 + 16 * b + acc_row<float>(g, r) : vr0 + acc_row<float>(g, r);
      const int col = FIXA ? vr0 + li : col0 + 16 * b + li;
      if (full || (row < p.M && col < p.N)) {
        V2 o;
        o.x = p.alpha * xr[r];
        o.y = p.alpha * xi[r];
        *(V2*)(Cv + 2 * ((long)row * p.ldc + col)) = o;
      }
    }
  };
  // with the LDS copies, the previous v's products are stored one block at a
  // time between the MFMA steps of v (the register-load path keeps one burst
  // per v: the extra accumulators would halve its occupancy)
  f32x4 pr[DMA ? 5 : 1], pi[DMA ? 5 : 1];

  if (!DMA) {
    load(0);
    split();
  }
  for (int v = 0; v < p.nv; ++v) {
    if (DMA) {
      // v's copy has landed: every vector memory operation of the wavefront
      // has completed (the stores of v - 2 were issued after the copy, and
      // loads and stores do not complete in issue order, so a count that
      // leaves those stores in flight does not cover the copy)
      wait_vm<0>();
      asm volatile("" ::: "memory");
      fetch();
      split();
      asm volatile("" ::: "memory");  // the reads are done before the next copy
      if (v + 1 < p.nv) dma(v + 1);
    } else {
      load(v + 1 < p.nv ? v + 1 : v);
    }
    f32x4 accr[5], acci[5];
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      accr[b] = zero4<float>();
      acci[b] = zero4<float>();
    }
    // the four panel planes of step (kc, b), read one step ahead of its MFMAs
    auto rd = [&](int kc, int b, u16x8 (&q)[4]) {
      const int o = (16 * b + li) * kSplitLS + 32 * kc + 8 * g;
#pragma unroll
      for (int c = 0; c < 4; ++c) q[c] = *(const u16x8*)&pl[c][o];
    };
    u16x8 qc[4], qn[4];
    rd(0, 0, qc);
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
#pragma unroll
      for (int b = 0; b < 5; ++b) {
        const int st = 5 * kc + b;
        if (st + 1 < 10) rd((st + 1) / 5, (st + 1) % 5, qn);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (DMA)
          if (v > 0 && (st & 1) == 0) store(v - 1, st >> 1, pr[st >> 1], pi[st >> 1]);
        const bf16x8 phr = as_bf16x8(qc[0]);
        const bf16x8 phm = as_bf16x8(qc[1]);
        const bf16x8 plr = as_bf16x8(qc[2]);
        const bf16x8 plm = as_bf16x8(qc[3]);
        const bf16x8* w = own[kc];
        if (FIXA) {  // A = panel, B = own: re += Ar Br + Ai (-Bi); im += Ar Bi + Ai Br
          accr[b] = prod3(phr, plr, w[0], w[2], accr[b]);
          accr[b] = prod3(phm, plm, w[4], w[5], accr[b]);
          acci[b] = prod3(phr, plr, w[1], w[3], acci[b]);
          acci[b] = prod3(phm, plm, w[0], w[2], acci[b]);
        } else {     // A = own, B = panel: re += Ar Br + (-Ai) Bi; im += Ar Bi + Ai Br
          accr[b] = prod3(w[0], w[2], phr, plr, accr[b]);
          accr[b] = prod3(w[4], w[5], phm, plm, accr[b]);
          acci[b] = prod3(w[0], w[2], phm, plm, acci[b]);
          acci[b] = prod3(w[1], w[3], phr, plr, acci[b]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < 4; ++c) qc[c] = qn[c];
      }
    }
    if constexpr (DMA) {
#pragma unroll
      for (int b = 0; b < 5; ++b) {
        pr[b] = accr[b];
        pi[b] = acci[b];
      }
    } else {
#pragma unroll
      for (int b = 0; b < 5; ++b) store(v, b, accr[b], acci[b]);
      split();
    }
  }
  if constexpr (DMA) {
#pragma unroll
    for (int b = 0; b < 5; ++b) store(p.nv - 1, b, pr[b], pi[b]);
    wait_vm<0>();  // no copy of this workgroup in flight past its end
  }
}

inline hipError_t launch_cgemm_panel_bf16x3(CgArgs<float, float> a, int nz, bool fixa,
                                            hipStream_t s) {
  if (a.K < 1 || a.K > 64 || a.conjA || a.conjB || a.S || a.accumulate ||
      a.splitA != (1 << 30) || a.splitB != (1 << 30) || a.splitC != (1 << 30) || a.ksA != 1 ||
      a.ksB != 1 || (fixa ? a.vsA : a.vsB) != 0)
    return hipErrorNotSupported;
  if (a.M <= 0 || a.N <= 0 || nz <= 0 || a.nv <= 0) return hipSuccess;
  constexpr int NW = 4;
  a.nz = nz;
  a.tiles_m = (a.M + (fixa ? kPanelRows : 16 * NW) - 1) / (fixa ? kPanelRows : 16 * NW);
  a.tiles_n = (a.N + (fixa ? 16 * NW : kPanelRows) - 1) / (fixa ? 16 * NW : kPanelRows);
  const int gy = nz < 65535 ? nz : 65535;
  const int gz = (nz + gy - 1) / gy;
  const long gx = (long)a.tiles_m * a.tiles_n;
  if (!grid_fits(gx, 64 * NW, gy, gz)) return hipErrorInvalidValue;
  dim3 grid((unsigned)gx, gy, gz);
  // LDS copies of the own rows: rows K complex apart (a contiguous 16-row
  // block), K even (16-byte pieces never straddle a row), 16-byte aligned
  const float* own = fixa ? a.B : a.A;
  const long old = fixa ? a.ldB : a.ldA;
  const long ovs = fixa ? a.vsB : a.vsA;
  const long oso = fixa ? a.soB : a.soA, osi = fixa ? a.siB : a.siA;
  const bool dma = old == a.K && a.K % 2 == 0 && ((uintptr_t)own & 15) == 0 &&
                   ovs % 2 == 0 && oso % 2 == 0 && osi % 2 == 0;
#define SOX_PANEL3(F_, D_)                                                                   \
  hipLaunchKernelGGL((cgemm_panel_bf16x3_kernel<F_, NW, D_>), grid, dim3(64 * NW), 0, s, a)
  if (fixa) {
    if (dma) SOX_PANEL3(true, true); else SOX_PANEL3(true, false);
  } else {
    if (dma) SOX_PANEL3(false, true); else SOX_PANEL3(false, false);
  }
#undef SOX_PANEL3
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The merge product of the one-pass SOSEX_dyn on a k mesh (float plans):
// A(tau_l)[pair][P][u] += sum_q A_bare[l][pair][q][P] G^{k}(tau_l)[u][q],
// k = gidx[pair].  One workgroup per (pair, node): G^k(tau_l) (n x n,
// n <= 64) is staged in LDS once, and each wavefront takes 16-row P blocks
// of A_bare in turn.  Complex values interleaved; each complex multiply-add
// is four real 16x16x4 float32 MFMAs, lane group g holding k = 4 s + g in
// step s.  The accumulators start from the A(tau) values, so A(tau) is read
// and written once per element and A_bare read once.
struct MergeArgs {
  const float* ab;    // complex A_bare: (P, q) at pair ab_so + node ab_si + q N + P
  const float* g;     // complex G: (u, q) at gidx[pair] g_so + node g_si + u n + q
  const int* gidx;
  float* a;           // complex A(tau): (P, u) at pair a_so + node a_si + P n + u
  long ab_so, ab_si, g_so, g_si, a_so, a_si;
  int nodes, n, N;
};
constexpr int kMergeLd = 65;  // LDS row stride of G (complex), n <= 64

template <int SM>
__global__ __launch_bounds__(256) void merge_bare_kernel(const MergeArgs p) {
  __shared__ f32x2 gl[64 * kMergeLd];
  const int pair = blockIdx.x / p.nodes, node = blockIdx.x - pair * p.nodes;
  const int n = p.n, N = p.N;
  const f32x2* G = (const f32x2*)p.g + (long)p.gidx[pair] * p.g_so + (long)node * p.g_si;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int u = e / n, q = e - u * n;
    gl[u * kMergeLd + q] = G[e];
  }
  __syncthreads();
  const f32x2* Ab = (const f32x2*)p.ab + (long)pair * p.ab_so + (long)node * p.ab_si;
  f32x2* Ac = (f32x2*)p.a + (long)pair * p.a_so + (long)node * p.a_si;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int nrb = (N + 15) / 16;
  for (int rb = wave; rb < nrb; rb += 4) {
    const int P0 = 16 * rb;
    const bool prow = P0 + li < N;
    f32x2 av[SM];  // A_bare (P0 + li, 4 s + g)
#pragma unroll
    for (int s = 0; s < SM; ++s) {
      const int q = 4 * s + g;
      av[s] = (prow && q < n) ? Ab[(long)q * N + P0 + li] : f32x2{0.f, 0.f};
    }
    f32x4 re[4], im[4];  // element r of column block c: (P0 + 4 g + r, 16 c + li)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int P = P0 + acc_row<float>(g, r), u = 16 * c + li;
        const f32x2 x = (P < N && u < n) ? Ac[(long)P * n + u] : f32x2{0.f, 0.f};
        re[c][r] = x.x;
        im[c][r] = x.y;
      }
#pragma unroll
    for (int s = 0; s < SM; ++s) {
      const int q = 4 * s + g;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int u = 16 * c + li;
        const f32x2 b = (u < n && q < n) ? gl[u * kMergeLd + q] : f32x2{0.f, 0.f};
        re[c] = mfma16x16x4(av[s].x, b.x, re[c]);
        re[c] = mfma16x16x4(-av[s].y, b.y, re[c]);
        im[c] = mfma16x16x4(av[s].x, b.y, im[c]);
        im[c] = mfma16x16x4(av[s].y, b.x, im[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int P = P0 + acc_row<float>(g, r), u = 16 * c + li;
        if (P < N && u < n) Ac[(long)P * n + u] = f32x2{re[c][r], im[c][r]};
      }
  }
}

// hipErrorNotSupported for n > 64 (the caller takes the generic product)
inline hipError_t launch_merge_bare(const MergeArgs& a, int np2, hipStream_t s) {
  if (a.n < 1 || a.n > 64 || a.N < 1 || a.nodes < 1) return hipErrorNotSupported;
  const long nb = (long)np2 * a.nodes;
  if (nb <= 0) return hipSuccess;
  if (!grid_fits(nb, 256)) return hipErrorInvalidValue;
  const int S = (a.n + 3) / 4;
#define SOX_MERGE(SM_)                                                                    \
  if (S <= SM_) {                                                                         \
    hipLaunchKernelGGL((merge_bare_kernel<SM_>), dim3((unsigned)nb), dim3(256), 0, s, a);  \
    return hipGetLastError();                                                             \
  }
  SOX_MERGE(4)
  SOX_MERGE(8)
  SOX_MERGE(13)
  SOX_MERGE(16)
#undef SOX_MERGE
  return hipErrorNotSupported;
}

// ---------------------------------------------------------------------------
template <int M1, int M2, int M3>
__host__ __device__ constexpr int kdiff_of(int a, int b) {
  return ((((a / (M2 * M3)) - (b / (M2 * M3)) + M1) % M1) * M2 +
          (((a / M3) % M2 - (b / M3) % M2 + M2) % M2)) * M3 +
         ((a % M3 - b % M3 + M3) % M3);
}

// In-register discrete Fourier transform over the momentum mesh (axes of
// length 1, 2 or 3): x[k] <- sum_j x[j] w^(SIGN xi.j), w_a = exp(2 pi i / m_a),
// with k = (k0 M2 + k1) M3 + k2.  One radix-2 or radix-3 butterfly pass per
// axis.
template <typename R, int SIGN, int M1, int M2, int M3, int AX>
__device__ __forceinline__ void mesh_dft_axis(R (&xr)[M1 * M2 * M3], R (&xi)[M1 * M2 * M3]) {
  constexpr int m = AX == 0 ? M1 : (AX == 1 ? M2 : M3);
  constexpr int stride = AX == 0 ? M2 * M3 : (AX == 1 ? M3 : 1);
  constexpr int NK = M1 * M2 * M3;
  if constexpr (m == 2) {
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      if ((k / stride) % 2 != 0) continue;
      const int k1 = k + stride;
      const R ar = xr[k], ai = xi[k], br = xr[k1], bi = xi[k1];
      xr[k] = ar + br; xi[k] = ai + bi;
      xr[k1] = ar - br; xi[k1] = ai - bi;
    }
  } else if constexpr (m == 3) {
    const R s = R(SIGN) * R(0.86602540378443864676);  // sin(2 pi / 3) with the sign
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      if ((k / stride) % 3 != 0) continue;
      const int k1 = k + stride, k2 = k + 2 * stride;
      const R tr = xr[k1] + xr[k2], ti = xi[k1] + xi[k2];
      const R dr = xr[k1] - xr[k2], di = xi[k1] - xi[k2];
      const R hr = xr[k] - R(0.5) * tr, hi = xi[k] - R(0.5) * ti;
      xr[k] += tr; xi[k] += ti;
      // y1 = h + i s d, y2 = h - i s d
      xr[k1] = hr - s * di; xi[k1] = hi + s * dr;
      xr[k2] = hr + s * di; xi[k2] = hi - s * dr;
    }
  }
}

template <typename R, int SIGN, int M1, int M2, int M3>
__device__ __forceinline__ void mesh_dft(R (&xr)[M1 * M2 * M3], R (&xi)[M1 * M2 * M3]) {
  mesh_dft_axis<R, SIGN, M1, M2, M3, 0>(xr, xi);
  mesh_dft_axis<R, SIGN, M1, M2, M3, 1>(xr, xi);
  mesh_dft_axis<R, SIGN, M1, M2, M3, 2>(xr, xi);
}

// The n_k^3 D step of a solid (section on solids: for every (P, R) pair,
// D^{k_t}_PR accumulates C^{q2,k_w}_RvP B^{q1,k_w-q2}_PRv over k_w, q2 and
// v with q1 = k_w - k_t).  B and C are stored [pair][v][P][R] with pair =
// q * n_k + k; with k_v = k_w - q2 the sum reads, per element e = (P, R),
//
//   D[k_t][e] += scale * sum_{k_v, v} sum_{k_w} c_{k_v}[k_w] b_{k_v}[k_w - k_t],
//   c_{k_v}[k_w] = C[(k_w - k_v, k_w)][v][e],  b_{k_v}[j] = B[(j, k_v)][v][e].
//
// The inner sum is a cyclic cross-correlation over the momentum group, so
// with F[f](xi) = sum_k f[k] w^(xi.k) it is F^-1[ F[c] * F~[b] ] where F~
// uses the conjugate phases.  One thread per element: for each (k_v, v) it
// loads the n_k values of b and of c (non-temporal loads: each is read
// once), transforms both in registers (one butterfly pass per mesh axis),
// and accumulates the n_k products of the transforms in float64; the
// inverse transform runs once at the end.  This
// is the same sum as the direct n_k^2 products, in n_k log n_k work.  The
// mesh is a template parameter (every index a compile-time register).
// Pairs are sp elements apart, v slices NN apart; nv slices are summed.  The
// k_v range is split over the rows of the grid (gk momenta each) so that the
// launch fills the chip; each row writes its own partial D, summed by
// dsum_kernel; grid layer z is the z-th tau node of a slab (B, C sbt and D
// sdt apart).
template <typename T, int M1, int M2, int M3>
__global__ __launch_bounds__(256) void dstep_mesh_kernel(const T* __restrict__ B,
                                                         const T* __restrict__ C, double* D,
                                                         long NN, long sp, int nv, int gk,
                                                         long sbt, long sdt, double scale,
                                                         int accumulate) {
  constexpr int NK = M1 * M2 * M3;
  using V2 = vec2_t<T>;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  const int kv0 = blockIdx.y * gk;
  const int kv1 = kv0 + gk < NK ? kv0 + gk : NK;
  D += 2 * ((long)blockIdx.y * NK * NN + (long)blockIdx.z * sdt);
  B += 2 * (long)blockIdx.z * sbt;
  C += 2 * (long)blockIdx.z * sbt;
  const V2* Bp = (const V2*)B + e;
  const V2* Cp = (const V2*)C + e;
  double hr[NK], hi[NK];  // F[D] accumulated
#pragma unroll
  for (int k = 0; k < NK; ++k) hr[k] = hi[k] = 0.0;
  for (int kv = kv0; kv < kv1; ++kv) {
    for (int v = 0; v < nv; ++v) {
      const long ov = (long)v * NN;
      T br[NK], bi[NK], cr[NK], ci[NK];
#pragma unroll
      for (int q1 = 0; q1 < NK; ++q1) {
        const V2 x = __builtin_nontemporal_load(&Bp[(long)(q1 * NK + kv) * sp + ov]);
        br[q1] = x.x;
        bi[q1] = x.y;
      }
#pragma unroll
      for (int kw = 0; kw < NK; ++kw) {
        const int q2 = kdiff_of<M1, M2, M3>(kw, kv);
        const V2 x = __builtin_nontemporal_load(&Cp[(long)(q2 * NK + kw) * sp + ov]);
        cr[kw] = x.x;
        ci[kw] = x.y;
      }
      mesh_dft<T, +1, M1, M2, M3>(cr, ci);
      mesh_dft<T, -1, M1, M2, M3>(br, bi);
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        hr[k] += (double)(cr[k] * br[k] - ci[k] * bi[k]);
        hi[k] += (double)(cr[k] * bi[k] + ci[k] * br[k]);
      }
    }
  }
  mesh_dft<double, -1, M1, M2, M3>(hr, hi);
  const double f = scale / NK;
#pragma unroll
  for (int kt = 0; kt < NK; ++kt) {
    double* o = D + 2 * ((long)kt * NN + e);
    double re = f * hr[kt], im = f * hi[kt];
    if (accumulate) {
      re += o[0];
      im += o[1];
    }
    o[0] = re;
    o[1] = im;
  }
}

// D[i] (+)= sum_g Dp[g][i], i < count (float64 values): the partial D sums of
// the k_v groups.
__global__ __launch_bounds__(256) void dsum_kernel(const double* Dp, int ng, long count, double* D,
                                                   int accumulate) {
  SOX_FOR_FLAT(i, count) {
    double acc = accumulate ? D[i] : 0.0;
    for (int g = 0; g < ng; ++g) acc += Dp[(long)g * count + i];
    D[i] = acc;
  }
}

// Any mesh (runtime momentum-difference table kdiff[n_k][n_k]): one thread
// per (element, k_t), operands re-read per k_t.
template <typename T>
__global__ __launch_bounds__(256) void dstep_any_kernel(const T* __restrict__ B,
                                                        const T* __restrict__ C,
                                                        const int* __restrict__ kdiff, double* D,
                                                        long NN, int nk, long sp, int nv, long sbt,
                                                        long sdt, double scale, int accumulate) {
  using V2 = vec2_t<T>;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= NN * nk) return;
  D += 2 * (long)blockIdx.y * sdt;
  B += 2 * (long)blockIdx.y * sbt;
  C += 2 * (long)blockIdx.y * sbt;
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
// eq:GG for a slab of momentum pairs and one orbital v (float64):
//   GG[tau][l][u][Q] = GwP^{k_v - q1}(tau)[u][Q] * GRqT^{k_v}(beta - tau)[v][Q]
// for pair = p0 + l = q1 n_k + k_v; GwP and GRqT are stored [tau][k][n][N].
__global__ __launch_bounds__(256) void gg_solid_kernel(const double* __restrict__ gwp,
                                                       const double* __restrict__ grqt,
                                                       const int* __restrict__ k_of,
                                                       const int* __restrict__ kmq_of, double* gg,
                                                       int nt, int nk, int n, int N, int p0, int cnt,
                                                       int ps, int v) {
  const long per = (long)n * N;
  SOX_FOR_FLAT(idx, (long)nt * cnt * per) {
    const long tl = idx / per;
    const long uq = idx - tl * per;
    const int t = (int)(tl / cnt);
    const int l = (int)(tl - (long)t * cnt);
    const int Q = (int)(uq % N);
    const int pair = p0 + l;
    const int kv = k_of[pair], kq = kmq_of[pair];
    const double* a = gwp + 2 * (((long)t * nk + kq) * per + uq);
    const double* b = grqt + 2 * (((long)(nt - 1 - t) * nk + kv) * per + (long)v * N + Q);
    double* o = gg + 2 * (((long)t * ps + l) * per + uq);
    o[0] = a[0] * b[0] - a[1] * b[1];
    o[1] = a[0] * b[1] + a[1] * b[0];
  }
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
// out[k][v][t][s] = G^k(tau_{n_tau-1-t})[s][v] in T (complex): for each
// momentum k and orbital v, rows t of the mirrored node's column v, the A
// operand of the bare term taken one v at a time over every node.
template <typename T>
__global__ void mirror_columns_kernel(const double* G, T* out, int nk, int nt, int n) {
  const long count = (long)nk * n * nt * n;
  SOX_FOR_FLAT(i, count) {
    const int s = (int)(i % n);
    const long r = i / n;
    const int t = (int)(r % nt);
    const long r2 = r / nt;
    const int v = (int)(r2 % n);
    const int k = (int)(r2 / n);
    const long src = (((long)k * nt + (nt - 1 - t)) * n + s) * n + v;
    out[2 * i] = T(G[2 * src]);
    out[2 * i + 1] = T(G[2 * src + 1]);
  }
}

// Real block form of the complex product A(Omega) = W(Omega) GG(Omega) on a
// real NT GEMM: with A rows [Re W | -Im W] (K = 2 Nq) and, per complex
// column c, the two B rows [Re GG | Im GG] and [Im GG | -Re GG], the real
// product writes Re and Im of column c next to each other (interleaved
// complex).  Both B rows of c are read from one [Re | Im | -Re] row of 3 Nq
// (row 2c + s starts s Nq into it).  Each half is Nq wide (N rounded up to
// 16) and zero past N.  Output float (f != null) or bf16 hi / lo planes.
__device__ __forceinline__ void put_split(float x, long i, float* f, bf16_t* hi, bf16_t* lo) {
  if (f) {
    f[i] = x;
  } else {
    const bf16_t h = f32_to_bf16(x);
    hi[i] = h;
    lo[i] = f32_to_bf16(x - bf16_to_f32(h));
  }
}

// wm [batch][N][N] complex -> [batch][N][2 Nq] = [Re W | -Im W]
__global__ void wblock_kernel(const float* wm, long nbatch, int N, int Nq, float* f, bf16_t* hi,
                              bf16_t* lo) {
  const long row = 2L * Nq;
  SOX_FOR_FLAT(i, nbatch * N * row) {
    const long br = i / row;              // (batch, P)
    const int k = (int)(i - br * row);
    const int half = k >= Nq, Q = k - half * Nq;
    float x = 0.f;
    if (Q < N) {
      const float* w = wm + 2 * (br * N + Q);
      x = half ? -w[1] : w[0];
    }
    put_split(x, i, f, hi, lo);
  }
}

// GG rows: ggw [r][ldr complex][...] with ncols columns of N per row r ->
// [r][ncols][3 Nq] = [Re | Im | -Re] (row stride ncols * 3 Nq per r)
__global__ void gblock_kernel(const float* ggw, long nr, long ldr, long ncols, int N, int Nq,
                              float* f, bf16_t* hi, bf16_t* lo) {
  const long row = 3L * Nq;
  SOX_FOR_FLAT(i, nr * ncols * row) {
    const long rc = i / row;
    const int k = (int)(i - rc * row);
    const long r = rc / ncols, c = rc - r * ncols;
    const int part = k / Nq, Q = k - part * Nq;
    float x = 0.f;
    if (Q < N) {
      const float* gv = ggw + 2 * (r * ldr + c * N + Q);
      x = part == 0 ? gv[0] : part == 1 ? gv[1] : -gv[0];
    }
    put_split(x, i, f, hi, lo);
  }
}

// The solid eq:GG chain's forward transform with GG formed in registers,
// written straight in the block form above:
//   GG(+-Omega_m)[l][u][Q] = sum_j T(+-)[m][j] G^{k_v - q1}_uQ(tau_j) G^{k_v}_Qv(beta - tau_j)
// for the pairs l of a slab and one orbital v, with T(+) = T_fwd = a + i b
// and T(-) = conj T_fwd.  For x = GG(tau) = xr + i xi both signs come from
// the same four real products P1 = a xr, P2 = b xi, P3 = a xi, P4 = b xr:
//   GG(+) = (P1 - P2) + i (P3 + P4),   GG(-) = (P1 + P2) + i (P3 - P4),
// half the multiplies of one complex product per sign.  GG is formed from
// float32 copies of the two projections and transformed on float32 MFMAs
// (float plans only: the block form it feeds holds float32 or bf16 hi and lo
// planes).  NRB row tiles of 16 frequencies.  T_fwd stays in LDS for
// the launch.  A wavefront owns 16 consecutive Q of one (k_q = k_v - q1, u)
// and one momentum transfer at a time, the transfers of the slab being the
// fastest index: the G^{k_q}_uQ columns it reads are read by its neighbours
// at the same time (once per slab from HBM instead of once per pair).  Rows
// r < n_omega of the output are +Omega_r, rows n_omega + m are -Omega_m;
// [Re | Im | -Re] of 3 Nq per (r, l, u) column, zero for Q >= N.
constexpr int kFtsRows = 64, kFtsLd = 113;  // n_omega <= 64, n_tau <= 112 nodes
constexpr int kFtsChunk = 4;                // k steps (of four nodes) per load chunk
struct FtSolidArgs {
  const double* tfc;   // [2 n_omega][nt] complex; rows < n_omega hold T_fwd
  const float* gwp;    // [nt][nk][n][N] complex, G_uQ(tau)
  const float* grqt;   // [nt][nk][n][N] complex, G_vQ(tau), read at beta - tau
  const int* kdiff;    // [nk][nk]: index of k_a - k_b (index 0 is k = 0)
  float* f;            // float output, or
  bf16_t* hi;          // bf16 hi and lo planes
  bf16_t* lo;
  long rstride;        // output elements between rows r: cp n 3 Nq
  int nw, nt, nk, n, N, Nq, p0, cp, v;
};

// 16 NRB rows of T_fwd in LDS (43 KB for three row tiles): three workgroups
// of four wavefronts per CU, at most 168 VGPRs
template <int NRB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void ft_solid_kernel(const FtSolidArgs a, long nblocks) {
  __shared__ float tr[16 * NRB * kFtsLd], ti[16 * NRB * kFtsLd];
  const int K = a.nt, Kp = (K + 3) & ~3;
  for (int e = threadIdx.x; e < 16 * NRB * Kp; e += blockDim.x) {
    const int r = e / Kp, k = e - (e / Kp) * Kp;
    const bool ok = r < a.nw && k < K;
    tr[r * kFtsLd + k] = ok ? (float)a.tfc[2 * ((long)r * K + k)] : 0.f;
    ti[r * kFtsLd + k] = ok ? (float)a.tfc[2 * ((long)r * K + k) + 1] : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nwaves = blockDim.x >> 6;
  const int nqb = a.Nq / 16;
  const int ntr = a.cp / a.nk;  // momentum transfers in the slab
  const long per = (long)a.n * a.N;
  const long tsb = 8L * a.nk * per;  // bytes between nodes
  // workgroups remapped per XCD: in each round of the persistent loop an
  // XCD takes a contiguous range of items, so the items sharing G rows
  // (transfers of one (k_q, u, Q block), then the u of one G_Qv block) run
  // behind one L2 (C5: GG + FT 0.72 - 0.87 -> 0.63 s per sweep, steady)
  for (long blk = (long)xcd_remap(blockIdx.x, gridDim.x) * nwaves + wave; blk < nblocks;
       blk += (long)gridDim.x * nwaves) {
    const int t = (int)(blk % ntr);
    long rest = blk / ntr;
    const int qb = (int)(rest % nqb);
    rest /= nqb;
    const int u = (int)(rest % a.n);
    const int kq = (int)(rest / a.n);
    const int q1 = a.p0 / a.nk + t;
    // k_q + q1 = k_q - (0 - q1), the same for the whole wavefront
    const int kv = __builtin_amdgcn_readfirstlane(a.kdiff[kq * a.nk + a.kdiff[q1]]);
    const int l = t * a.nk + kv;                     // pair - p0
    const int Q = 16 * qb + li;
    const bool qok = Q < a.N;
    const int Qc = qok ? Q : a.N - 1;
    // wavefront-uniform bases (scalar registers) plus one 32-bit lane offset
    // each: node g of a step of four and column Q (G(beta - tau) runs
    // backwards: node K - 1 - k = (K - 4 - 4 step) + 3 - g)
    const char* gu0 = (const char*)(a.gwp + 2 * ((long)kq * per + (long)u * a.N + 16 * qb));
    const char* gv0 = (const char*)(a.grqt + 2 * ((long)kv * per + (long)a.v * a.N + 16 * qb));
    const unsigned lu = (unsigned)(g * tsb + 8 * (Qc - 16 * qb));
    const unsigned lv = (unsigned)((3 - g) * tsb + 8 * (Qc - 16 * qb));
    f32x4 p1[NRB], p2[NRB], p3[NRB], p4[NRB];
#pragma unroll
    for (int b = 0; b < NRB; ++b) {
      p1[b] = zero4<float>();
      p2[b] = zero4<float>();
      p3[b] = zero4<float>();
      p4[b] = zero4<float>();
    }
    // nodes in chunks of kFtsChunk steps of four; the next chunk's G values
    // are loaded while the MFMAs of the current one run
    const int nst = Kp / 4, nch = (nst + kFtsChunk - 1) / kFtsChunk;
    f32x2 ru[kFtsChunk], rv[kFtsChunk];
    auto load = [&](int kc) {
      // (the chunk index through readfirstlane keeps the addresses a scalar
      // base plus the lane offset instead of one 64-bit register pair per load)
      kc = __builtin_amdgcn_readfirstlane(kc);
#pragma unroll
      for (int j = 0; j < kFtsChunk; ++j) {
        const int st = kc * kFtsChunk + j;
        const bool ok = qok && 4 * st + g < K;
        ru[j] = ok ? *(const f32x2*)(gu0 + 4L * st * tsb + lu) : f32x2{0.f, 0.f};
        rv[j] = ok ? *(const f32x2*)(gv0 + (long)(K - 4 - 4 * st) * tsb + lv) : f32x2{0.f, 0.f};
      }
    };
    // the T_fwd values of step st + 1 are read from LDS while the MFMAs of
    // step st run
    auto rd = [&](int st, float (&x)[NRB], float (&y)[NRB]) {
#pragma unroll
      for (int b = 0; b < NRB; ++b) {
        const int o = (16 * b + li) * kFtsLd + 4 * st + g;
        x[b] = tr[o];
        y[b] = ti[o];
      }
    };
    float ta[NRB], tb[NRB];
    rd(0, ta, tb);
    load(0);
    for (int kc = 0; kc < nch; ++kc) {
      float xr[kFtsChunk], xi[kFtsChunk];
#pragma unroll
      for (int j = 0; j < kFtsChunk; ++j) {
        xr[j] = ru[j].x * rv[j].x - ru[j].y * rv[j].y;
        xi[j] = ru[j].x * rv[j].y + ru[j].y * rv[j].x;
      }
      if (kc + 1 < nch) load(kc + 1);
#pragma unroll
      for (int j = 0; j < kFtsChunk; ++j) {
        const int st = kc * kFtsChunk + j;
        if (st >= nst) break;
        float na[NRB], nb[NRB];
#pragma unroll
        for (int b = 0; b < NRB; ++b) na[b] = nb[b] = 0.f;
        if (st + 1 < nst) rd(st + 1, na, nb);
#pragma unroll
        for (int b = 0; b < NRB; ++b) {
          p1[b] = mfma16x16x4(ta[b], xr[j], p1[b]);
          p2[b] = mfma16x16x4(tb[b], xi[j], p2[b]);
          p3[b] = mfma16x16x4(ta[b], xi[j], p3[b]);
          p4[b] = mfma16x16x4(tb[b], xr[j], p4[b]);
        }
#pragma unroll
        for (int b = 0; b < NRB; ++b) {
          ta[b] = na[b];
          tb[b] = nb[b];
        }
        // one step in flight at a time (short live ranges, no spills)
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // lane (li, g) holds frequencies m = 16 b + 4 g + i of column Q
    const long col = ((long)l * a.n + u) * 3 * a.Nq + Q;
#pragma unroll
    for (int b = 0; b < NRB; ++b) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 16 * b + acc_row<float>(g, i);
        if (m >= a.nw) continue;
        const float pr = qok ? p1[b][i] - p2[b][i] : 0.f, pi = qok ? p3[b][i] + p4[b][i] : 0.f;
        const float mr = qok ? p1[b][i] + p2[b][i] : 0.f, mi = qok ? p3[b][i] - p4[b][i] : 0.f;
        const long op = (long)m * a.rstride + col, om = (long)(a.nw + m) * a.rstride + col;
        put_split(pr, op, a.f, a.hi, a.lo);
        put_split(pi, op + a.Nq, a.f, a.hi, a.lo);
        put_split(-pr, op + 2 * a.Nq, a.f, a.hi, a.lo);
        put_split(mr, om, a.f, a.hi, a.lo);
        put_split(mi, om + a.Nq, a.f, a.hi, a.lo);
        put_split(-mr, om + 2 * a.Nq, a.f, a.hi, a.lo);
      }
    }
  }
}

// The matching inverse transform (float plans).  With c = T_bwd / 2 = cr +
// i ci the coefficient of A(+i Omega_m) and conj c that of A(-i Omega_m),
// and A(+-i Omega_m) = a+- + i b+-:
//   Re A(tau) = sum_m cr (a+ + a-) + ci (b- - b+)
//   Im A(tau) = sum_m cr (b+ + b-) + ci (a+ - a-),
// one real product over K = 2 n_omega with two output columns per complex
// column: half the multiplies of the complex product over both signs.
// Float32 MFMAs; [cr; ci] stays in LDS for the launch; a wavefront owns 16
// consecutive complex columns and every node (up to eight row tiles of 16)
// at a time, so each A(+-Omega) value is read once.
// n_tau <= 128; n_omega <= W, the kernel's template width: 40 (three
// workgroups per CU) or 64 (the wider grids, e.g. IR grids: two per CU)
constexpr int kIftRows = 128, kIftW = 40, kIftWMax = 64, kIftLd = 144;
struct IftSolidArgs {
  const double* tbc;  // [nt][2 n_omega] complex; columns < n_omega hold T_bwd / 2
  const float* aw;    // [2 n_omega][fstride] complex: +Omega rows, then -Omega rows
  float* out;         // [nt][ldo] complex
  long fstride, ldo, cols;
  int nt, nw;
};

// W = 40: three workgroups per CU (LDS), three wavefronts per SIMD
template <int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W <= 40 ? 3 : 2)))
void ift_solid_kernel(const IftSolidArgs a) {
  __shared__ float cr[W * kIftLd], ci[W * kIftLd];  // [m][tau]
  for (int e = threadIdx.x; e < W * kIftRows; e += blockDim.x) {
    const int m = e / kIftRows, t = e - m * kIftRows;
    const bool ok = m < a.nw && t < a.nt;
    const double* c = a.tbc + 2 * ((long)t * 2 * a.nw + m);
    cr[m * kIftLd + t] = ok ? (float)c[0] : 0.f;
    ci[m * kIftLd + t] = ok ? (float)c[1] : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nwaves = blockDim.x >> 6;
  const int ns = (a.nw + 3) / 4;    // k steps of four frequencies
  const int nrt = (a.nt + 15) / 16;  // row tiles of nodes
  const long ntiles = (a.cols + 15) / 16;
  constexpr int kS = W / 4;
  const long tstep = (long)gridDim.x * nwaves;
  // lane (li, g) holds frequency m = 4 s + g of its column; the next tile's
  // values are loaded while the MFMAs of the current one run
  // a tile's values: a wavefront-uniform base per step (scalar registers)
  // plus one 32-bit lane offset, frequency g of the step and column li
  const long fsb = 8 * a.fstride;  // bytes between frequencies
  const unsigned loff = (unsigned)(g * fsb + 8 * li);
  const long soff = 8 * ((long)(4 * g) * a.ldo + li);  // output: node 4 g, column li
  f32x2 np[kS], nm[kS];
  auto load = [&](long tl) {
    const bool ok = tl < ntiles && tl * 16 + li < a.cols;
    const char* b0 = (const char*)a.aw + 128 * (tl < ntiles ? tl : 0);  // uniform
#pragma unroll
    for (int s = 0; s < kS; ++s) {
      const bool mk = ok && s < ns && 4 * s + g < a.nw;
      np[s] = mk ? *(const f32x2*)(b0 + 4L * s * fsb + loff) : f32x2{0.f, 0.f};
      nm[s] = mk ? *(const f32x2*)(b0 + (a.nw + 4L * s) * fsb + loff) : f32x2{0.f, 0.f};
    }
  };
  long tile = (long)blockIdx.x * nwaves + wave;
  load(tile);
  for (; tile < ntiles; tile += tstep) {
    const long c = tile * 16 + li;
    const bool cok = c < a.cols;
    float sa[kS], db[kS], sb[kS], da[kS];
#pragma unroll
    for (int s = 0; s < kS; ++s) {
      sa[s] = np[s].x + nm[s].x;
      db[s] = nm[s].y - np[s].y;
      sb[s] = np[s].y + nm[s].y;
      da[s] = np[s].x - nm[s].x;
    }
    load(tile + tstep);
    // the nodes in two groups of four row tiles (32 accumulator registers)
#pragma unroll
    for (int h = 0; h < kIftRows / 64; ++h) {
      if (4 * h >= nrt) break;
      f32x4 ar[4], ai[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ar[i] = zero4<float>();
        ai[i] = zero4<float>();
      }
#pragma unroll
      for (int s = 0; s < kS; ++s) {
        if (s >= ns) break;
        const int m = 4 * s + g;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (4 * h + i >= nrt) break;
          const int o = m * kIftLd + 16 * (4 * h + i) + li;
          const float tR = cr[o], tI = ci[o];
          ar[i] = mfma16x16x4(tR, sa[s], ar[i]);
          ar[i] = mfma16x16x4(tI, db[s], ar[i]);
          ai[i] = mfma16x16x4(tR, sb[s], ai[i]);
          ai[i] = mfma16x16x4(tI, da[s], ai[i]);
        }
        // one step's LDS reads at a time (short live ranges, no spills)
        __builtin_amdgcn_sched_barrier(0);
      }
      if (!cok) continue;
      // lane (li, g) holds nodes 16 rt + 4 g + r of column c: a uniform base
      // per (rt, r) plus the lane's offset
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int t = 16 * (4 * h + i) + acc_row<float>(g, r);
          char* ob = (char*)a.out + 8 * ((long)(16 * (4 * h + i) + r) * a.ldo + 16 * tile);
          if (t < a.nt) *(f32x2*)(ob + soff) = f32x2{ar[i][r], ai[i][r]};
        }
      }
    }
  }
}

__global__ void real_to_complex_kernel(const double* x, double* out, long count) {
  SOX_FOR_FLAT(i, count) {
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
