// Launch sequence of the k-point (periodic solid) SOX path.  Included by
// sox_api.hip inside its internal namespace (it uses the plan, the status
// helpers and the per-stage profiling scopes defined there).
//
// The chain is the paper's momentum-resolved one (section "THC-SOX and
// THC-SOSEX: algorithm and implementation details for solids and
// molecules"), with pair = q * n_k + k for every (q, k) momentum pair:
//
//   Ut^{(q,k)}[a][P][b] = sum_Q U^q_PQ conj(X^{k-q}_aQ) X^k_bQ   (eq:U_contraction)
//   GRq^k[R][q]   = sum_u X^k_uR G^k_uq          GwPt^k[P][w] = sum_p conj(X^k_pP) G^k_wp
//   A[(q1,k_v)][v][P][q] = sum_s G^{k_v}(beta - tau)_sv Ut1^{(q1,k_v)}[q][P][s]
//   B[(q1,k_v)][v][P][R] = sum_q A[(q1,k_v)][v][P][q] GRq^{k_v - q1}[R][q]
//   C[(q2,k_w)][v][P][R] = sum_w GwPt^{k_w}[P][w] Ut2^{(q2,k_w)}[v][R][w]
//   D^{k_t}[P][R] = (1/n_k) sum_{k_w, q2, v} C[(q2,k_w)][v][P][R] B[(k_w - k_t, k_w - q2)][v][P][R]
//   Sigma^{k_t}_tr = -(1/n_k) sum_{P,R} conj(X^{k_t}_tR) D^{k_t}[P][R] X^{k_t}_rP
//
// Per tau node the A step runs once for every v (the U-tensor is streamed
// once per node); B, C and D then run over v slabs whose width keeps B and C
// within the workspace budget, and D accumulates over the slabs in float64.
// The U-contraction, the projections and the back-transform run in float64;
// A, B, C and the D step in the plan's precision.

struct SolidLayout {
  size_t ut1, ut2, xtd, gtd, gtt, grq, gwp, abuf, bbuf, cbuf, dbuf, dpart, ebuf, total;
};

// Number of k_v groups of the D step: enough workgroup rows that the launch
// holds at least 16384 wavefronts.
int solid_dgroups(const sox_plan& p) {
  const long NN = (long)p.N * p.N;
  const long want = (16384L * 64 + NN - 1) / NN;
  const int gk = (int)((p.nk + std::min<long>(want, p.nk) - 1) / std::min<long>(want, p.nk));
  return (p.nk + gk - 1) / gk;
}

SolidLayout solid_layout_for(const sox_plan& p, int entry, int vc) {
  SolidLayout L{};
  const size_t es = 2 * elem_size(p.precision);  // complex element
  const size_t n = p.n, N = p.N, nt = p.n_tau, nk = p.nk, np2 = nk * nk;
  Carver c;
  L.ut1 = c.take(np2 * n * N * n * es);
  L.ut2 = (entry == SOX_ENTRY_BARE) ? L.ut1 : c.take(np2 * n * N * n * es);
  L.xtd = c.take(nk * N * n * 16);
  L.gtd = c.take(nk * nt * n * n * 16);
  L.gtt = c.take(nk * nt * n * n * es);
  L.grq = c.take(nt * nk * N * n * es);
  L.gwp = c.take(nt * nk * N * n * es);
  L.abuf = c.take(np2 * n * N * n * es);
  L.bbuf = c.take(np2 * (size_t)vc * N * N * es);
  L.cbuf = c.take(np2 * (size_t)vc * N * N * es);
  L.dbuf = c.take(nk * N * N * 16);
  const int ng = solid_dgroups(p);
  L.dpart = ng > 1 ? c.take((size_t)ng * nk * N * N * 16) : L.dbuf;
  L.ebuf = c.take(nk * n * N * 16);
  L.total = c.off;
  return L;
}

int solid_vc(const sox_plan& p, int entry) { return entry == SOX_ENTRY_BARE ? p.vcs_bare : p.vcs; }

size_t solid_dyn_total(const sox_plan& p, bool with_bare = false);  // with the dynamic launch sequence

size_t solid_workspace_bytes(const sox_plan& p, int entry) {
  if (entry == SOX_ENTRY_DYNAMIC) return p.n_omega > 0 ? solid_dyn_total(p) : 0;
  return solid_layout_for(p, entry, solid_vc(p, entry)).total;
}

// Largest v-slab width that keeps the entry's workspace within the budget,
// then evened out over the slabs it implies.
int pick_solid_vc(const sox_plan& p, int entry) {
  const size_t budget = ws_budget();
  int vc = p.n;
  while (vc > 1 && solid_layout_for(p, entry, vc).total > budget) --vc;
  const int slabs = (p.n + vc - 1) / vc;
  return (p.n + slabs - 1) / slabs;
}

// Host momentum tables, uploaded once per plan: for pair = q * n_k + k,
// k_of = k, q_of = q, kmq_of = index of k - q; kdiff[a][b] = index of k_a - k_b.
std::vector<int> solid_tables(const int mesh[3]) {
  const int m0 = mesh[0], m1 = mesh[1], m2 = mesh[2], nk = m0 * m1 * m2;
  auto kd = [&](int a, int b) {
    const int a0 = a / (m1 * m2), a1 = (a / m2) % m1, a2 = a % m2;
    const int b0 = b / (m1 * m2), b1 = (b / m2) % m1, b2 = b % m2;
    return (((a0 - b0 + m0) % m0) * m1 + ((a1 - b1 + m1) % m1)) * m2 + ((a2 - b2 + m2) % m2);
  };
  const int np2 = nk * nk;
  std::vector<int> t(4 * (size_t)np2);
  for (int q = 0; q < nk; ++q)
    for (int k = 0; k < nk; ++k) {
      const int pr = q * nk + k;
      t[pr] = k;
      t[np2 + pr] = q;
      t[2 * np2 + pr] = kd(k, q);
    }
  for (int a = 0; a < nk; ++a)
    for (int b = 0; b < nk; ++b) t[3 * (size_t)np2 + a * nk + b] = kd(a, b);
  return t;
}

// Tile shapes of the complex product.  0: 64 x 64 workgroup tile (2 x 2
// wavefronts of 32 x 32).  1: 64 x 64 as four 64 x 16 wavefronts, for the A
// step, whose 64 rows hold every v so that each U-tensor row is read once.
// 2: the B and C steps, five wavefronts stacked along the rows, each 16 x 80
// (float32) or 16 x 16 (float64): an 80 x 80 or 80 x 16 tile, which divides
// N = 400 exactly.  3: 128 x 64 (eight 64 x 16 wavefronts), for the inverse
// transform over up to 128 tau nodes.  4: 80 x 64 (float32) or 80 x 32
// (float64) for W(Omega) GG(Omega) and the forward transforms (2 n_Omega
// rows).  5: 112 x 32 (seven 16 x 32 wavefronts), for the inverse transform
// over up to 112 tau nodes.
template <typename T, typename TC>
sox_status cg_launch(const CgArgs<T, TC>& a, int nz, int shape, hipStream_t s) {
  if (shape == 1) {
    SOX_HIP((launch_cgemm<T, TC, 1, 4, 4, 1>(a, nz, s)));
  } else if (shape == 3) {
    SOX_HIP((launch_cgemm<T, TC, 2, 4, 4, 1>(a, nz, s)));
  } else if (shape == 4) {
    if constexpr (sizeof(T) == 4) SOX_HIP((launch_cgemm<T, TC, 5, 1, 1, 4>(a, nz, s)));
    else SOX_HIP((launch_cgemm<T, TC, 5, 1, 1, 2>(a, nz, s)));
  } else if (shape == 5) {
    SOX_HIP((launch_cgemm<T, TC, 7, 1, 1, 2>(a, nz, s)));
  } else if (shape == 2) {
    if constexpr (sizeof(T) == 4) SOX_HIP((launch_cgemm<T, TC, 5, 1, 1, 5>(a, nz, s)));
    else SOX_HIP((launch_cgemm<T, TC, 5, 1, 1, 1>(a, nz, s)));
  } else {
    SOX_HIP((launch_cgemm<T, TC, 2, 2, 2, 2>(a, nz, s)));
  }
  return SOX_OK;
}

// The B (fixa = false) and C (fixa = true) steps: the LDS-panel kernel where
// it applies (float32, K <= 64; split bf16 x 3 products for bf16 plans), else
// the generic kernel with tile `shape`.
template <typename T>
sox_status bc_launch(const CgArgs<T, T>& a, int nz, bool fixa, int shape, hipStream_t s,
                     bool bf16 = false) {
  if constexpr (sizeof(T) == 4) {
    if (bf16) {
      const hipError_t e = launch_cgemm_panel_bf16x3(a, nz, fixa, s);
      if (e == hipSuccess) return SOX_OK;
      if (e != hipErrorNotSupported)
        return fail(SOX_ERR_HIP, "split panel kernel launch failed: %s", hipGetErrorString(e));
    }
    if (getenv("SOX_NO_PANEL") == nullptr) {
      const hipError_t e = launch_cgemm_panel(a, nz, fixa, s);
      if (e == hipSuccess) return SOX_OK;
      if (e != hipErrorNotSupported)
        return fail(SOX_ERR_HIP, "panel kernel launch failed: %s", hipGetErrorString(e));
    }
  }
  return cg_launch(a, nz, shape, s);
}

// Tile of the B and C steps for this N: the 80-row tiles when they pad less
// than the 64 x 64 ones.
int bc_shape(int N) {
  const long w80 = ((N + 79) / 80) * 80L, w64 = ((N + 63) / 64) * 64L;
  return w80 < w64 ? 2 : 0;
}

// D (+)= the D step of nv orbitals v for ntl tau nodes (B and C sbt apart
// per node, pairs sp apart; D sdt apart).  grouped: the templated kernels
// split k_v over solid_dgroups(p) workgroup rows that write per-group partial
// sums into Dp (summed by solid_dsum); otherwise, and for the any-mesh
// kernel, D is written directly.
template <typename T>
sox_status launch_dstep(const sox_plan& p, const T* B, const T* C, double* D, double* Dp, long sp,
                        int nv, int ntl, long sbt, long sdt, bool grouped, bool acc,
                        hipStream_t s) {
  const long NN = (long)p.N * p.N;
  const double scale = 1.0 / p.nk;
  const int ng = grouped ? solid_dgroups(p) : 1;
  const int gk = (p.nk + ng - 1) / ng;
  double* out = grouped ? Dp : D;
  const dim3 grid((unsigned)((NN + 255) / 256), (unsigned)ng, (unsigned)ntl);
  const int* m = p.mesh_canon;
#define SOX_DSTEP(A_, B_, C_)                                                                 \
  if (m[0] == A_ && m[1] == B_ && m[2] == C_) {                                              \
    hipLaunchKernelGGL((dstep_mesh_kernel<T, A_, B_, C_>), grid, dim3(256), 0, s, B, C, out,   \
                       NN, sp, nv, gk, sbt, sdt, scale, acc ? 1 : 0);                         \
    SOX_HIP(hipGetLastError());                                                               \
    return SOX_OK;                                                                            \
  }
  SOX_DSTEP(2, 1, 1)
  SOX_DSTEP(3, 1, 1)
  SOX_DSTEP(2, 2, 1)
  SOX_DSTEP(2, 3, 1)
  SOX_DSTEP(3, 2, 1)
  SOX_DSTEP(3, 3, 1)
  SOX_DSTEP(2, 2, 2)
  SOX_DSTEP(3, 3, 3)
#undef SOX_DSTEP
  const long tot = NN * p.nk;
  hipLaunchKernelGGL((dstep_any_kernel<T>), dim3((unsigned)((tot + 255) / 256), (unsigned)ntl),
                     dim3(256), 0, s, B, C, p.d_ktab + 3 * (size_t)p.nk * p.nk, D, NN, p.nk, sp,
                     nv, sbt, sdt, scale, acc ? 1 : 0);
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}

bool dstep_templated(const sox_plan& p) {
  static const int meshes[8][3] = {{2, 1, 1}, {3, 1, 1}, {2, 2, 1}, {2, 3, 1},
                                   {3, 2, 1}, {3, 3, 1}, {2, 2, 2}, {3, 3, 3}};
  for (auto& m : meshes)
    if (p.mesh_canon[0] == m[0] && p.mesh_canon[1] == m[1] && p.mesh_canon[2] == m[2]) return true;
  return false;
}

// D = sum of the per-group partial sums (templated D step with several groups).
sox_status solid_dsum(const sox_plan& p, const double* Dp, double* D, hipStream_t s) {
  const int ng = solid_dgroups(p);
  if (!dstep_templated(p) || Dp == D) return SOX_OK;
  const long count = 2L * p.nk * p.N * p.N;
  hipLaunchKernelGGL(dsum_kernel, grid1d(count), dim3(256), 0, s, Dp, ng,
                     count, D, 0);
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}

template <typename TI, typename TO>
sox_status launch_ctranspose(const TI* in, TO* out, int rows, int cols, long batch,
                             hipStream_t s) {
  if (batch <= 0 || rows <= 0 || cols <= 0) return SOX_OK;
  if (batch > 65535) return fail(SOX_ERR_SHAPE, "internal: transpose batch too large");
  dim3 grid((cols + 31) / 32, (rows + 31) / 32, (unsigned)batch);
  hipLaunchKernelGGL((ctranspose_kernel<TI, TO>), grid, dim3(256), 0, s, in, out, rows, cols);
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}

// The solid U-contraction into ut [pair][a][P][b] (float64 arithmetic).
template <typename T>
sox_status launch_solid_utensor(const sox_plan& p, const double* U, const double* X, T* ut,
                                hipStream_t s) {
  const int n = p.n, N = p.N, np2 = p.nk * p.nk;
  const int* kOf = p.d_ktab;
  const int* qOf = p.d_ktab + np2;
  const int* kmqOf = p.d_ktab + 2 * np2;
  CgArgs<double, T> a = cg_args<double, T>();
  a.A = U; a.idxA = qOf; a.soA = (long)N * N; a.ldA = N;
  a.B = X; a.idxB = kOf; a.soB = (long)n * N; a.ldB = N;
  a.S = X; a.idxS = kmqOf; a.soS = (long)n * N; a.siS = N; a.conjS = 1;
  a.C = ut; a.soC = (long)n * N * n; a.siC = (long)N * n; a.ldc = n;
  a.nzi = n;
  a.M = N; a.N = n; a.K = N;
  return cg_launch(a, np2 * n, 0, s);
}

template <typename T>
sox_status run_solid(sox_plan& p, int entry, const double* X, const double* U1, const double* U2,
                     const double* G, double* Sigma, void* ws, hipStream_t s) {
  const int n = p.n, N = p.N, nt = p.n_tau, nk = p.nk, np2 = nk * nk, vcs = solid_vc(p, entry);
  const SolidLayout L = solid_layout_for(p, entry, vcs);
  char* base = (char*)ws;
  T* ut1 = (T*)(base + L.ut1);
  T* ut2 = (T*)(base + L.ut2);
  double* xtd = (double*)(base + L.xtd);
  double* gtd = (double*)(base + L.gtd);
  T* gtt = (T*)(base + L.gtt);
  T* grq = (T*)(base + L.grq);
  T* gwp = (T*)(base + L.gwp);
  T* abuf = (T*)(base + L.abuf);
  T* bbuf = (T*)(base + L.bbuf);
  T* cbuf = (T*)(base + L.cbuf);
  double* dbuf = (double*)(base + L.dbuf);
  double* dpart = (double*)(base + L.dpart);
  const int bcs = bc_shape(N);
  double* ebuf = (double*)(base + L.ebuf);
  const int* kOf = p.d_ktab;
  const int* kqOf = p.d_ktab + 2 * np2;  // index of k_v - q1 for pair (q1, k_v)
  sox_status st;
  {
    ProfScope ps(p, SOX_STAGE_UTENSOR, s);
    if ((st = launch_solid_utensor<T>(p, U1, X, ut1, s))) return st;
    if (entry != SOX_ENTRY_BARE && (st = launch_solid_utensor<T>(p, U2, X, ut2, s))) return st;
  }
  {
    ProfScope ps(p, SOX_STAGE_PROJECT, s);
    if ((st = launch_ctranspose<double, double>(X, xtd, n, N, nk, s))) return st;
    for (long b0 = 0; b0 < (long)nk * nt; b0 += 65535) {
      const long cnt = std::min(65535L, (long)nk * nt - b0);
      if ((st = launch_ctranspose<double, double>(G + 2 * b0 * n * n, gtd + 2 * b0 * n * n, n, n,
                                                  cnt, s)))
        return st;
    }
    const long cnt = 2L * nk * nt * n * n;
    hipLaunchKernelGGL((cast_kernel<T>), grid1d(cnt), dim3(256), 0, s,
                       gtd, gtt, cnt);
    SOX_HIP(hipGetLastError());
    // GRq[tau][k][R][q] and GwPt[tau][k][P][w] for every node
    CgArgs<double, T> a = cg_args<double, T>();
    a.A = xtd; a.soA = (long)N * n; a.ldA = n;
    a.B = gtd; a.soB = (long)nt * n * n; a.siB = (long)n * n; a.ldB = n;
    a.C = grq; a.soC = (long)N * n; a.siC = (long)nk * N * n; a.ldc = n;
    a.nzi = nt;
    a.M = N; a.N = n; a.K = n;
    if ((st = cg_launch(a, nk * nt, 0, s))) return st;
    a.conjA = 1;
    a.B = G;
    a.C = gwp;
    if ((st = cg_launch(a, nk * nt, 0, s))) return st;
  }
  for (int t = 0; t < nt; ++t) {
    const int tm = nt - 1 - t;
    {
      // A[pair][v][(P, q)] for every v: rows v of G^{k_v}(beta - tau)^T
      ProfScope ps(p, SOX_STAGE_ASTEP, s);
      CgArgs<T, T> a = cg_args<T, T>();
      a.A = gtt + 2 * (long)tm * n * n;
      a.idxA = kOf; a.soA = (long)nt * n * n; a.ldA = n;
      a.B = ut1; a.soB = (long)n * N * n; a.splitB = n; a.hiB = n; a.ldB = (long)N * n;
      a.C = abuf; a.soC = (long)n * N * n; a.ldc = (long)N * n;
      a.M = n; a.N = N * n; a.K = n;
      // 64 x 64 tiles of 2 x 2 wavefronts (3x3x3 mesh: 925 -> 844 ms per
      // bare step against 1 x 4 wavefronts of 64 x 16)
      if ((st = cg_launch(a, np2, 0, s))) return st;
    }
    for (int v0 = 0; v0 < n; v0 += vcs) {
      const int cnt = std::min(vcs, n - v0);
      {
        // B[pair][v] = A[pair][v0 + v] GRq^{k_v - q1}^T, the GRq panel shared by every v
        ProfScope ps(p, SOX_STAGE_KBC, s);
        CgArgs<T, T> b = cg_args<T, T>();
        b.A = abuf + 2 * (long)v0 * N * n; b.soA = (long)n * N * n; b.vsA = (long)N * n; b.ldA = n;
        b.B = grq + 2 * (long)t * nk * N * n; b.idxB = kqOf; b.soB = (long)N * n; b.ldB = n;
        b.C = bbuf; b.soC = (long)vcs * N * N; b.vsC = (long)N * N; b.ldc = N;
        b.nv = cnt;
        b.M = N; b.N = N; b.K = n;
        if ((st = bc_launch(b, np2, false, bcs, s, p.precision == SOX_BF16X3))) return st;
      }
      {
        // C[pair][v] = GwPt^{k_w} Ut2[pair][v0 + v]^T, the GwPt panel shared by every v
        ProfScope ps(p, SOX_STAGE_KBC, s);
        CgArgs<T, T> c = cg_args<T, T>();
        c.A = gwp + 2 * (long)t * nk * N * n; c.idxA = kOf; c.soA = (long)N * n; c.ldA = n;
        c.B = ut2 + 2 * (long)v0 * N * n; c.soB = (long)n * N * n; c.vsB = (long)N * n; c.ldB = n;
        c.C = cbuf; c.soC = (long)vcs * N * N; c.vsC = (long)N * N; c.ldc = N;
        c.nv = cnt;
        c.M = N; c.N = N; c.K = n;
        if ((st = bc_launch(c, np2, true, bcs, s, p.precision == SOX_BF16X3))) return st;
      }
      {
        ProfScope ps(p, SOX_STAGE_KD, s);
        if ((st = launch_dstep<T>(p, bbuf, cbuf, dbuf, dpart, (long)vcs * N * N, cnt, 1, 0, 0,
                                  true, v0 > 0, s)))
          return st;
      }
    }
    {
      ProfScope ps(p, SOX_STAGE_KD, s);
      if ((st = solid_dsum(p, dpart, dbuf, s))) return st;
    }
    {
      ProfScope ps(p, SOX_STAGE_BACK, s);
      CgArgs<double, double> e = cg_args<double, double>();
      e.A = X; e.soA = (long)n * N; e.ldA = N; e.conjA = 1;
      e.B = dbuf; e.soB = (long)N * N; e.ldB = N;
      e.C = ebuf; e.soC = (long)n * N; e.ldc = N;
      e.M = n; e.N = N; e.K = N;
      if ((st = cg_launch(e, nk, 0, s))) return st;
      CgArgs<double, double> f = cg_args<double, double>();
      f.A = ebuf; f.soA = (long)n * N; f.ldA = N;
      f.B = X; f.soB = (long)n * N; f.ldB = N;
      f.C = Sigma + 2 * (long)t * n * n; f.soC = (long)nt * n * n; f.ldc = n;
      f.alpha = -1.0 / nk;
      f.M = n; f.N = n; f.K = N;
      if ((st = cg_launch(f, nk, 0, s))) return st;
    }
  }
  return SOX_OK;
}

// G^k(tau) = -Q_k diag(n(eps_k, tau)) Q_k^dagger for every k and node.
sox_status solid_build_g(sox_plan& p, const double* Q, const double* eps, double mu, double* G,
                         hipStream_t s) {
  const int n = p.n, nt = p.n_tau, nk = p.nk;
  double* occ = p.d_scratch;                                  // [n_tau][n_k n]
  double* occc = occ + round_up((long)nt * nk * n, 2);        // complex copy, 16-byte aligned
  const long tot = (long)nt * nk * n;
  ProfScope ps(p, SOX_STAGE_GBUILD, s);
  hipLaunchKernelGGL(occupation_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, eps,
                     p.d_tau, mu, p.beta, nk * n, nt, occ);
  SOX_HIP(hipGetLastError());
  hipLaunchKernelGGL(real_to_complex_kernel, grid1d(tot), dim3(256), 0, s,
                     occ, occc, tot);
  SOX_HIP(hipGetLastError());
  CgArgs<double, double> a = cg_args<double, double>();
  a.A = Q; a.soA = (long)n * n; a.ldA = n;
  a.B = Q; a.soB = (long)n * n; a.ldB = n; a.conjB = 1;
  a.S = occc; a.soS = n; a.siS = (long)nk * n;
  a.C = G; a.soC = (long)nt * n * n; a.siC = (long)n * n; a.ldc = n;
  a.nzi = nt;
  a.alpha = -1.0;
  a.M = n; a.N = n; a.K = n;
  return cg_launch(a, nk * nt, 0, s);
}

// Queues the energy into e (device; null: the plan's scratch slot, returned
// in *slot).
sox_status solid_energy(sox_plan& p, const double* Sigma, const double* G, double* e,
                        double** slot, hipStream_t s) {
  const int n = p.n, nt = p.n_tau, nk = p.nk;
  double* tr = p.d_scratch + round_up((long)nt * nk * n, 2) + 2L * nt * nk * n;
  if (!e) e = tr + (size_t)nt * nk;
  if (slot) *slot = e;
  ProfScope ps(p, SOX_STAGE_ENERGY, s);
  hipLaunchKernelGGL(energy_trace_c_kernel, dim3(nt, nk), dim3(256), 0, s, Sigma, G, n, nt, tr);
  SOX_HIP(hipGetLastError());
  hipLaunchKernelGGL(energy_reduce_c_kernel, dim3(1), dim3(256), 0, s, tr, p.d_w, nt, nk, e);
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}

// -----------------------------------------------------------------------------
// Dynamic interaction on a k-point mesh (eq:GG for solids).
//
// Functions of imaginary time are complex here, so the plan's transform pair
// (made for real functions) is applied at +Omega_m with T_fwd and at -Omega_m
// with conj(T_fwd); the inverse transform is
// f(tau) = 1/2 sum_m [T_bwd f(+i Omega_m) + conj(T_bwd) f(-i Omega_m)], one
// product with the [n_tau][2 n_omega] matrix d_tbc.  The periodic convolution
// W^{q1} * GG becomes one W(Omega) GG(Omega) product per signed frequency.
//
// v runs outermost (the paper moves v to an outer loop for memory).  For
// each v: per slab of momentum pairs, GG(tau) -> FT -> W GG -> IFT gives
// A^{pair}(tau)[P][u] for every node; then per slab of tau nodes, B = A X,
// C = GwPt Ut2^v and the D step accumulate into D(tau) of every node.  The
// projections, GG and both transforms run in float64, W GG, B, C and D in the
// plan's precision; D and the back-transform in float64.
struct SolidDynLayout {
  size_t ut2, xtd, gtd, xtt, gwpd, grqtd, gwpt, wm, gg, ggw, aw, atau, bbuf, cbuf, dtau, ebuf;
  size_t gtm, gct, abare;  // bare line-1 term (ta > 0 only)
  size_t wblk, gblk;       // real block form of W(Omega) GG(Omega) (float plans, even n)
  size_t total;
};

// W(Omega) GG(Omega) as one real LDS-staged product per momentum transfer
// (float32 and bf16 x 3 plans): A rows [Re W | -Im W], B rows [Re GG | Im GG]
// and [Im GG | -Re GG] read from [Re | Im | -Re] rows, K = 2 Nq, interleaved
// complex float64 output (the column split 2n needs n even).
bool solid_wgg_block(const sox_plan& p) { return p.precision != SOX_FP64 && p.n % 2 == 0; }
int solid_nq(const sox_plan& p) { return (int)round_up(p.N, 16); }
// the forward transform with GG formed in registers, written in that block
// form (ft_solid_kernel): the transform matrix must fit its LDS
// The two transform kernels address their loads as a wavefront-uniform base
// plus a 32-bit lane offset: three frequency rows of a pair slab (inverse)
// or three nodes of the projections (forward) must stay below 2^32 bytes.
// Both need one momentum transfer's n_k n N columns within this bound, and
// the pair slab is capped to it.
constexpr long kTransformSlabCols = 1L << 26;
bool solid_ft_fused(const sox_plan& p) {
  return solid_wgg_block(p) && p.n_omega <= kFtsRows && p.n_tau <= kFtsLd - 1 &&
         (long)p.nk * p.n * p.N <= kTransformSlabCols;
}
// the inverse transform in real form on float32 MFMAs (ift_solid_kernel):
// W(Omega) GG(Omega) then writes its products in float32
bool solid_ift_real(const sox_plan& p) {
  return solid_wgg_block(p) && p.n_tau <= kIftRows && p.n_omega <= kIftWMax &&
         (long)p.nk * p.n * p.N <= kTransformSlabCols;
}

// workgroups of a persistent launch: as many as are resident at once
template <typename K>
unsigned resident_grid(const sox_plan& p, K kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1)
    nb = 1;
  return (unsigned)(nb * p.n_cu);
}

// ta > 0: the layout of the pass that also carries the bare line-1 term in
// tau slabs of ta nodes.
SolidDynLayout solid_dyn_layout_for(const sox_plan& p, int ps, int ts, int ta = 0) {
  SolidDynLayout L{};
  const size_t es = 2 * elem_size(p.precision);
  const size_t n = p.n, N = p.N, nt = p.n_tau, nk = p.nk, np2 = nk * nk, nw = p.n_omega;
  Carver c;
  L.ut2 = c.take(np2 * n * N * n * es);
  L.xtd = c.take(nk * N * n * 16);
  L.gtd = c.take(nk * nt * n * n * 16);
  L.xtt = c.take(nk * N * n * es);
  L.gwpd = c.take(nt * nk * n * N * 16);
  L.grqtd = c.take(nt * nk * n * N * 16);
  L.gwpt = c.take(nt * nk * N * n * es);
  L.wm = c.take(nk * 2 * nw * N * N * es);
  const bool fused_ft = solid_ft_fused(p);
  L.gg = fused_ft ? c.off : c.take(nt * (size_t)ps * n * N * 16);
  L.ggw = fused_ft ? c.off : c.take(2 * nw * (size_t)ps * n * N * es);
  L.aw = c.take(2 * nw * (size_t)ps * N * n * (solid_ift_real(p) ? 8 : 16));
  L.atau = c.take(nt * np2 * N * n * es);
  L.bbuf = c.take((size_t)ts * np2 * N * N * es);
  L.cbuf = c.take((size_t)ts * np2 * N * N * es);
  L.dtau = c.take(nt * nk * N * N * 16);
  L.ebuf = c.take(nt * nk * n * N * 16);
  if (ta > 0) {
    L.gtm = c.take(nk * n * nt * n * es);
    L.gct = c.take(nk * nt * n * n * es);
    L.abare = c.take((size_t)ta * np2 * N * n * es);
  }
  if (solid_wgg_block(p)) {
    // float, or bf16 hi and lo planes: 4 bytes per real value either way
    const size_t nq = solid_nq(p);
    L.wblk = c.take(nk * 2 * nw * N * 2 * nq * 4);
    L.gblk = c.take(2 * nw * (size_t)ps * n * 3 * nq * 4);
  }
  L.total = c.off;
  return L;
}

// Pair slab ps (whole momentum transfers q1, n_k pairs each) and tau slab
// ts within the budget: shrink the pair slab first (down to one transfer),
// then the tau slab.
void pick_solid_dyn(sox_plan& p) {
  const size_t budget = ws_budget();
  // the bare term's tau slab first: it is the row count of that term's
  // product, at most 64 nodes (one row tile), evened out over the slabs
  // (3x3x3 mesh: 25 rows instead of 50 took its two products 2.1 -> 2.8 s)
  const int slabs = (p.n_tau + 63) / 64;
  int ta = (p.n_tau + slabs - 1) / slabs;
  int nq = p.nk, ts = std::min(p.n_tau, 8);
  auto total = [&]() { return solid_dyn_layout_for(p, nq * p.nk, ts, ta).total; };
  while (nq > 1 && total() > budget) nq = (nq + 1) / 2;
  while (nq > 1 && (long)nq * p.nk * p.n * p.N > kTransformSlabCols) nq = (nq + 1) / 2;
  while (ts > 1 && total() > budget) ts = (ts + 1) / 2;
  while (ta > 1 && total() > budget) ta = (ta + 1) / 2;
  p.dyn_ps = nq * p.nk;
  p.dyn_ts = ts;
  p.dyn_ta = ta;
}

size_t solid_dyn_total(const sox_plan& p, bool with_bare) {
  return solid_dyn_layout_for(p, p.dyn_ps, p.dyn_ts, with_bare ? p.dyn_ta : 0).total;
}

// with_bare: Sigma = SOX(V + W_d(tau), V) = SOX(V, V) + SOX(W_d(tau), V) in one
// pass.  Both terms share line 2 (C), so by bilinearity they share the B, C
// and D steps: with G_Rq = X^T G the bare chain's B^v = A^v G_Rq^T equals
// (A^v G(tau)^T) X, so the bare A^v_Pq = sum_s Ut_Pqs G_sv(beta - tau)
// enters the dynamic A(tau) as A_bare G(tau)^T before the B step.
template <typename T>
sox_status run_solid_dynamic(sox_plan& p, const double* X, const double* W, const double* V,
                             const double* G, double* Sigma, void* ws, hipStream_t s,
                             bool with_bare = false) {
  const int n = p.n, N = p.N, nt = p.n_tau, nk = p.nk, np2 = nk * nk, nw = p.n_omega;
  const int ps = p.dyn_ps, ts = p.dyn_ts, ta = with_bare ? p.dyn_ta : 0;
  const SolidDynLayout L = solid_dyn_layout_for(p, ps, ts, ta);
  char* base = (char*)ws;
  T* ut2 = (T*)(base + L.ut2);
  double* xtd = (double*)(base + L.xtd);
  double* gtd = (double*)(base + L.gtd);
  T* xtt = (T*)(base + L.xtt);
  double* gwpd = (double*)(base + L.gwpd);
  double* grqtd = (double*)(base + L.grqtd);
  T* gwpt = (T*)(base + L.gwpt);
  T* wm = (T*)(base + L.wm);
  double* gg = (double*)(base + L.gg);
  T* ggw = (T*)(base + L.ggw);
  double* aw = (double*)(base + L.aw);
  T* atau = (T*)(base + L.atau);
  T* bbuf = (T*)(base + L.bbuf);
  T* cbuf = (T*)(base + L.cbuf);
  double* dtau = (double*)(base + L.dtau);
  double* ebuf = (double*)(base + L.ebuf);
  const bool blk = solid_wgg_block(p);
  const int Nq = solid_nq(p);
  const bool split = p.precision == SOX_BF16X3;
  T* gtm = ta ? (T*)(base + L.gtm) : nullptr;
  T* gct = ta ? (T*)(base + L.gct) : nullptr;
  T* abare = ta ? (T*)(base + L.abare) : nullptr;
  const int* kOf = p.d_ktab;
  const int* qOf = p.d_ktab + np2;
  const int* kmqOf = p.d_ktab + 2 * np2;
  const long nN = (long)n * N, NN = (long)N * N;
  sox_status st;
  {
    ProfScope ps_(p, SOX_STAGE_UTENSOR, s);
    if ((st = launch_solid_utensor<T>(p, V, X, ut2, s))) return st;
  }
  {
    ProfScope ps_(p, SOX_STAGE_PROJECT, s);
    if ((st = launch_ctranspose<double, double>(X, xtd, n, N, nk, s))) return st;
    for (long b0 = 0; b0 < (long)nk * nt; b0 += 65535) {
      const long cnt = std::min(65535L, (long)nk * nt - b0);
      if ((st = launch_ctranspose<double, double>(G + 2 * b0 * n * n, gtd + 2 * b0 * n * n, n, n,
                                                  cnt, s)))
        return st;
    }
    const long cx = 2L * nk * N * n;
    hipLaunchKernelGGL((cast_kernel<T>), grid1d(cx), dim3(256), 0, s, xtd,
                       xtt, cx);
    SOX_HIP(hipGetLastError());
    // GwP^k(tau)[w][P] = sum_p G^k_wp conj(X^k_pP) and GRqT^k(tau)[v][Q] =
    // sum_s G^k_sv X^k_sQ, the operands of GG: float64 products, stored in
    // float64, or in float32 for the forward transform that forms GG on
    // float32 MFMAs
    auto gg_operands = [&](auto* gw, auto* gr) -> sox_status {
      using TO = std::remove_pointer_t<decltype(gw)>;
      CgArgs<double, TO> a = cg_args<double, TO>();
      a.A = G; a.soA = (long)nt * n * n; a.siA = (long)n * n; a.ldA = n;
      a.B = xtd; a.soB = nN; a.ldB = n; a.conjB = 1;
      a.C = gw; a.soC = nN; a.siC = (long)nk * nN; a.ldc = N;
      a.nzi = nt;
      a.M = n; a.N = N; a.K = n;
      sox_status r;
      if ((r = cg_launch(a, nk * nt, 0, s))) return r;
      a = cg_args<double, TO>();
      a.A = gtd; a.soA = (long)nt * n * n; a.siA = (long)n * n; a.ldA = n;
      a.B = xtd; a.soB = nN; a.ldB = n;
      a.C = gr; a.soC = nN; a.siC = (long)nk * nN; a.ldc = N;
      a.nzi = nt;
      a.M = n; a.N = N; a.K = n;
      return cg_launch(a, nk * nt, 0, s);
    };
    if ((st = solid_ft_fused(p) ? gg_operands((float*)gwpd, (float*)grqtd)
                                : gg_operands(gwpd, grqtd)))
      return st;
    // GwPt^k(tau)[P][w] in the plan's precision (the C step)
    CgArgs<double, T> b = cg_args<double, T>();
    b.A = xtd; b.soA = nN; b.ldA = n; b.conjA = 1;
    b.B = G; b.soB = (long)nt * n * n; b.siB = (long)n * n; b.ldB = n;
    b.C = gwpt; b.soC = nN; b.siC = (long)nk * nN; b.ldc = n;
    b.nzi = nt;
    b.M = N; b.N = n; b.K = n;
    if ((st = cg_launch(b, nk * nt, 0, s))) return st;
    if (ta) {
      // the bare term's operands: G^k(beta - tau) by columns v, G^k(tau) in T
      const long cg = (long)nk * n * nt * n;
      hipLaunchKernelGGL((mirror_columns_kernel<T>), grid1d(cg), dim3(256), 0, s, G, gtm, nk, nt, n);
      SOX_HIP(hipGetLastError());
      hipLaunchKernelGGL((cast_kernel<T>), grid1d(2 * cg), dim3(256), 0, s, G, gct, 2 * cg);
      SOX_HIP(hipGetLastError());
    }
  }
  {
    // W^q(+-Omega)[P][Q] = sum_j [T_fwd; conj(T_fwd)][(+-, m)][j] W^q(tau_j)[P][Q]
    ProfScope ps_(p, SOX_STAGE_GG_FT, s);
    CgArgs<double, T> a = cg_args<double, T>();
    a.A = p.d_tfc; a.ldA = nt; a.soA = 0;
    a.B = W; a.soB = (long)nt * NN; a.ldB = 1; a.ksB = NN;
    a.C = wm; a.soC = 2L * nw * NN; a.ldc = NN;
    a.M = 2 * nw; a.N = (int)NN; a.K = nt;
    if ((st = cg_launch(a, nk, 4, s))) return st;
    if (blk) {
      // [Re W | -Im W] rows of every (q, +-Omega), float or bf16 hi / lo planes
      const long nb = (long)nk * 2 * nw;
      const long tot = nb * N * 2L * Nq;
      float* f = split ? nullptr : (float*)(base + L.wblk);
      bf16_t* hi = split ? (bf16_t*)(base + L.wblk) : nullptr;
      hipLaunchKernelGGL(wblock_kernel, grid1d(tot), dim3(256), 0, s, (const float*)wm, nb, N, Nq,
                         f, hi, hi ? hi + tot : nullptr);
      SOX_HIP(hipGetLastError());
    }
  }
  for (int v = 0; v < n; ++v) {
    for (int p0 = 0; p0 < np2; p0 += ps) {
      const int cp = std::min(ps, np2 - p0);
      const bool fft = solid_ft_fused(p);
      if (fft) {
        // GG formed in registers, transformed, stored in the W GG block form
        ProfScope ps_(p, SOX_STAGE_GG_FT, s);
        FtSolidArgs f{};
        f.tfc = p.d_tfc; f.gwp = (const float*)gwpd; f.grqt = (const float*)grqtd;
        f.kdiff = p.d_ktab + 3 * np2;
        const long gplane = 2L * nw * ps * n * 3L * Nq;
        if (split) {
          f.hi = (bf16_t*)(base + L.gblk);
          f.lo = f.hi + gplane;
        } else {
          f.f = (float*)(base + L.gblk);
        }
        f.rstride = (long)cp * n * 3 * Nq;
        f.nw = nw; f.nt = nt; f.nk = nk; f.n = n; f.N = N; f.Nq = Nq;
        f.p0 = p0; f.cp = cp; f.v = v;
        const long nblocks = (long)cp * n * (Nq / 16);
        switch ((nw + 15) / 16) {
#define SOX_FTS(R_)                                                                          \
  case R_:                                                                                   \
    hipLaunchKernelGGL(ft_solid_kernel<R_>, dim3(resident_grid(p, &ft_solid_kernel<R_>, 256)), \
                       dim3(256), 0, s, f, nblocks);                                         \
    break;
          SOX_FTS(1)
          SOX_FTS(2)
          SOX_FTS(3)
          SOX_FTS(4)
#undef SOX_FTS
          default: return fail(SOX_ERR_SHAPE, "internal: forward transform rows");
        }
        SOX_HIP(hipGetLastError());
      } else {
        ProfScope ps_(p, SOX_STAGE_GG_FT, s);
        const long tot = (long)nt * cp * nN;
        hipLaunchKernelGGL(gg_solid_kernel, grid1d(tot), dim3(256), 0, s,
                           gwpd, grqtd, kOf, kmqOf, gg, nt, nk, n, N, p0, cp, ps, v);
        SOX_HIP(hipGetLastError());
        CgArgs<double, T> a = cg_args<double, T>();
        a.A = p.d_tfc; a.ldA = nt;
        a.B = gg; a.ldB = 1; a.ksB = (long)ps * nN;
        a.C = ggw; a.ldc = (long)ps * nN;
        a.M = 2 * nw; a.N = (int)(cp * nN); a.K = nt;
        // 80 x 16 tiles (C5: 2.40 s -> 2.32 s against 80 x 32)
        if ((st = cg_launch(a, 1, 2, s))) return st;
      }
      if (blk) {
        // the same product in real block form on the LDS-staged GEMM: per
        // transfer q1, batched over +-Omega; columns j = 2 (l u) + re/im
        ProfScope ps_(p, SOX_STAGE_WGEMM, s);
        float* gf = split ? nullptr : (float*)(base + L.gblk);
        bf16_t* gh = split ? (bf16_t*)(base + L.gblk) : nullptr;
        const long gplane = 2L * nw * ps * n * 3L * Nq;  // lo plane offset (allocated extent)
        if (!fft) {
          const long gtot = 2L * nw * cp * n * 3L * Nq;
          hipLaunchKernelGGL(gblock_kernel, grid1d(gtot), dim3(256), 0, s, (const float*)ggw,
                             (long)2 * nw, (long)ps * nN, (long)cp * n, N, Nq, gf, gh,
                             gh ? gh + gplane : nullptr);
          SOX_HIP(hipGetLastError());
        }
        // gblock writes [r][cp n][3 Nq]: r stride cp n 3 Nq
        const long rstride = (long)cp * n * 3 * Nq;
        const long wb = (long)N * 2 * Nq;
        const bool f32out = solid_ift_real(p);
        for (int t = 0; t < cp / nk; ++t) {
          const int q1 = p0 / nk + t;
          double* C64 = f32out ? nullptr : aw + 2 * (long)t * nk * nN;
          float* C32 = f32out ? (float*)aw + 2 * (long)t * nk * nN : nullptr;
          if (split) {
            const bf16_t* wh = (const bf16_t*)(base + L.wblk);
            const bf16_t* wl = wh + (long)nk * 2 * nw * wb;
            DenseLdsSplitArgs l{};
            l.Ah = wh + (long)q1 * 2 * nw * wb; l.Al = wl + (long)q1 * 2 * nw * wb;
            l.Bh = gh + (long)t * nk * n * 3 * Nq; l.Bl = gh + gplane + (long)t * nk * n * 3 * Nq;
            l.C64 = C64; l.C = C32;
            l.lda = 2L * Nq; l.ldb = Nq; l.bsplit = 2; l.bhi = 3L * Nq;
            l.ldc = 2L * n; l.csplit = 2 * n; l.chi = 2 * nN;
            l.sA = wb; l.sB = rstride; l.sC = 2L * ps * nN;
            l.M = N; l.N = 2 * nk * n; l.K = 2 * Nq;
            SOX_HIP(launch_dense_lds_bf16x3<2>(l, 2 * nw, s));
          } else {
            const float* wf = (const float*)(base + L.wblk);
            DenseLdsArgs l{};
            l.A = wf + (long)q1 * 2 * nw * wb;
            l.B = gf + (long)t * nk * n * 3 * Nq;
            l.C64 = C64; l.C = C32;
            l.lda = 2L * Nq; l.ldb = Nq; l.bsplit = 2; l.bhi = 3L * Nq;
            l.ldc = 2L * n; l.csplit = 2 * n; l.chi = 2 * nN;
            l.c_gstride = 0; l.rgroup = N; l.rvalid = N;
            l.sA = wb; l.sB = rstride; l.sC = 2L * ps * nN;
            l.M = N; l.N = 2 * nk * n; l.K = 2 * Nq;
            SOX_HIP(launch_dense_lds_f32(l, 2 * nw, s));
          }
        }
      } else {
        // A(+-Omega)[l][P][u] = sum_Q W^{q1}(+-Omega)[P][Q] GG(+-Omega)[l][u][Q]: one
        // product per (+-Omega, q1) over the columns (k_v, u) of that transfer's n_k pairs
        ProfScope ps_(p, SOX_STAGE_WGEMM, s);
        CgArgs<T, double> a = cg_args<T, double>();
        a.A = wm + 2 * (long)(p0 / nk) * 2 * nw * NN; a.soA = 2L * nw * NN; a.siA = NN; a.ldA = N;
        a.B = ggw; a.soB = (long)nk * nN; a.siB = (long)ps * nN; a.ldB = N;
        a.C = aw; a.soC = (long)nk * nN; a.siC = (long)ps * nN; a.ldc = n;
        a.splitC = n; a.hiC = nN;
        a.nzi = 2 * nw;
        a.M = N; a.N = nk * n; a.K = N;
        // 64 x 64 tiles of four wavefronts (C5: 3.82 s -> 3.44 s against 80 x 64)
        if ((st = cg_launch(a, (cp / nk) * 2 * nw, 0, s))) return st;
      }
      if (solid_ift_real(p)) {
        // A(tau)[pair][P][u] from the float32 A(+-Omega_m)[l][P][u], real form
        ProfScope ps_(p, SOX_STAGE_IFT, s);
        IftSolidArgs f{};
        f.tbc = p.d_tbc; f.aw = (const float*)aw; f.out = (float*)(atau + 2 * (long)p0 * nN);
        f.fstride = (long)ps * nN; f.ldo = (long)np2 * nN; f.cols = (long)cp * nN;
        f.nt = nt; f.nw = nw;
        if (nw <= kIftW)
          hipLaunchKernelGGL(ift_solid_kernel<kIftW>,
                             dim3(resident_grid(p, &ift_solid_kernel<kIftW>, 256)), dim3(256), 0,
                             s, f);
        else
          hipLaunchKernelGGL(ift_solid_kernel<kIftWMax>,
                             dim3(resident_grid(p, &ift_solid_kernel<kIftWMax>, 256)), dim3(256),
                             0, s, f);
        SOX_HIP(hipGetLastError());
      } else {
        // A(tau)[pair][P][u] = sum_{+-m} Tb[tau][+-m] A(+-Omega_m)[l][P][u]
        ProfScope ps_(p, SOX_STAGE_IFT, s);
        CgArgs<double, T> a = cg_args<double, T>();
        a.A = p.d_tbc; a.ldA = 2 * nw;
        a.B = aw; a.ldB = 1; a.ksB = (long)ps * nN;
        a.C = atau + 2 * (long)p0 * nN; a.ldc = (long)np2 * nN;
        a.M = nt; a.N = (int)(cp * nN); a.K = 2 * nw;
        if ((st = cg_launch(a, 1, nt <= 112 ? 5 : 3, s))) return st;
      }
    }
    for (int a0 = 0; a0 < nt && ta; a0 += ta) {
      const int ca = std::min(ta, nt - a0);
      ProfScope ps_(p, SOX_STAGE_ASTEP, s);
      // A_bare[l][pair][q][P] = sum_s G^{k_v}(beta - tau_{a0+l})_sv Ut[pair][q][P][s]
      // (rows: the slab's nodes; columns (q, P), so that the U-tensor rows of
      // a column block are one contiguous block; Ut of V, the line-2 U-tensor).
      // On the panel kernels the nodes' rows are the staged panel (ca <= 64
      // rows) and the columns are streamed in nvb blocks per workgroup.
      int nvb = 8;
      while (nvb > 1 && nN % nvb) --nvb;
      CgArgs<T, T> a = cg_args<T, T>();
      a.A = gtm + 2 * ((long)v * nt + a0) * n;
      a.idxA = kOf; a.soA = (long)n * nt * n; a.ldA = n;
      a.B = ut2; a.soB = (long)n * N * n; a.ldB = n; a.vsB = nN / nvb * n;
      a.C = abare; a.soC = nN; a.ldc = (long)np2 * nN; a.vsC = nN / nvb;
      a.nv = nvb;
      a.M = ca; a.N = (int)(nN / nvb); a.K = n;
      if ((st = bc_launch(a, np2, true, 1, s, split))) return st;
      // A(tau)[pair][P][u] += sum_q A_bare[pair][q][P] G^{k_v - q1}(tau)[u][q]
      // (A rows P consecutive, k = q N apart)
      if constexpr (sizeof(T) == 4) {
        MergeArgs m{};
        m.ab = abare; m.ab_so = nN; m.ab_si = (long)np2 * nN;
        m.g = gct + 2 * (long)a0 * n * n; m.gidx = kmqOf; m.g_so = (long)nt * n * n;
        m.g_si = (long)n * n;
        m.a = atau + 2 * (long)a0 * np2 * nN; m.a_so = nN; m.a_si = (long)np2 * nN;
        m.nodes = ca; m.n = n; m.N = N;
        const hipError_t e = launch_merge_bare(m, np2, s);
        if (e == hipSuccess) continue;
        if (e != hipErrorNotSupported)
          return fail(SOX_ERR_HIP, "merge kernel launch failed: %s", hipGetErrorString(e));
      }
      CgArgs<T, T> b = cg_args<T, T>();
      b.A = abare; b.soA = nN; b.siA = (long)np2 * nN; b.ldA = 1; b.ksA = N;
      b.B = gct + 2 * (long)a0 * n * n; b.idxB = kmqOf; b.soB = (long)nt * n * n;
      b.siB = (long)n * n; b.ldB = n;
      b.C = atau + 2 * (long)a0 * np2 * nN; b.soC = nN; b.siC = (long)np2 * nN; b.ldc = n;
      b.accumulate = 1;
      b.nzi = ca;
      b.M = N; b.N = n; b.K = n;
      if ((st = cg_launch(b, np2 * ca, 0, s))) return st;
    }
    for (int t0 = 0; t0 < nt; t0 += ts) {
      const int ct = std::min(ts, nt - t0);
      {
        ProfScope ps_(p, SOX_STAGE_KBC, s);
        // B[l][pair][P][R] = sum_u A(tau)[pair][P][u] X^{k_v - q1}[u][R]; the X panel is
        // the same for every node l of the slab (the workgroup's inner loop)
        CgArgs<T, T> b = cg_args<T, T>();
        b.A = atau + 2 * (long)t0 * np2 * nN; b.soA = nN; b.vsA = (long)np2 * nN; b.ldA = n;
        b.B = xtt; b.idxB = kmqOf; b.soB = nN; b.ldB = n;
        b.C = bbuf; b.soC = NN; b.vsC = (long)np2 * NN; b.ldc = N;
        b.nv = ct;
        b.M = N; b.N = N; b.K = n;
        if ((st = bc_launch(b, np2, false, bc_shape(N), s, p.precision == SOX_BF16X3))) return st;
      }
      {
        ProfScope ps_(p, SOX_STAGE_KBC, s);
        // C[l][pair][P][R] = sum_w GwPt^{k_w}(tau)[P][w] Ut2[pair][v][R][w]; the Ut2^v panel
        // is the same for every node l of the slab
        CgArgs<T, T> c = cg_args<T, T>();
        c.A = gwpt + 2 * (long)t0 * nk * nN; c.idxA = kOf; c.soA = nN; c.vsA = (long)nk * nN;
        c.ldA = n;
        c.B = ut2 + 2 * (long)v * nN; c.soB = (long)n * nN; c.ldB = n;
        c.C = cbuf; c.soC = NN; c.vsC = (long)np2 * NN; c.ldc = N;
        c.nv = ct;
        c.M = N; c.N = N; c.K = n;
        if ((st = bc_launch(c, np2, false, bc_shape(N), s, p.precision == SOX_BF16X3))) return st;
      }
      {
        ProfScope ps_(p, SOX_STAGE_KD, s);
        if ((st = launch_dstep<T>(p, bbuf, cbuf, dtau + 2 * (long)t0 * nk * NN, nullptr, NN, 1,
                                  ct, (long)np2 * NN, (long)nk * NN, false, v > 0, s)))
          return st;
      }
    }
  }
  {
    ProfScope ps_(p, SOX_STAGE_BACK, s);
    CgArgs<double, double> e = cg_args<double, double>();
    e.A = X; e.soA = nN; e.ldA = N; e.conjA = 1;
    e.B = dtau; e.soB = NN; e.siB = (long)nk * NN; e.ldB = N;
    e.C = ebuf; e.soC = nN; e.siC = (long)nk * nN; e.ldc = N;
    e.nzi = nt;
    e.M = n; e.N = N; e.K = N;
    if ((st = cg_launch(e, nk * nt, 0, s))) return st;
    CgArgs<double, double> f = cg_args<double, double>();
    f.A = ebuf; f.soA = nN; f.siA = (long)nk * nN; f.ldA = N;
    f.B = X; f.soB = nN; f.ldB = N;
    f.C = Sigma; f.soC = (long)nt * n * n; f.siC = (long)n * n; f.ldc = n;
    f.nzi = nt;
    f.alpha = -1.0 / nk;
    f.M = n; f.N = n; f.K = N;
    if ((st = cg_launch(f, nk * nt, 0, s))) return st;
  }
  return SOX_OK;
}
