#include <hip/hip_runtime.h>
// Host bounds check of every entry point of libsox: the real sources are
// compiled for the CPU with a HIP shim under AddressSanitizer, each carved
// workspace buffer is followed by a poisoned guard gap, and every caller
// buffer is allocated to its exact size.
#include <vector>
#include <cstdio>
#include <string>
thread_local uint3e threadIdx, blockIdx, blockDim, gridDim;
const char* g_emu_kernel = "";
// workspace guard: every carved buffer is followed by a poisoned gap
static char* g_ws_base = nullptr;
static size_t g_ws_size = 0;
struct EmuCarver {
  size_t off = 0;
  EmuCarver() { if (g_ws_base) ASAN_UNPOISON_MEMORY_REGION(g_ws_base, g_ws_size); }
  size_t take(size_t bytes) {
    size_t o = off;
    size_t end = o + bytes;
    off = ((end + 4096) + 255) & ~size_t(255);
    if (g_ws_base && off <= g_ws_size) ASAN_POISON_MEMORY_REGION(g_ws_base + end, off - end);
    return o;
  }
};
#define Carver EmuCarver
#include "../../paper_2412_18829_amd/csrc/sox_api.hip"
#undef Carver

static double* dalloc(size_t n, double fill_scale = 0.1) {
  double* p = (double*)malloc(n * sizeof(double));
  for (size_t i = 0; i < n; ++i) p[i] = fill_scale * (((i * 2654435761u) % 1000) / 1000.0 - 0.5);
  return p;
}

int run_case(int n, int N, int nt, int prec, int entry, bool vjp, bool dyn) {
  std::vector<double> tau(nt), w(nt, 1.0);
  const double beta = 5.0;
  for (int k = 0; k < nt; ++k) tau[k] = beta * (k + 0.5) / nt;
  sox_problem pr{};
  pr.n_orb = n; pr.n_thc = N; pr.n_tau = nt; pr.kmesh[0] = pr.kmesh[1] = pr.kmesh[2] = 1;
  pr.beta = beta; pr.tau = tau.data(); pr.weights = w.data();
  int nw = 3;
  std::vector<double> tf(2 * nw * nt, 0.01), tb(2 * nw * nt, 0.01);
  if (dyn) { pr.n_omega = nw; pr.t_fwd = tf.data(); pr.t_bwd = tb.data(); }
  sox_plan* plan = nullptr;
  if (sox_plan_create(&pr, prec, &plan)) { printf("create failed: %s\n", sox_last_error()); return 1; }
  {
    char desc[2048];
    sox_plan_describe(plan, desc, sizeof(desc));
    printf("plan %s\n", desc);
  }
  size_t wsb = 0;
  const bool tune = getenv("EMU_AUTOTUNE") != nullptr && !vjp;
  if (tune) sox_autotune_workspace_size(plan, entry, 0, &wsb);
  else sox_workspace_size(plan, entry, &wsb);
  g_ws_size = wsb + 4096;
  g_ws_base = (char*)aligned_alloc(256, (g_ws_size + 255) & ~size_t(255));
  double* X = dalloc((size_t)n * N);
  double* U1 = dalloc((size_t)N * N * (entry == 2 || entry == 4 ? nt : 1));
  double* U2 = dalloc((size_t)N * N);
  double* G = dalloc((size_t)nt * n * n);
  double* S = dalloc((size_t)nt * n * n);
  double* R = dalloc((size_t)nt * n * n);
  double* dG = dalloc((size_t)nt * n * n);
  double* dX = dalloc((size_t)n * N);
  double* dU1 = dalloc((size_t)N * N * (entry == 2 ? nt : 1));
  double* dU2 = dalloc((size_t)N * N);
  sox_status st;
  if (tune) {
    st = sox_autotune(plan, entry, 0, X, U1, entry == 0 ? nullptr : U2, G, S, g_ws_base, wsb, nullptr);
    char desc[8192];
    sox_plan_describe(plan, desc, sizeof(desc));
    printf("tuned %s (status %d %s)\n", desc, st, st ? sox_last_error() : "");
    if (st) return st;
  }
  if (!vjp) {
    if (entry == 0) st = sox_sigma_bare(plan, X, U1, G, S, g_ws_base, wsb, nullptr);
    else if (entry == 1) st = sox_sigma_static(plan, X, U1, U2, G, S, g_ws_base, wsb, nullptr);
    else if (entry == 4) st = sox_sigma_gw(plan, X, U1, G, S, g_ws_base, wsb, nullptr);
    else st = sox_sigma_dynamic(plan, X, U1, U2, G, S, g_ws_base, wsb, nullptr);
  } else {
    st = sox_sigma_vjp(plan, entry, X, U1, entry == 0 ? nullptr : U2, G, R, dG, dX, dU1,
                       entry == 0 ? nullptr : dU2, g_ws_base, wsb, nullptr);
  }
  printf("case n=%d N=%d nt=%d prec=%d entry=%d vjp=%d -> status %d %s\n", n, N, nt, prec, entry, vjp, st, st ? sox_last_error() : "");
  ASAN_UNPOISON_MEMORY_REGION(g_ws_base, g_ws_size);
  g_ws_base = nullptr;
  sox_plan_destroy(plan);
  return st;
}

// k-point plans: complex128 buffers of their exact sizes; G is built on the
// mesh, then the bare, static or dynamic entry (0, 1, 2), the vertex entry
// with kind entry - 3 (3 .. 7) or the GW entry (8), and the energy run.
int run_solid_case(int n, int N, int nt, int prec, int entry, const int mesh[3]) {
  const int nk = mesh[0] * mesh[1] * mesh[2];
  std::vector<double> tau(nt), w(nt, 1.0);
  const double beta = 5.0;
  for (int k = 0; k < nt; ++k) tau[k] = beta * (k + 0.5) / nt;
  sox_problem pr{};
  pr.n_orb = n; pr.n_thc = N; pr.n_tau = nt;
  for (int i = 0; i < 3; ++i) pr.kmesh[i] = mesh[i];
  pr.beta = beta; pr.tau = tau.data(); pr.weights = w.data();
  const int nw = getenv("EMU_NW") ? atoi(getenv("EMU_NW")) : 3;
  const bool dyn = entry == 2 || entry >= 3 + SOX_VERTEX_SOSEX_DYN;
  std::vector<double> tf(2 * nw * nt, 0.01), tb(2 * nw * nt, 0.01);
  if (dyn) { pr.n_omega = nw; pr.t_fwd = tf.data(); pr.t_bwd = tb.data(); }
  sox_plan* plan = nullptr;
  if (sox_plan_create(&pr, prec, &plan)) { printf("create failed: %s\n", sox_last_error()); return 1; }
  size_t wsb = 0;
  const bool tune = getenv("EMU_AUTOTUNE") != nullptr;
  const bool gw = entry == 8;
  const int ent = gw ? SOX_ENTRY_GW : entry >= 3 ? SOX_ENTRY_VERTEX : entry;
  const int kind = !gw && entry >= 3 ? entry - 3 : 0;
  if (tune) sox_autotune_workspace_size(plan, ent, kind, &wsb);
  else sox_workspace_size(plan, ent, &wsb);
  g_ws_size = wsb + 4096;
  g_ws_base = (char*)aligned_alloc(256, (g_ws_size + 255) & ~size_t(255));
  double* X = dalloc(2 * (size_t)nk * n * N);
  double* U1 = dalloc(2 * (size_t)nk * N * N * (dyn ? nt : 1));
  double* U2 = dalloc(2 * (size_t)nk * N * N);
  double* Q = dalloc(2 * (size_t)nk * n * n);
  double* eps = dalloc((size_t)nk * n, 3.0);
  double* G = dalloc(2 * (size_t)nk * nt * n * n);
  double* S = dalloc(2 * (size_t)nk * nt * n * n);
  sox_status st = sox_build_g_tau(plan, Q, eps, 0.0, G, nullptr);
  if (!st && tune) {
    const double* u1 = ent == SOX_ENTRY_VERTEX ? U2 : U1;
    const double* u2 = ent == SOX_ENTRY_VERTEX ? U1 : (entry == 0 ? nullptr : U2);
    st = sox_autotune(plan, ent, kind, X, u1, u2, G, S, g_ws_base, wsb, nullptr);
    char desc[8192];
    sox_plan_describe(plan, desc, sizeof(desc));
    printf("tuned %s (status %d %s)\n", desc, st, st ? sox_last_error() : "");
  }
  if (!st) {
    if (entry == 0) st = sox_sigma_bare(plan, X, U1, G, S, g_ws_base, wsb, nullptr);
    else if (entry == 1) st = sox_sigma_static(plan, X, U1, U2, G, S, g_ws_base, wsb, nullptr);
    else if (entry == 2) st = sox_sigma_dynamic(plan, X, U1, U2, G, S, g_ws_base, wsb, nullptr);
    else if (gw) st = sox_sigma_gw(plan, X, U1, G, S, g_ws_base, wsb, nullptr);
    else st = sox_sigma_vertex(plan, entry - 3, X, U2, U1, G, S, g_ws_base, wsb, nullptr);
  }
  double E = 0.0;
  if (!st) st = sox_energy_gm(plan, S, G, &E, nullptr);
  char desc[1024];
  sox_plan_describe(plan, desc, sizeof(desc));
  printf("plan %s\n", desc);
  printf("case n=%d N=%d nt=%d prec=%d entry=%d mesh=%dx%dx%d -> status %d %s\n", n, N, nt, prec,
         entry, mesh[0], mesh[1], mesh[2], st, st ? sox_last_error() : "");
  ASAN_UNPOISON_MEMORY_REGION(g_ws_base, g_ws_size);
  g_ws_base = nullptr;
  sox_plan_destroy(plan);
  return st;
}

// Every tiled launcher refuses a grid whose x extent reaches 2^32
// work-items (the 32-bit field of a dispatch packet) with hipErrorInvalidValue
// and launches nothing (a launch would abort in the shim above).  The
// arguments are otherwise valid, the pointers never dereferenced.
int run_guards() {
  using namespace sox;
  static float fdummy[64];
  static double ddummy[64];
  static bf16_t bdummy[64];
  int bad = 0;
  auto expect = [&](const char* what, hipError_t e) {
    printf("guard %-28s -> %s\n", what, e == hipErrorInvalidValue ? "refused" : "LAUNCHED");
    if (e != hipErrorInvalidValue) ++bad;
  };
  {
    HcArgs<float, double> a{};
    a.nz = 32; a.nk = 16; a.ny = 64; a.n_ot = 1 << 12; a.n_ov = 1 << 12;
    a.L = a.Rm = a.W = a.FT = fdummy; a.Out = ddummy;
    expect("hc_kernel", launch_hc<float, double, 1, 4>(a, 64 * 1024, nullptr));
  }
  {
    LdsFusedArgs a{};
    a.nP = 16; a.NP = 128; a.tiles_p = a.tiles_r = 1; a.n_tau = 1 << 23; a.vsplit = 1; a.vchunk = 1;
    a.u_rstride = 256; a.D = fdummy;
    expect("fused_bcd_lds_kernel", launch_fused_lds<kLdsFp32, kFp32LdsPB>(a, nullptr));
  }
  {
    DenseLdsArgs a{};
    a.A = a.B = fdummy; a.C = fdummy; a.M = a.N = 1 << 22; a.K = 16; a.rgroup = 1; a.rvalid = 1;
    a.lda = a.ldb = 16; a.ldc = 1 << 22;
    expect("dense_lds_f32_kernel", launch_dense_lds_f32(a, 1, nullptr));
  }
  {
    DenseLdsSplitArgs a{};
    a.Ah = a.Al = a.Bh = a.Bl = bdummy; a.C = fdummy; a.M = a.N = 1 << 22; a.K = 32;
    a.lda = a.ldb = 32; a.ldc = 1 << 22;
    expect("dense_lds_bf16x3_kernel", launch_dense_lds_bf16x3<2>(a, 1, nullptr));
  }
  {
    CgArgs<float, float> a = cg_args<float, float>();
    a.A = a.B = fdummy; a.C = fdummy; a.M = a.N = 1 << 22; a.K = 16; a.ldA = a.ldB = 16;
    a.ldc = 1 << 22;
    expect("cgemm_nt_kernel", launch_cgemm<float, float, 2, 2, 2, 2>(a, 1, nullptr));
    expect("cgemm_panel_kernel", launch_cgemm_panel(a, 1, true, nullptr));
  }
  {
    DenseArgs<double, double> a{};
    a.A = a.B = ddummy; a.C = ddummy; a.M = a.N = 1 << 22; a.K = 16;
    expect("dense_nt_kernel", launch_dense<double, double, 1, 4, 2, 2>(a, 1, nullptr));
  }
  {
    FusedArgs<float> a{};
    a.tiles_p = a.tiles_r = 1 << 12; a.n_tau = 1 << 12; a.vsplit = 1;
    expect("fused_bcd_kernel", launch_fused<float, 32, 32>(a, nullptr));
  }
  printf("guards: %d launched\n", bad);
  return bad;
}

// The no-allocation bare entry on the static scratch array: a plan whose
// bare workspace exceeds the array is refused, then two calls in a row (the
// second on a smaller problem) run inside the array's bounds.
int run_noalloc(int prec) {
  const int shapes[3][3] = {{64, 384, 64}, {13, 70, 5}, {6, 20, 3}};
  int rc = 0;
  for (int c = 0; c < 3; ++c) {
    const int n = shapes[c][0], N = shapes[c][1], nt = shapes[c][2];
    std::vector<double> tau(nt), w(nt, 1.0);
    for (int k = 0; k < nt; ++k) tau[k] = 5.0 * (k + 0.5) / nt;
    sox_problem pr{};
    pr.n_orb = n; pr.n_thc = N; pr.n_tau = nt; pr.kmesh[0] = pr.kmesh[1] = pr.kmesh[2] = 1;
    pr.beta = 5.0; pr.tau = tau.data(); pr.weights = w.data();
    sox_plan* plan = nullptr;
    if (sox_plan_create(&pr, prec, &plan)) { printf("create failed: %s\n", sox_last_error()); return 1; }
    size_t wsb = 0;
    sox_workspace_size(plan, SOX_ENTRY_BARE, &wsb);
    double* X = dalloc((size_t)n * N);
    double* V = dalloc((size_t)N * N);
    double* G = dalloc((size_t)nt * n * n);
    double* S = dalloc((size_t)nt * n * n);
    const sox_status st = sox_sigma_bare_noalloc(plan, X, V, G, S, nullptr);
    const sox_status want = wsb > kNoallocScratchBytes ? SOX_ERR_WORKSPACE : SOX_OK;
    printf("noalloc n=%d N=%d nt=%d prec=%d ws=%zu -> status %d (want %d) %s\n", n, N, nt, prec,
           wsb, st, want, st ? sox_last_error() : "");
    if (st != want) rc = 1;
    free(X); free(V); free(G); free(S);
    sox_plan_destroy(plan);
  }
  printf("noalloc %s\n", rc ? "FAILED" : "ok");
  return rc;
}

// The self-consistent loop (sox_scf) on a small molecule: two iterations
// with every kernel of the loop, the GW chain (bit 0) and the bare SOX
// entry (bit 1); transform values are arbitrary (only accesses matter).
int run_scf_case(int n, int N, int nt, int nnu, int terms, int prec) {
  std::vector<double> tau(nt), w(nt, 1.0);
  const double beta = 5.0;
  for (int k = 0; k < nt; ++k) tau[k] = beta * (k + 0.5) / nt;
  sox_problem pr{};
  pr.n_orb = n; pr.n_thc = N; pr.n_tau = nt; pr.kmesh[0] = pr.kmesh[1] = pr.kmesh[2] = 1;
  pr.beta = beta; pr.tau = tau.data(); pr.weights = w.data();
  sox_plan* plan = nullptr;
  if (sox_plan_create(&pr, prec, &plan)) { printf("create failed: %s\n", sox_last_error()); return 1; }
  std::vector<double> nu(nnu), tf(2 * (size_t)nnu * nt, 0.01), tb(2 * (size_t)nt * nnu, 0.01),
      tbeta(nt, -0.1);
  for (int q = 0; q < nnu; ++q) nu[q] = (2 * q + 1) * M_PI / beta;
  sox_scf_params prm{};
  prm.n_elec = 0.5 * n; prm.mix = 0.5; prm.tol = 1e-30; prm.max_iter = 2; prm.terms = terms;
  prm.n_nu = nnu; prm.nu = nu.data(); prm.t_fwd = tf.data(); prm.t_bwd = tb.data();
  prm.t_beta = tbeta.data();
  size_t wsb = 0;
  sox_scf_workspace_size(plan, nnu, terms, &wsb);
  g_ws_size = wsb + 4096;
  g_ws_base = (char*)aligned_alloc(256, (g_ws_size + 255) & ~size_t(255));
  double* X = dalloc((size_t)n * N);
  double* V = dalloc((size_t)N * N);
  double* W = dalloc((size_t)nt * N * N);
  double* h = dalloc((size_t)n * n, 3.0);
  double* G = dalloc((size_t)nt * n * n);
  sox_scf_result res{};
  const sox_status st = sox_scf(plan, &prm, X, V, (terms & 1) ? W : nullptr, h, nullptr, G, &res,
                                g_ws_base, wsb, nullptr);
  printf("scf n=%d N=%d nt=%d nnu=%d terms=%d -> status %d %s\n", n, N, nt, nnu, terms, st,
         st ? sox_last_error() : "");
  ASAN_UNPOISON_MEMORY_REGION(g_ws_base, g_ws_size);
  g_ws_base = nullptr;
  free(X); free(V); free(W); free(h); free(G);
  sox_plan_destroy(plan);
  return st;
}

int main(int argc, char** argv) {
  if (argc == 8 && std::string(argv[1]) == "scf")
    return run_scf_case(atoi(argv[2]), atoi(argv[3]), atoi(argv[4]), atoi(argv[5]), atoi(argv[6]),
                        atoi(argv[7]));
  if (argc == 2 && std::string(argv[1]) == "guards") return run_guards();
  if (argc == 3 && std::string(argv[1]) == "noalloc") return run_noalloc(atoi(argv[2]));
  int n = atoi(argv[1]), N = atoi(argv[2]), nt = atoi(argv[3]), prec = atoi(argv[4]), entry = atoi(argv[5]), vjp = atoi(argv[6]);
  if (argc >= 10) {
    const int mesh[3] = {atoi(argv[7]), atoi(argv[8]), atoi(argv[9])};
    return run_solid_case(n, N, nt, prec, entry, mesh);
  }
  return run_case(n, N, nt, prec, entry, vjp, entry == 2);
}
