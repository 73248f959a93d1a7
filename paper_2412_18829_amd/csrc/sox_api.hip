// C ABI of the SOX library: plan, validation, workspace carving and the
// launch sequence of each entry point.  Declarations and argument contracts
// are in include/sox.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/sox.h"
#include "sox_common.hpp"
#include "sox_dense.hpp"
#include "sox_fused.hpp"
#include "sox_gemm.hpp"
#include "sox_steps.hpp"
#include "sox_adjoint.hpp"
#include "sox_bf16.hpp"
#include "sox_fused_lds.hpp"
#include "sox_dense_lds.hpp"
#include "sox_vjp_steps.hpp"
#include "sox_complex.hpp"
#include "sox_gw.hpp"
#include "sox_ir.hpp"
#include "sox_scf.hpp"

using namespace sox;

namespace {

thread_local std::string g_last_error;

sox_status fail(sox_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define SOX_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(SOX_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),   \
                  __FILE__, __LINE__);                                                  \
  } while (0)

inline long round_up(long x, long m) { return (x + m - 1) / m * m; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Wave-tile shapes of the fused B, C -> D kernel (P rows x R columns per
// wavefront; a workgroup is 2 x 2 wavefronts).
struct FusedCfg {
  int wp, wr;
  bool fp32, fp64, bf16;
};
static const FusedCfg kFusedCfgs[] = {
    {32, 32, true, true, false},   // 0
    {64, 32, true, false, false},  // 1
    {32, 64, true, false, false},  // 2
    {64, 64, true, false, false},  // 3
    {32, 16, true, true, false},   // 4
    {16, 32, false, true, false},  // 5
    {32, 32, false, false, true},  // 6  bf16 x 3
    {64, 32, false, false, true},  // 7  bf16 x 3
    {64, 64, false, false, true},  // 8  bf16 x 3, LDS-staged 128 x 128 workgroup tile
    {64, 64, true, false, false},  // 9  float32, LDS-staged 128 x 128 workgroup tile
};
static const int kNumFusedCfgs = sizeof(kFusedCfgs) / sizeof(kFusedCfgs[0]);

// 16-row P blocks per wavefront of the LDS-staged fused kernels (configs 8
// and 9): 4 = four wavefronts of 64 x 64, 2 = eight of 32 x 64, two per
// SIMD.  Eight against four, per sweep: split precision n=64 N=384 0.533
// -> 0.508 ms, n=200 N=1200 88.4 -> 85.4 ms, dynamic n=300 N=1800 529 ->
// 489 ms; float32 n=64 N=384 1.307 -> 1.225 ms, n=200 N=1200 207 -> 198 ms.
constexpr int kBf16LdsPB = 2;
constexpr int kFp32LdsPB = 2;

struct sox_plan {
  int n, N, n_tau;
  int nP, NP;
  int precision;
  int fused_cfg;   // index into kFusedCfgs
  int fused_vsplit = 1;  // workgroups sharing one D tile's v sum (static entries)
  int n_cu = 256;        // compute units of the device
  long dense_wg = 512;   // short-K LDS-staged GEMM: workgroups in the grid at most
  int wg_tile;     // NP granule: 2 * max(wave tile edges)
  int slab;        // tau nodes per slab
  double beta;
  std::vector<double> tau, weights;
  int n_omega;
  std::vector<double> t_fwd, t_bwd;  // complex interleaved (host copies)
  int vjp_slab = 1; // tau nodes per slab of the adjoint chain
  int vc = 0;       // dynamic entry: v-slab width
  int vc_vjp = 0;   // dynamic entry: v-slab width of the adjoint
  int eslab = 0;    // dynamic entry: tau nodes per back-transform slab
  // k-point meshes (nk > 1): mesh with unit dimensions moved last, v-slab
  // width of the solid chain and the device momentum tables
  int kmesh[3] = {1, 1, 1};
  int mesh_canon[3] = {1, 1, 1};
  int nk = 1;
  int vcs = 0;       // statically screened entry
  int vcs_bare = 0;  // bare entry (one U-tensor: wider slabs fit)
  int dyn_ps = 0;    // dynamic entry: momentum pairs per slab
  int dyn_ts = 0;    // dynamic entry: tau nodes per B, C, D slab
  int dyn_ta = 0;    // bare + dynamic pass: tau nodes per slab of the bare A term
  int* d_ktab = nullptr;
  double* d_tfc = nullptr;  // [2 n_omega][n_tau] complex [T_fwd; conj(T_fwd)]
  double* d_tbc = nullptr;  // [n_tau][2 n_omega] complex [T_bwd / 2 | conj(T_bwd) / 2]
  // device copies
  double* d_tf2 = nullptr;  // [2 n_omega][n_tau]  Re / Im of t_fwd
  double* d_tb2 = nullptr;  // [n_tau][2 n_omega]  [Re t_bwd | -Im t_bwd]
  double* d_tau = nullptr;
  double* d_w = nullptr;
  double* d_scratch = nullptr;  // occupations / traces / energy: n_tau*(n+1)+1
  double* d_wchk = nullptr;     // molecular dynamic plans: mirror-symmetry partial maxima
  int last_w_real = -1;         // molecular dynamic entry: 1 if the last call ran the real W product
  int device = 0;
  // per-stage event timing (sox_profile_enable / sox_profile_read)
  struct Ev {
    hipEvent_t a, b;
    int stage;
  };
  // whole-sweep HIP graphs keyed by the call's pointers
  struct GraphEntry {
    uintptr_t key[9];
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  bool graph_on = false;
  hipStream_t cap_stream = nullptr;
  std::vector<GraphEntry> graphs;
  // fused-tile autotuner results: (config, ms per tau)
  std::vector<std::pair<int, double>> tune_ms;
  bool tune_from_cache = false;
  // sox_autotune: every candidate's launch choices and its ms per call
  struct TuneResult {
    int fused_cfg, fused_vsplit, dyn_ts, dyn_ps, vcs, vcs_bare;
    double ms;
  };
  std::vector<TuneResult> autotune;
  int autotune_cached = 0;  // 1: the choices came from the tune cache
  bool prof_on = false;
  uint32_t prof_mask = 0xFFFFFFFFu;  // stages recorded while profiling is on
  std::vector<Ev> ev_pool;
  size_t ev_used = 0;
  int64_t ev_dropped = 0;
  static constexpr size_t kMaxEvents = 65536;

  int prof_begin(int stage, hipStream_t s) {
    if (!prof_on || !((prof_mask >> stage) & 1u)) return -1;
    if (ev_used >= kMaxEvents) {
      ++ev_dropped;
      return -1;
    }
    if (ev_used == ev_pool.size()) {
      Ev e{};
      if (hipEventCreate(&e.a) != hipSuccess) return -1;
      if (hipEventCreate(&e.b) != hipSuccess) {
        (void)hipEventDestroy(e.a);
        return -1;
      }
      ev_pool.push_back(e);
    }
    Ev& e = ev_pool[ev_used];
    e.stage = stage;
    if (hipEventRecord(e.a, s) != hipSuccess) return -1;
    return (int)ev_used++;
  }
  void prof_end(int idx, hipStream_t s) {
    if (idx >= 0) (void)hipEventRecord(ev_pool[idx].b, s);
  }
};

namespace {
// Brackets the launches of one stage with events when profiling is on.
struct ProfScope {
  sox_plan& p;
  hipStream_t s;
  int idx;
  ProfScope(sox_plan& plan, int stage, hipStream_t stream) : p(plan), s(stream) {
    idx = p.prof_begin(stage, s);
  }
  ~ProfScope() { p.prof_end(idx, s); }
};
}  // namespace

namespace {

// -- workspace layout --------------------------------------------------------
struct Layout {
  size_t u1, u2, a, p1, p2t, d, e, gbt, ukr, xp, d64;
  size_t ah, al, p1h, p1l, p2h, p2l, u2h, u2l;  // bf16 x 3 split operands
  size_t total;
};

struct DynLayout {
  size_t p1d, p2td, p1q, p2q, p2t, xt, u2, w2, gg2, aw, adyn, d, e, ukr, xp, d64, total;
  size_t xth, xtl, p2h, p2l, u2h, u2l;  // bf16 x 3 split operands of the fused contraction
  size_t w2h, w2l;                      // bf16 x 3 split W(Omega)
};

size_t elem_size(int precision) { return precision == SOX_FP64 ? 8 : 4; }

// float32 scratch of the U-contraction on the LDS-staged GEMM (the
// Khatri-Rao factor and the padded interaction); none in float64 plans
// K splits of the float32 U-contraction: doubled while the output tiles
// alone give fewer than two workgroups per CU (small molecules), each split
// a multiple of 16 deep
int utensor_ksplit(const sox_plan& p) {
  const long tiles = (long)((p.NP + kLdsTile - 1) / kLdsTile) *
                     (((long)p.nP * p.nP + kLdsTile - 1) / kLdsTile);
  int ks = 1;
  while (ks < 4 && tiles * ks < 2L * p.n_cu && p.NP % (32 * ks) == 0) ks *= 2;
  return ks;
}

size_t utensor_scratch_bytes(const sox_plan& p) {
  if (p.precision == SOX_FP64) return 0;
  const int ks = utensor_ksplit(p);
  return ((size_t)p.nP * p.nP * p.NP + (size_t)p.NP * p.NP +
          (ks > 1 ? (size_t)ks * p.NP * p.nP * p.nP : 0)) * 4;
}


struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  }
};

Layout layout_for(const sox_plan& p, int entry, int slab) {
  Layout L{};
  const size_t es = elem_size(p.precision);
  const size_t nP = p.nP, NP = p.NP, n = p.n;
  Carver c;
  L.u1 = c.take(NP * nP * nP * es);
  L.u2 = (entry == SOX_ENTRY_BARE) ? L.u1 : c.take(NP * nP * nP * es);
  // split precision keeps A only as its bf16 hi and lo planes (written by the A step)
  L.a = c.take(p.precision == SOX_BF16X3 ? 0 : (size_t)slab * n * NP * nP * es);
  L.p1 = c.take((size_t)slab * NP * nP * es);
  L.p2t = c.take((size_t)slab * NP * nP * es);
  L.d = c.take((size_t)slab * NP * NP * es * std::max(1, p.fused_vsplit));
  L.e = c.take((size_t)slab * n * NP * 8);
  L.gbt = c.take((size_t)slab * nP * nP * es);
  L.ukr = c.take(utensor_scratch_bytes(p));
  L.xp = c.take((size_t)n * NP * 8);
  L.d64 = c.take(p.precision == SOX_FP64 ? 0 : (size_t)slab * NP * NP * 8);
  if (p.precision == SOX_BF16X3) {
    const size_t na = (size_t)slab * n * NP * nP, np1 = (size_t)slab * NP * nP, nu = NP * nP * nP;
    L.ah = c.take(na * 2); L.al = c.take(na * 2);
    L.p1h = c.take(np1 * 2); L.p1l = c.take(np1 * 2);
    L.p2h = c.take(np1 * 2); L.p2l = c.take(np1 * 2);
    L.u2h = c.take(nu * 2); L.u2l = c.take(nu * 2);
  }
  L.total = c.off;
  return L;
}

DynLayout dyn_layout_for(const sox_plan& p, int vc, int eslab) {
  DynLayout L{};
  const size_t es = elem_size(p.precision);
  const size_t nP = p.nP, NP = p.NP, n = p.n, nt = p.n_tau, nw = p.n_omega;
  Carver c;
  L.p1d = c.take(nt * NP * nP * 8);
  L.p2td = c.take(nt * NP * nP * 8);
  L.p1q = c.take(nt * NP * nP * 8);
  L.p2q = c.take(nt * NP * nP * 8);
  L.p2t = c.take(nt * NP * nP * es);
  L.xt = c.take(NP * nP * es);
  L.u2 = c.take(NP * nP * nP * es);
  L.w2 = c.take(nw * 4 * NP * NP * es);
  L.gg2 = c.take(nw * (size_t)vc * n * 2 * NP * es);
  L.aw = c.take(nw * 2 * NP * (size_t)vc * n * es);
  L.adyn = c.take(nt * (size_t)vc * NP * nP * es);
  L.d = c.take(nt * NP * NP * es);
  L.e = c.take((size_t)eslab * n * NP * 8);
  L.ukr = c.take(utensor_scratch_bytes(p));
  L.xp = c.take((size_t)n * NP * 8);
  L.d64 = c.take(p.precision == SOX_FP64 ? 0 : (size_t)eslab * NP * NP * 8);
  if (p.precision == SOX_BF16X3) {
    L.xth = c.take(NP * nP * 2); L.xtl = c.take(NP * nP * 2);
    L.p2h = c.take(nt * NP * nP * 2); L.p2l = c.take(nt * NP * nP * 2);
    L.u2h = c.take(NP * nP * nP * 2); L.u2l = c.take(NP * nP * nP * 2);
    L.w2h = c.take(nw * 4 * NP * NP * 2); L.w2l = c.take(nw * 4 * NP * NP * 2);
  }
  L.total = c.off;
  return L;
}

size_t ws_budget() {
  double budget_mb = 65536.0;
  if (const char* s = getenv("SOX_WS_BUDGET_MB")) {
    double v = atof(s);
    if (v > 0) budget_mb = v;
  }
  return (size_t)(budget_mb * 1048576.0);
}

int pick_slab(const sox_plan& p, int entry) {
  const size_t budget = ws_budget();
  int slab = p.n_tau;
  while (slab > 1 && layout_for(p, entry, slab).total > budget) slab = (slab + 1) / 2;
  return slab;
}

size_t dyn_vjp_total(const sox_plan& p, int vc);  // defined with the adjoint layout

void pick_dyn(sox_plan& p) {
  const size_t budget = ws_budget();
  p.eslab = std::min(p.n_tau, 16);
  int vc = p.n;
  while (vc > 1 && dyn_layout_for(p, vc, p.eslab).total > budget) vc = (vc + 1) / 2;
  p.vc = vc;
  vc = p.n;
  while (vc > 1 && dyn_vjp_total(p, vc) > budget) vc = (vc + 1) / 2;
  p.vc_vjp = vc;
}

bool cfg_allowed(int precision, int cfg) {
  const FusedCfg& c = kFusedCfgs[cfg];
  return precision == SOX_FP64 ? c.fp64 : precision == SOX_FP32 ? c.fp32 : c.bf16;
}

int default_fused_cfg(int precision, int N) {
  if (precision == SOX_FP64) return 0;
  // split precision: the LDS-staged 128 x 128 workgroup tile (2.3x the
  // direct-load 64 x 32 wave tile at n = 64, N = 384 and 1.7x at n = 200,
  // N = 1200)
  if (precision == SOX_BF16X3) return 8;
  // float32: the LDS-staged 128 x 128 workgroup tile (64 x 64 per
  // wavefront) measured 1.18x (N = 384) and 1.20x (N = 1200) the direct-load
  // 64 x 64 wave tile; tiny N keeps the small direct-load tile
  return N >= 256 ? 9 : 0;
}

// the LDS-staged fused kernel's 32-bit byte offsets within one (tau, v)
// panel set: NP rows of nP values, and NP rows of the U-tensor (stride nP^2)
bool lds_offsets_fit(int precision, long NP, long nP) {
  const double es = precision == SOX_BF16X3 ? 2.0 : 4.0;
  const double lim = 4294967296.0;
  return (double)NP * nP * es < lim && (double)NP * nP * nP * es < lim;
}
bool lds_offsets_fit(const sox_plan& p) { return lds_offsets_fit(p.precision, p.NP, p.nP); }

void set_fused_cfg(sox_plan& p, int cfg) {
  p.fused_cfg = cfg;
  const FusedCfg& fc = kFusedCfgs[cfg];
  p.wg_tile = 2 * std::max(fc.wp, fc.wr);
  p.NP = (int)round_up(p.N, p.wg_tile);
}

// A fused config this plan can launch: one of its precision, and for the
// LDS-staged configs (8, 9) panel offsets within 32 bits at that config's
// padding.  Leaves the plan's config unchanged.
bool cfg_usable(const sox_plan& p, int cfg) {
  if (cfg < 0 || cfg >= kNumFusedCfgs || !cfg_allowed(p.precision, cfg)) return false;
  if (cfg != 8 && cfg != 9) return true;
  const FusedCfg& fc = kFusedCfgs[cfg];
  return lds_offsets_fit(p.precision, round_up(p.N, 2 * std::max(fc.wp, fc.wr)), p.nP);
}

sox_status check_plan(const sox_plan* plan) {
  if (!plan) return fail(SOX_ERR_INVALID_ARG, "plan is NULL");
  return SOX_OK;
}

struct VjpLayout {
  size_t u1t, u2t, u2tT, du1t, du2t, mbuf, dgs, dxs;
  size_t p1, p1t, p2t, p2, gbt, a, at, e2, e3, dd, ddt, da, dp1, dp2t, d, total;
};

VjpLayout vjp_layout_for(const sox_plan& p, int entry, int slab) {
  VjpLayout L{};
  const size_t es = elem_size(p.precision);
  const size_t nP = p.nP, NP = p.NP, n = p.n, N = p.N, nt = p.n_tau, c = slab;
  Carver k;
  L.u1t = k.take(NP * nP * nP * es);
  L.u2t = (entry == SOX_ENTRY_BARE) ? L.u1t : k.take(NP * nP * nP * es);
  L.u2tT = k.take(nP * nP * NP * es);
  L.du1t = k.take(NP * nP * nP * 8);
  L.du2t = k.take(nP * NP * nP * 8);
  L.mbuf = k.take(NP * nP * nP * 8);
  L.dgs = k.take(nt * n * n * 8);
  L.dxs = k.take(n * N * 8);
  L.p1 = k.take(c * NP * nP * es);
  L.p1t = k.take(c * nP * NP * es);
  L.p2t = k.take(c * NP * nP * es);
  L.p2 = k.take(c * nP * NP * es);
  L.gbt = k.take(c * nP * nP * es);
  L.a = k.take(c * n * NP * nP * es);
  L.at = k.take(c * n * nP * NP * es);
  L.e2 = k.take(c * n * NP * 8);
  L.e3 = k.take(c * n * NP * 8);
  L.dd = k.take(c * NP * NP * es);
  L.ddt = k.take(c * NP * NP * es);
  L.da = k.take(c * n * NP * nP * 8);
  L.dp1 = k.take(c * NP * nP * 8);
  L.dp2t = k.take(c * NP * nP * 8);
  L.d = k.take(c * NP * NP * es);
  L.total = k.off;
  return L;
}

int pick_vjp_slab(const sox_plan& p, int entry) {
  const size_t budget = ws_budget();
  int slab = p.n_tau;
  while (slab > 1 && vjp_layout_for(p, entry, slab).total > budget) slab = (slab + 1) / 2;
  return slab;
}

size_t solid_workspace_bytes(const sox_plan& p, int entry);  // with the solid launch sequence

size_t vertex_workspace_bytes(const sox_plan& p);  // with the composite entry

size_t gw_workspace_bytes(const sox_plan& p);  // with the GW entry

size_t workspace_bytes(const sox_plan& p, int entry) {
  if (entry == SOX_ENTRY_VERTEX) return vertex_workspace_bytes(p);
  if (entry == SOX_ENTRY_GW) return gw_workspace_bytes(p);
  if (p.nk > 1) return solid_workspace_bytes(p, entry);
  if (entry == SOX_ENTRY_DYNAMIC)
    return p.n_omega > 0 ? std::max(dyn_layout_for(p, p.vc, p.eslab).total, dyn_vjp_total(p, p.vc_vjp))
                         : 0;
  const size_t fwd = layout_for(p, entry, p.slab).total;
  const size_t vjp = vjp_layout_for(p, entry, p.vjp_slab).total;
  return std::max(fwd, vjp);
}

sox_status check_ws(const sox_plan* plan, int entry, const void* ws, size_t ws_bytes) {
  const size_t need = workspace_bytes(*plan, entry);
  if (!ws) return fail(SOX_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (((uintptr_t)ws & 255) != 0) return fail(SOX_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < need)
    return fail(SOX_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  return SOX_OK;
}

// -- launch sequences ----------------------------------------------------------
template <typename T>
sox_status launch_utensor(const sox_plan& p, const double* U, const double* X, T* out,
                          hipStream_t s, float* scratch = nullptr) {
  if (sizeof(T) == 4 && scratch) {
    // float32: U[P][(q,s)] = sum_Q V_PQ KR[(q,s)][Q] on the LDS-staged GEMM
    // (C3: 14.6 ms for both U-tensors with the float64 loader-formed
    // Khatri-Rao product)
    float* KR = scratch;
    float* V32 = scratch + (size_t)p.nP * p.nP * p.NP;
    const long nkr = (long)p.nP * p.nP * p.NP, nv = (long)p.NP * p.NP;
    hipLaunchKernelGGL(kr_kernel, grid1d(nkr), dim3(256), 0, s, X, KR, p.n, p.N, p.nP, p.NP);
    SOX_HIP(hipGetLastError());
    hipLaunchKernelGGL(pad_cast_kernel, grid1d(nv), dim3(256), 0, s, U, V32, p.N, p.N, p.NP,
                       p.NP);
    SOX_HIP(hipGetLastError());
    // ks > 1: K split over the batch index into ks partial blocks, then summed
    const int ks = utensor_ksplit(p);
    const long blk = (long)p.NP * p.nP * p.nP;
    float* part = V32 + nv;
    DenseLdsArgs l{};
    l.A = V32;
    l.B = KR;
    l.C = ks > 1 ? part : (float*)out;
    l.lda = p.NP;
    l.ldb = p.NP;
    l.ldc = (long)p.nP * p.nP;
    l.M = p.NP;
    l.N = p.nP * p.nP;
    l.K = p.NP / ks;
    l.rgroup = l.M;
    l.rvalid = l.M;
    l.sA = l.K;
    l.sB = l.K;
    l.sC = blk;
    SOX_HIP(launch_dense_lds_f32(l, ks, s, p.dense_wg));
    if (ks > 1) {
      hipLaunchKernelGGL(sum_blocks_kernel, grid1d(blk), dim3(256), 0, s, part, (float*)out, blk,
                         blk, ks);
      SOX_HIP(hipGetLastError());
    }
    return SOX_OK;
  }
  UTensorProb<T> pr{U, X, out, p.n, p.N, p.nP, p.NP, p.nP * p.nP, p.N, 0, p.NP};
  SOX_HIP((launch_gemm<UTensorProb<T>, double, 2, 2, 2, 2>(pr, 1, s)));
  return SOX_OK;
}

// A step on the dense kernel: A[b][v][(P,q)] = sum_s GbT[b][v][s] U1t[(P,q)][s]
// (rows v, columns (P,q), stored row-major so stores are contiguous in q).
template <typename T>
sox_status launch_astep(const sox_plan& p, const T* u1t, const T* gbt, T* A, int cnt,
                        hipStream_t s, bf16_t* a_hi = nullptr, bf16_t* a_lo = nullptr) {
  if (sizeof(T) == 4) {
    // LDS-staged GEMM (C3: 37.5 -> 22.4 ms per sweep against the direct-load
    // kernel below); rows (tau, v) with v padded to nP, one launch per slab
    DenseLdsArgs l{};
    l.A = (const float*)gbt;
    l.B = (const float*)u1t;
    l.lda = p.nP;
    l.ldb = p.nP;
    l.M = cnt * p.nP;
    l.N = p.NP * p.nP;
    l.K = p.nP;
    l.rgroup = p.nP;
    l.rvalid = p.n;
    l.c_gstride = (long)p.n * p.NP * p.nP;
    l.ldc = (long)p.NP * p.nP;
    l.C = (float*)A;
    l.Chi = a_hi;  // split-precision path: A is stored only as its hi and lo planes
    l.Clo = a_lo;
    SOX_HIP(launch_dense_lds_f32(l, 1, s, p.dense_wg));
    return SOX_OK;
  }
  DenseArgs<T, T> d{};
  d.Chi = a_hi;
  d.Clo = a_lo;
  d.A = gbt;
  d.B = u1t;
  d.C = A;
  d.lda = p.nP;
  d.ldb = p.nP;
  d.ldc = (long)p.NP * p.nP;
  d.sA = (long)p.nP * p.nP;
  d.sB = 0;
  d.sC = (long)p.n * p.NP * p.nP;
  d.M = p.n;
  d.N = p.NP * p.nP;
  d.K = p.nP;
  d.alpha = T(1);
  d.transposed = 0;
  d.accumulate = 0;
  d.m_fast = 1;  // the v row tiles of one U-tensor column panel back to back
  if (sizeof(T) == 8) {
    SOX_HIP((launch_dense<T, T, 1, 4, 2, 2>(d, cnt, s)));
  } else if ((round_up(p.n, 64) - p.n) * 10 <= p.n) {
    SOX_HIP((launch_dense<T, T, 1, 4, 4, 4>(d, cnt, s)));
  } else {
    SOX_HIP((launch_dense<T, T, 1, 4, 2, 4>(d, cnt, s)));
  }
  return SOX_OK;
}

template <typename T>
sox_status launch_gbar_t(const sox_plan& p, const double* G, T* gbt, int t0, int cnt,
                         hipStream_t s) {
  const long tot = (long)cnt * p.nP * p.nP;
  hipLaunchKernelGGL(gbar_t_kernel<T>, grid1d(tot), dim3(256), 0, s, G,
                     gbt, p.n, p.nP, p.n_tau, t0, cnt);
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}

template <typename T>
sox_status launch_fused_cfg(const sox_plan& p, const FusedArgs<T>& fa, hipStream_t s);

// Resident workgroups per CU of the plan's fused kernel (register-limited).
int fused_blocks_per_cu(const sox_plan& p) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  if (p.precision == SOX_FP32) {
    switch (p.fused_cfg) {
      case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_bcd_kernel<float, 32, 32>, 256, 0); break;
      case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_bcd_kernel<float, 64, 32>, 256, 0); break;
      case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_bcd_kernel<float, 32, 64>, 256, 0); break;
      case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_bcd_kernel<float, 64, 64>, 256, 0); break;
      case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_bcd_kernel<float, 32, 16>, 256, 0); break;
      case 9:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, fused_bcd_lds_kernel<kLdsFp32, kFp32LdsPB>, 1024 / kFp32LdsPB, 0);
        break;
      default: break;
    }
  } else if (p.precision == SOX_BF16X3) {
    if (p.fused_cfg == 8)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, fused_bcd_lds_kernel<kLdsBf16x3, kBf16LdsPB>, 1024 / kBf16LdsPB, 0);
  } else if (p.precision == SOX_FP64) {
    switch (p.fused_cfg) {
      case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_bcd_kernel<double, 32, 32>, 256, 0); break;
      case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_bcd_kernel<double, 32, 16>, 256, 0); break;
      case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_bcd_kernel<double, 16, 32>, 256, 0); break;
      default: break;
    }
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

// Split of the fused kernel's v sum (chunks of at least 8 orbitals): the
// split whose launch over one tau slab fills complete rounds of resident
// workgroups best, each extra split charged 2% for its extra epilogue and
// partial-D traffic; 1 when the launch already holds many rounds.
void pick_vsplit(sox_plan& p) {
  p.fused_vsplit = 1;
  // the split-precision kernels other than the LDS-staged one sum all v
  if ((p.precision == SOX_BF16X3 && p.fused_cfg != 8) || p.nk > 1) return;
  const FusedCfg& fc = kFusedCfgs[p.fused_cfg];
  const long tiles = (long)(p.NP / (2 * fc.wp)) * (p.NP / (2 * fc.wr)) * p.slab;
  const long resident = (long)fused_blocks_per_cu(p) * p.n_cu;
  double best = -1.0;
  for (int s : {1, 2, 3, 4, 6, 8}) {
    const int chunk = (p.n + s - 1) / s;
    if (s > 1 && chunk < 8) break;
    const int se = (p.n + chunk - 1) / chunk;
    const long wgs = tiles * se;
    const long rounds = (wgs + resident - 1) / resident;
    const double score = (double)wgs / (double)(rounds * resident) - 0.02 * (se - 1);
    if (score > best) {
      best = score;
      p.fused_vsplit = se;
    }
  }
  if (layout_for(p, SOX_ENTRY_STATIC, p.slab).total > ws_budget()) p.fused_vsplit = 1;
}

// Arguments of the LDS-staged kernel from the direct-load kernel's (strides
// in elements; one plane per operand in float32, hi and lo in bf16 x 3).
template <typename E>
LdsFusedArgs lds_args(const FusedArgs<float>& fa, const E* a[2], const E* y[2], const E* pt[2],
                      const E* u[2]) {
  LdsFusedArgs l{};
  for (int q = 0; q < 2; ++q) {
    l.bp[q] = (const char*)a[q];
    l.br[q] = (const char*)y[q];
    l.cp[q] = (const char*)pt[q];
    l.cr[q] = (const char*)u[q];
  }
  l.a_tstride = fa.a_tstride; l.a_vstride = fa.a_vstride; l.y_tstride = fa.y_tstride;
  l.p_tstride = fa.p_tstride; l.u_rstride = fa.u_rstride; l.u_vstride = fa.u_vstride;
  l.d_tstride = fa.d_tstride; l.d_sstride = fa.d_sstride;
  l.D = fa.D;
  l.accumulate = fa.accumulate;
  l.n = fa.n; l.nP = fa.nP; l.NP = fa.NP;
  l.tiles_p = fa.tiles_p; l.tiles_r = fa.tiles_r; l.n_tau = fa.n_tau;
  l.vsplit = fa.vsplit > 1 ? fa.vsplit : 1;
  l.vchunk = fa.vsplit > 1 ? fa.vchunk : fa.n;
  return l;
}

template <>
sox_status launch_fused_cfg<float>(const sox_plan& p, const FusedArgs<float>& fa, hipStream_t s) {
  switch (p.fused_cfg) {
    case 9: {
      const float* a[2] = {fa.A, fa.A};
      const float* y[2] = {fa.Y, fa.Y};
      const float* pt[2] = {fa.P2T, fa.P2T};
      const float* u[2] = {fa.U2, fa.U2};
      SOX_HIP((launch_fused_lds<kLdsFp32, kFp32LdsPB>(lds_args(fa, a, y, pt, u), s)));
      break;
    }
    case 0: SOX_HIP((launch_fused<float, 32, 32>(fa, s))); break;
    case 1: SOX_HIP((launch_fused<float, 64, 32>(fa, s))); break;
    case 2: SOX_HIP((launch_fused<float, 32, 64>(fa, s))); break;
    case 3: SOX_HIP((launch_fused<float, 64, 64>(fa, s))); break;
    case 4: SOX_HIP((launch_fused<float, 32, 16>(fa, s))); break;
    default: return fail(SOX_ERR_UNSUPPORTED, "fused config %d has no float32 kernel", p.fused_cfg);
  }
  return SOX_OK;
}

template <>
sox_status launch_fused_cfg<double>(const sox_plan& p, const FusedArgs<double>& fa,
                                    hipStream_t s) {
  switch (p.fused_cfg) {
    case 0: SOX_HIP((launch_fused<double, 32, 32>(fa, s))); break;
    case 4: SOX_HIP((launch_fused<double, 32, 16>(fa, s))); break;
    case 5: SOX_HIP((launch_fused<double, 16, 32>(fa, s))); break;
    default: return fail(SOX_ERR_UNSUPPORTED, "fused config %d has no float64 kernel", p.fused_cfg);
  }
  return SOX_OK;
}

sox_status launch_split(const float* src, bf16_t* hi, bf16_t* lo, long count, hipStream_t s) {
  if (count <= 0) return SOX_OK;
  hipLaunchKernelGGL(split_bf16_kernel, grid1d(count), dim3(256), 0, s, src,
                     hi, lo, count);
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}

// Back-transform of cnt tau nodes in float64 (THC section): Sigma_RP =
// -D_PR, E = X D^T, Sigma[t0 + b] = -E X^T, both products on the direct-load
// float64 MFMA GEMM from the zero-padded XP [n][NP] (float32 D, summed over
// its nsplit partial blocks, is widened into D64 first; float64 D is read in
// place).
template <typename T>
sox_status launch_back(const sox_plan& p, const double* XP, const T* D, double* D64, double* E,
                       double* Sigma, int t0, int cnt, hipStream_t s, int nsplit = 1,
                       long sstride = 0) {
  const int n = p.n, NP = p.NP;
  const double* Dd = (const double*)D;
  if (sizeof(T) == 4) {
    // float32 D (the nsplit partial blocks of a split v sum, if any) summed
    // and widened to float64 in one pass
    const long cd = (long)cnt * NP * NP;
    if (nsplit <= 8 && cd % 4 == 0 && sstride % 4 == 0 && (uintptr_t)D % 16 == 0 &&
        (uintptr_t)D64 % 32 == 0)
      hipLaunchKernelGGL(widen_sum4_kernel, grid1d(cd / 4), dim3(256), 0, s, (const float*)D, D64,
                         cd / 4, sstride, nsplit);
    else if (nsplit > 1)
      hipLaunchKernelGGL(widen_sum_kernel, grid1d(cd), dim3(256), 0, s, (const float*)D, D64, cd,
                         sstride, nsplit);
    else
      hipLaunchKernelGGL(widen_kernel, grid1d(cd), dim3(256), 0, s, (const float*)D, D64, cd);
    SOX_HIP(hipGetLastError());
    Dd = D64;
  } else if (nsplit > 1) {
    return fail(SOX_ERR_SHAPE, "internal: split D blocks in a float64 back-transform");
  }
  DenseArgs<double, double> e{};
  e.A = XP; e.B = Dd; e.C = E;
  e.lda = NP; e.ldb = NP; e.ldc = NP;
  e.sA = 0; e.sB = (long)NP * NP; e.sC = (long)n * NP;
  e.M = n; e.N = NP; e.K = NP; e.alpha = 1.0;
  SOX_HIP((launch_dense<double, double, 1, 4, 2, 2>(e, cnt, s)));
  DenseArgs<double, double> g{};
  g.A = E; g.B = XP; g.C = Sigma + (long)t0 * n * n;
  g.lda = NP; g.ldb = NP; g.ldc = n;
  g.sA = (long)n * NP; g.sB = 0; g.sC = (long)n * n;
  g.M = n; g.N = n; g.K = NP; g.alpha = -1.0;
  SOX_HIP((launch_dense<double, double, 1, 4, 2, 2>(g, cnt, s)));
  return SOX_OK;
}

// XP = X zero padded to [n][NP] float64
sox_status launch_xpad64(const sox_plan& p, const double* X, double* XP, hipStream_t s) {
  const long cx = (long)p.n * p.NP;
  hipLaunchKernelGGL(xpad64_kernel, grid1d(cx), dim3(256), 0, s, X, XP, p.n, p.N, p.NP);
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}

template <typename T>
sox_status run_static(sox_plan& p, int entry, const double* X, const double* U1, const double* U2,
                      const double* G, double* Sigma, void* ws, hipStream_t s) {
  const Layout L = layout_for(p, entry, p.slab);
  char* base = (char*)ws;
  T* u1t = (T*)(base + L.u1);
  T* u2t = (T*)(base + L.u2);
  T* A = (T*)(base + L.a);
  T* P1 = (T*)(base + L.p1);
  T* P2T = (T*)(base + L.p2t);
  T* D = (T*)(base + L.d);
  double* E = (double*)(base + L.e);
  T* gbt = (T*)(base + L.gbt);
  const int n = p.n, N = p.N, nP = p.nP, NP = p.NP;

  if (NP % p.wg_tile != 0) return fail(SOX_ERR_SHAPE, "internal: padded extent not a tile multiple");
  sox_status st;
  {
    ProfScope ps(p, SOX_STAGE_UTENSOR, s);
    float* ukr = (float*)(base + L.ukr);
    st = launch_utensor<T>(p, U1, X, u1t, s, ukr);
    if (st) return st;
    if ((st = launch_xpad64(p, X, (double*)(base + L.xp), s))) return st;
    if (entry != SOX_ENTRY_BARE) {
      st = launch_utensor<T>(p, U2, X, u2t, s, ukr);
      if (st) return st;
    }

  }
  const FusedCfg& fc = kFusedCfgs[p.fused_cfg];
  if (NP % (2 * fc.wp) != 0 || NP % (2 * fc.wr) != 0)
    return fail(SOX_ERR_SHAPE, "internal: padded extent does not fit the fused tile");
  const int tiles_p = NP / (2 * fc.wp), tiles_r = NP / (2 * fc.wr);
  for (int t0 = 0; t0 < p.n_tau; t0 += p.slab) {
    const int cnt = std::min(p.slab, p.n_tau - t0);
    {
      ProfScope ps(p, SOX_STAGE_PROJECT, s);
      ProjP1Prob<T> pr1{X, G, P1, n, N, nP, NP, t0, NP, nP, n};
      SOX_HIP((launch_gemm<ProjP1Prob<T>, double, 2, 2, 2, 2>(pr1, cnt, s)));
      ProjP2TProb<T> pr2{X, G, P2T, n, N, nP, NP, t0, NP, nP, n};
      SOX_HIP((launch_gemm<ProjP2TProb<T>, double, 2, 2, 2, 2>(pr2, cnt, s)));
    }
    {
      ProfScope ps(p, SOX_STAGE_ASTEP, s);
      st = launch_gbar_t<T>(p, G, gbt, t0, cnt, s);
      if (st) return st;
      if (p.precision == SOX_BF16X3)
        st = launch_astep<T>(p, u1t, gbt, A, cnt, s, (bf16_t*)(base + L.ah),
                             (bf16_t*)(base + L.al));
      else
        st = launch_astep<T>(p, u1t, gbt, A, cnt, s);
      if (st) return st;
    }
    FusedArgs<T> fa;
    fa.A = A;
    fa.Y = P1;
    fa.P2T = P2T;
    fa.U2 = u2t;
    fa.D = D;
    fa.a_tstride = (long)n * NP * nP;
    fa.a_vstride = (long)NP * nP;
    fa.y_tstride = (long)NP * nP;
    fa.p_tstride = (long)NP * nP;
    fa.u_rstride = (long)nP * nP;
    fa.u_vstride = nP;
    fa.d_tstride = (long)NP * NP;
    fa.n = n;
    fa.nP = nP;
    fa.NP = NP;
    fa.tiles_p = tiles_p;
    fa.tiles_r = tiles_r;
    fa.n_tau = cnt;
    fa.accumulate = 0;
    fa.vsplit = p.fused_vsplit;
    fa.vchunk = (n + p.fused_vsplit - 1) / p.fused_vsplit;
    fa.d_sstride = (long)p.slab * NP * NP;
    if (p.precision == SOX_BF16X3) {
      // x = hi + lo split of the float32 operands (A arrives split from the
      // A step), then bf16 x 3 MFMA
      bf16_t* ah = (bf16_t*)(base + L.ah); bf16_t* al = (bf16_t*)(base + L.al);
      bf16_t* p1h = (bf16_t*)(base + L.p1h); bf16_t* p1l = (bf16_t*)(base + L.p1l);
      bf16_t* p2h = (bf16_t*)(base + L.p2h); bf16_t* p2l = (bf16_t*)(base + L.p2l);
      bf16_t* u2h = (bf16_t*)(base + L.u2h); bf16_t* u2l = (bf16_t*)(base + L.u2l);
      {
        ProfScope ps(p, SOX_STAGE_SPLIT, s);
        const long np1 = (long)cnt * NP * nP;
        if ((st = launch_split((const float*)P1, p1h, p1l, np1, s))) return st;
        if ((st = launch_split((const float*)P2T, p2h, p2l, np1, s))) return st;
        if (t0 == 0 && (st = launch_split((const float*)u2t, u2h, u2l, (long)NP * nP * nP, s)))
          return st;
      }
      FusedSplitArgs fs;
      fs.Ah = ah; fs.Al = al; fs.Yh = p1h; fs.Yl = p1l; fs.Ph = p2h; fs.Pl = p2l;
      fs.Uh = u2h; fs.Ul = u2l; fs.D = (float*)D;
      fs.a_tstride = fa.a_tstride; fs.a_vstride = fa.a_vstride; fs.y_tstride = fa.y_tstride;
      fs.p_tstride = fa.p_tstride; fs.u_rstride = fa.u_rstride; fs.u_vstride = fa.u_vstride;
      fs.d_tstride = fa.d_tstride; fs.accumulate = 0; fs.n = n; fs.nP = nP; fs.NP = NP;
      fs.tiles_p = tiles_p; fs.tiles_r = tiles_r; fs.n_tau = cnt;
      ProfScope ps(p, SOX_STAGE_FUSED, s);
      if (p.fused_cfg == 8) {
        FusedArgs<float> fl;
        fl.a_tstride = fa.a_tstride; fl.a_vstride = fa.a_vstride; fl.y_tstride = fa.y_tstride;
        fl.p_tstride = fa.p_tstride; fl.u_rstride = fa.u_rstride; fl.u_vstride = fa.u_vstride;
        fl.d_tstride = fa.d_tstride; fl.d_sstride = fa.d_sstride; fl.D = (float*)D;
        fl.accumulate = 0; fl.n = n; fl.nP = nP; fl.NP = NP; fl.tiles_p = tiles_p;
        fl.tiles_r = tiles_r; fl.n_tau = cnt; fl.vsplit = p.fused_vsplit; fl.vchunk = fa.vchunk;
        const bf16_t* a[2] = {ah, al};
        const bf16_t* y[2] = {p1h, p1l};
        const bf16_t* pt[2] = {p2h, p2l};
        const bf16_t* u[2] = {u2h, u2l};
        SOX_HIP((launch_fused_lds<kLdsBf16x3, kBf16LdsPB>(lds_args(fl, a, y, pt, u), s)));
      } else if (p.fused_cfg == 7) {
        SOX_HIP((launch_fused_bf16x3<64, 32>(fs, s)));
      } else {
        SOX_HIP((launch_fused_bf16x3<32, 32>(fs, s)));
      }
    } else {
      ProfScope ps(p, SOX_STAGE_FUSED, s);
      st = launch_fused_cfg<T>(p, fa, s);
      if (st) return st;
    }
    // float32: the v splits' partial D blocks are summed while widening;
    // float64: summed here first
    const int nsplit = sizeof(T) == 4 ? p.fused_vsplit : 1;
    if (sizeof(T) == 8 && p.fused_vsplit > 1) {
      ProfScope ps(p, SOX_STAGE_BACK, s);
      const long count = (long)cnt * NP * NP;
      hipLaunchKernelGGL(dsplit_sum_kernel<T>, grid1d(count), dim3(256), 0,
                         s, D, count, fa.d_sstride, p.fused_vsplit);
      SOX_HIP(hipGetLastError());
    }
    {
      ProfScope ps(p, SOX_STAGE_BACK, s);
      if ((st = launch_back<T>(p, (const double*)(base + L.xp), D, (double*)(base + L.d64), E,
                               Sigma, t0, cnt, s, nsplit, fa.d_sstride)))
        return st;
    }
  }
  return SOX_OK;
}

// W(Omega) GG(Omega) for every Omega of a v-slab: AW[m] = W2[m] GG2[m]^T
// (W2 [2NP][2NP], GG2 [vcn][2NP], AW [2NP][vcn]).  float32 on the LDS-staged
// GEMM (C4: 1.28 s per sweep on the direct-load kernel), float64 on the
// direct-load one.
// Per-block partial maxima of |Im W(Omega)| and |Re W(Omega)| over the block
// operator W2 = [[Wr, -Wi], [Wi, Wr]] of every Matsubara sample.
constexpr int kWchkBlocks = 256;
template <typename T>
__global__ __launch_bounds__(256) void wimag_kernel(const T* W2, int nw, int NP, double* part) {
  __shared__ double si[256], sr[256];
  double a = 0.0, m = 0.0;
  const long ld = 2L * NP, per = (long)NP * NP;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < (long)nw * per;
       i += (long)gridDim.x * 256) {
    const long w = i / per, e = i - w * per;
    const long P = e / NP, Q = e - P * NP;
    const T* B = W2 + w * ld * ld;
    a = fmax(a, fabs((double)B[(NP + P) * ld + Q]));
    m = fmax(m, fabs((double)B[P * ld + Q]));
  }
  si[threadIdx.x] = a;
  sr[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      si[threadIdx.x] = fmax(si[threadIdx.x], si[threadIdx.x + w]);
      sr[threadIdx.x] = fmax(sr[threadIdx.x], sr[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = si[0];
    part[2 * blockIdx.x + 1] = sr[0];
  }
}

// Whether the molecular dynamic entry of a float32 or bf16x3 plan may run
// the real W(Omega) product: the plan's transform of W_d(tau) has an
// imaginary part below float32 resolution of its real part (max |Im W| <=
// 2^-24 max |Re W|), so its products lie below the rounding of the real
// ones.  A W(tau) mirror symmetric in tau has a real W(i Omega) in the
// continuum; on a fine grid the discrete pair keeps that (about 1e-8 on the
// n=300, 120-node workload), on a coarse one it does not, and an asymmetric
// W(tau) never does.  Builds W(Omega) into the dynamic workspace `dws` (the
// pass rebuilds it) and synchronises `s` once to read the maxima.
sox_status dynamic_w_is_real(sox_plan& p, const double* Wtau, void* dws, hipStream_t s,
                             bool* real_w) {
  *real_w = false;
  if (p.precision == SOX_FP64 || p.nk > 1 || !p.d_wchk) return SOX_OK;
  const DynLayout L = dyn_layout_for(p, p.vc, p.eslab);
  float* W2 = (float*)((char*)dws + L.w2);
  const int nw = p.n_omega, nt = p.n_tau, N = p.N, NP = p.NP;
  WOmegaProb<float> wp{p.d_tf2, Wtau, W2, nw, nt, N, NP, 2 * nw, NP * NP, nt, nullptr};
  SOX_HIP((launch_gemm<WOmegaProb<float>, double, 2, 2, 2, 2>(wp, 1, s)));
  hipLaunchKernelGGL(wimag_kernel<float>, dim3(kWchkBlocks), dim3(256), 0, s, W2, nw, NP,
                     p.d_wchk);
  SOX_HIP(hipGetLastError());
  double part[2 * kWchkBlocks];
  SOX_HIP(hipMemcpyAsync(part, p.d_wchk, sizeof(part), hipMemcpyDeviceToHost, s));
  SOX_HIP(hipStreamSynchronize(s));
  double a = 0.0, m = 0.0;
  for (int b = 0; b < kWchkBlocks; ++b) {
    a = std::max(a, part[2 * b]);
    m = std::max(m, part[2 * b + 1]);
  }
  *real_w = m > 0.0 && a <= std::ldexp(m, -24);
  return SOX_OK;
}

// W(Omega) GG(Omega) with the block operator W2 = [[Wr, -Wi], [Wi, Wr]] on
// GG2 rows [GGr | GGi]: AW rows [0, NP) = Re, [NP, 2NP) = Im.  real_w: W(Omega)
// is real (a mirror-symmetric W_d(tau)), so Re = Wr GGr and Im = Wr GGi, two
// products of half the depth over half the rows: a quarter of the block
// product's work each.
template <typename T>
sox_status launch_wgg(const T* W2, const T* GG2, T* AW, int NP, long vcn, int nw, hipStream_t s,
                      bool real_w = false) {
  if (sizeof(T) == 4 && real_w) {
    for (int c = 0; c < 2; ++c) {
      DenseLdsArgs l{};
      l.A = (const float*)W2;
      l.B = (const float*)GG2 + (long)c * NP;
      l.C = (float*)AW + (long)c * NP * vcn;
      l.lda = 2L * NP; l.ldb = 2L * NP; l.ldc = vcn;
      l.sA = 4L * NP * NP; l.sB = vcn * 2 * NP; l.sC = 2L * NP * vcn;
      l.M = NP; l.N = (int)vcn; l.K = NP;
      l.rgroup = l.M; l.rvalid = l.M;
      SOX_HIP(launch_dense_lds_f32(l, nw, s));
    }
    return SOX_OK;
  }
  if (sizeof(T) == 4) {
    DenseLdsArgs l{};
    l.A = (const float*)W2;
    l.B = (const float*)GG2;
    l.C = (float*)AW;
    l.lda = 2L * NP;
    l.ldb = 2L * NP;
    l.ldc = vcn;
    l.sA = 4L * NP * NP;
    l.sB = vcn * 2 * NP;
    l.sC = 2L * NP * vcn;
    l.M = 2 * NP;
    l.N = (int)vcn;
    l.K = 2 * NP;
    l.rgroup = l.M;
    l.rvalid = l.M;
    SOX_HIP(launch_dense_lds_f32(l, nw, s));
    return SOX_OK;
  }
  DenseArgs<T, T> d{};
  d.A = W2; d.B = GG2; d.C = AW;
  d.lda = 2L * NP; d.ldb = 2L * NP; d.ldc = vcn;
  d.sA = 4L * NP * NP; d.sB = vcn * 2 * NP; d.sC = 2L * NP * vcn;
  d.M = 2 * NP; d.N = (int)vcn; d.K = 2 * NP; d.alpha = T(1);
  SOX_HIP((launch_dense<T, T, 2, 2, 2, 2>(d, nw, s)));
  return SOX_OK;
}

template <typename T>
sox_status launch_transpose(const T* in, T* out, int rows, int cols, long batch, hipStream_t s);

template <typename T>
sox_status run_dynamic(sox_plan& p, const double* X, const double* Wtau, const double* V,
                       const double* G, double* Sigma, void* ws, hipStream_t s, int vcw = 0,
                       T* W2T = nullptr, bool real_w = false) {
  if (vcw <= 0) vcw = p.vc;
  const DynLayout L = dyn_layout_for(p, vcw, p.eslab);
  char* base = (char*)ws;
  double* P1d = (double*)(base + L.p1d);
  double* P2Td = (double*)(base + L.p2td);
  double* P1q = (double*)(base + L.p1q);
  double* P2q = (double*)(base + L.p2q);
  T* P2T = (T*)(base + L.p2t);
  T* XT = (T*)(base + L.xt);
  T* U2 = (T*)(base + L.u2);
  T* W2 = (T*)(base + L.w2);
  T* GG2 = (T*)(base + L.gg2);
  T* AW = (T*)(base + L.aw);
  T* Adyn = (T*)(base + L.adyn);
  T* D = (T*)(base + L.d);
  double* E = (double*)(base + L.e);
  const int n = p.n, N = p.N, nP = p.nP, NP = p.NP, nt = p.n_tau, nw = p.n_omega;
  const FusedCfg& fc = kFusedCfgs[p.fused_cfg];
  if (NP % (2 * fc.wp) != 0 || NP % (2 * fc.wr) != 0)
    return fail(SOX_ERR_SHAPE, "internal: padded extent does not fit the fused tile");
  sox_status st;
  {
    ProfScope ps(p, SOX_STAGE_UTENSOR, s);
    st = launch_utensor<T>(p, V, X, U2, s, (float*)(base + L.ukr));
    if (st) return st;
    if ((st = launch_xpad64(p, X, (double*)(base + L.xp), s))) return st;
  }
  {
    ProfScope ps(p, SOX_STAGE_PROJECT, s);
    ProjP1Prob<double> pr1{X, G, P1d, n, N, nP, NP, 0, NP, nP, n};
    SOX_HIP((launch_gemm<ProjP1Prob<double>, double, 2, 2, 2, 2>(pr1, nt, s)));
    ProjP2TProb<double> pr2{X, G, P2Td, n, N, nP, NP, 0, NP, nP, n};
    SOX_HIP((launch_gemm<ProjP2TProb<double>, double, 2, 2, 2, 2>(pr2, nt, s)));
    const long cnt = (long)nt * NP * nP;
    hipLaunchKernelGGL(cast_kernel<T>, grid1d(cnt), dim3(256), 0, s, P2Td,
                       P2T, cnt);
    SOX_HIP(hipGetLastError());
    const long cx = (long)NP * nP;
    hipLaunchKernelGGL(xt_kernel<T>, grid1d(cx), dim3(256), 0, s, X, XT,
                       n, N, nP, NP);
    SOX_HIP(hipGetLastError());
    // Q-contiguous copies for the forward transform's loads
    if ((st = launch_transpose<double>(P1d, P1q, NP, nP, nt, s))) return st;
    if ((st = launch_transpose<double>(P2Td, P2q, NP, nP, nt, s))) return st;
  }
  const bool split = p.precision == SOX_BF16X3;
  if (split) {
    // the v-independent operands of the fused contraction as bf16 hi/lo planes
    ProfScope ps(p, SOX_STAGE_SPLIT, s);
    if (p.fused_cfg != 8)
      return fail(SOX_ERR_UNSUPPORTED, "the dynamic entry in bf16x3 runs the LDS-staged kernel only");
    if ((st = launch_split((const float*)XT, (bf16_t*)(base + L.xth), (bf16_t*)(base + L.xtl),
                           (long)NP * nP, s)))
      return st;
    if ((st = launch_split((const float*)P2T, (bf16_t*)(base + L.p2h), (bf16_t*)(base + L.p2l),
                           (long)nt * NP * nP, s)))
      return st;
    if ((st = launch_split((const float*)U2, (bf16_t*)(base + L.u2h), (bf16_t*)(base + L.u2l),
                           (long)NP * nP * nP, s)))
      return st;
  }
  {
    ProfScope ps(p, SOX_STAGE_GG_FT, s);
    WOmegaProb<T> wp{p.d_tf2, Wtau, W2, nw, nt, N, NP, 2 * nw, NP * NP, nt, W2T};
    SOX_HIP((launch_gemm<WOmegaProb<T>, double, 2, 2, 2, 2>(wp, 1, s)));
    // split precision: W(Omega) as bf16 hi/lo planes for the W GG product
    if (split && (st = launch_split((const float*)W2, (bf16_t*)(base + L.w2h),
                                    (bf16_t*)(base + L.w2l), (long)nw * 4 * NP * NP, s)))
      return st;
  }
  const int tiles_p = NP / (2 * fc.wp), tiles_r = NP / (2 * fc.wr);
  for (int v0 = 0; v0 < n; v0 += vcw) {
    const int vc = std::min(vcw, n - v0);
    {
      ProfScope ps(p, SOX_STAGE_GG_FT, s);
      FTProb<T> ft{p.d_tf2, P1q, P2q, GG2, n, nP, NP, N, nw, nt, v0, vc, 2 * nw, vc * n * NP, nt,
                   nullptr, 0, 1};
      if (split) {  // GG(Omega) as hi and lo planes in the GG2 buffer
        ft.GGhi = (bf16_t*)GG2;
        ft.GGlo = ft.GGhi + (long)nw * vc * n * 2 * NP;
      }
      // 80-row tiles: all 2 n_Omega rows (72 at n_Omega = 36) in one tile, so
      // each GG column is formed once (C4: 279 -> 204 ms against 64-row tiles)
      SOX_HIP(launch_ft<T>(ft, p.n_cu, s));
    }
    {
      ProfScope ps(p, SOX_STAGE_WGEMM, s);
      if (split) {
        const long vcn = (long)vc * n;
        DenseLdsSplitArgs l{};
        l.Ah = (const bf16_t*)(base + L.w2h);
        l.Al = (const bf16_t*)(base + L.w2l);
        l.Bh = (const bf16_t*)GG2;
        l.Bl = l.Bh + (long)nw * vcn * 2 * NP;
        l.C = (float*)AW;
        l.lda = 2L * NP; l.ldb = 2L * NP; l.ldc = vcn;
        l.sA = 4L * NP * NP; l.sB = vcn * 2 * NP; l.sC = 2L * NP * vcn;
        l.M = 2 * NP; l.N = (int)vcn; l.K = 2 * NP;
        if (real_w) {
          // Re = Wr GGr, Im = Wr GGi (the top-left block of the split W2 planes)
          l.M = NP; l.K = NP;
          for (int c = 0; c < 2; ++c) {
            DenseLdsSplitArgs h = l;
            h.Bh = l.Bh + (long)c * NP;
            h.Bl = l.Bl + (long)c * NP;
            h.C = l.C + (long)c * NP * vcn;
            SOX_HIP(launch_dense_lds_bf16x3<2>(h, nw, s));
          }
        } else {
          // eight wavefronts of 64 x 32 (n=300 N=1800: 296 -> 274 ms per sweep
          // against four of 64 x 64)
          SOX_HIP(launch_dense_lds_bf16x3<2>(l, nw, s));
        }
      } else if ((st = launch_wgg<T>(W2, GG2, AW, NP, (long)vc * n, nw, s, real_w))) {
        return st;
      }
    }
    {
      ProfScope ps(p, SOX_STAGE_IFT, s);
      IFTProb<T> ift{p.d_tb2, AW, Adyn, n, nP, NP, nw, nt, vc, nt, NP * vc * nP, 2 * nw};
      if (split) {  // A(tau) as hi and lo planes in the A(tau) buffer
        ift.Ahi = (bf16_t*)Adyn;
        ift.Alo = ift.Ahi + (long)nt * vc * NP * nP;
      }
      SOX_HIP(launch_ift<T>(ift, p.n_cu, s));
    }
    FusedArgs<T> fa;
    fa.A = Adyn;
    fa.Y = XT;
    fa.P2T = P2T;
    fa.U2 = U2 + (long)v0 * nP;
    fa.D = D;
    fa.a_tstride = (long)vc * NP * nP;
    fa.a_vstride = (long)NP * nP;
    fa.y_tstride = 0;
    fa.p_tstride = (long)NP * nP;
    fa.u_rstride = (long)nP * nP;
    fa.u_vstride = nP;
    fa.d_tstride = (long)NP * NP;
    fa.accumulate = v0 > 0;
    fa.n = vc;
    fa.nP = nP;
    fa.NP = NP;
    fa.tiles_p = tiles_p;
    fa.tiles_r = tiles_r;
    fa.n_tau = nt;
    if (split) {
      ProfScope ps(p, SOX_STAGE_FUSED, s);
      FusedArgs<float> fl;
      fl.a_tstride = fa.a_tstride; fl.a_vstride = fa.a_vstride; fl.y_tstride = 0;
      fl.p_tstride = fa.p_tstride; fl.u_rstride = fa.u_rstride; fl.u_vstride = fa.u_vstride;
      fl.d_tstride = fa.d_tstride; fl.D = (float*)D; fl.accumulate = fa.accumulate;
      fl.n = vc; fl.nP = nP; fl.NP = NP; fl.tiles_p = tiles_p; fl.tiles_r = tiles_r;
      fl.n_tau = nt;
      const bf16_t* ah = (const bf16_t*)Adyn;
      const bf16_t* a[2] = {ah, ah + (long)nt * vc * NP * nP};
      const bf16_t* y[2] = {(const bf16_t*)(base + L.xth), (const bf16_t*)(base + L.xtl)};
      const bf16_t* pt[2] = {(const bf16_t*)(base + L.p2h), (const bf16_t*)(base + L.p2l)};
      const bf16_t* u[2] = {(const bf16_t*)(base + L.u2h) + (long)v0 * nP,
                            (const bf16_t*)(base + L.u2l) + (long)v0 * nP};
      SOX_HIP((launch_fused_lds<kLdsBf16x3, kBf16LdsPB>(lds_args(fl, a, y, pt, u), s)));
    } else {
      ProfScope ps(p, SOX_STAGE_FUSED, s);
      st = launch_fused_cfg<T>(p, fa, s);
      if (st) return st;
    }
  }
  for (int t0 = 0; Sigma && t0 < nt; t0 += p.eslab) {
    const int cnt = std::min(p.eslab, nt - t0);
    ProfScope ps(p, SOX_STAGE_BACK, s);
    if ((st = launch_back<T>(p, (const double*)(base + L.xp), D + (long)t0 * NP * NP,
                             (double*)(base + L.d64), E, Sigma, t0, cnt, s)))
      return st;
  }
  return SOX_OK;
}

template <typename T>
sox_status launch_transpose(const T* in, T* out, int rows, int cols, long batch, hipStream_t s) {
  if (batch <= 0) return SOX_OK;
  if (batch > 65535) return fail(SOX_ERR_SHAPE, "internal: transpose batch too large");
  dim3 grid((cols + 31) / 32, (rows + 31) / 32, (unsigned)batch);
  hipLaunchKernelGGL(transpose_kernel<T>, grid, dim3(256), 0, s, in, out, rows, cols, batch);
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}

template <typename T>
sox_status launch_fill(T* ptr, long count, hipStream_t s) {
  if (count <= 0) return SOX_OK;
  hipLaunchKernelGGL(fill_kernel<T>, grid1d(count), dim3(256), 0, s, ptr,
                     count, T(0));
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}

// A wavefront keeps all ny output columns in registers (at most 20 blocks of
// 16); a wider y range runs as several launches over 320-column chunks of F
// and Out, each recomputing the stage-1 tile it weights.
template <typename T>
sox_status launch_hc_cfg(const sox_plan& p, HcArgs<T, double> a, int nx, hipStream_t s) {
  constexpr int kYChunk = 320;
  if (a.ny > kYChunk) {
    for (int y0 = 0; y0 < a.ny; y0 += kYChunk) {
      HcArgs<T, double> b = a;
      b.FT = a.FT + (long)y0 * a.f_ld;
      b.Out = a.Out + y0;
      b.ny = std::min(kYChunk, a.ny - y0);
      sox_status st = launch_hc_cfg<T>(p, b, nx, s);
      if (st) return st;
    }
    return SOX_OK;
  }
  const int nyb = a.ny / 16;
  const bool wide = sizeof(T) == 4 && nx % 128 == 0;
#define SOX_HC(XB, YB) SOX_HIP((launch_hc<T, double, XB, YB>(a, nx, s)))
  if (nyb <= 4) { if (wide) SOX_HC(2, 4); else SOX_HC(1, 4); }
  else if (nyb <= 8) { if (wide) SOX_HC(2, 8); else SOX_HC(1, 8); }
  else if (nyb <= 13) { if (wide) SOX_HC(2, 13); else SOX_HC(1, 13); }
  else { if (wide) SOX_HC(2, 20); else SOX_HC(1, 20); }
#undef SOX_HC
  (void)p;
  return SOX_OK;
}

template <typename T>
sox_status run_vjp_static(sox_plan& p, int entry, const double* X, const double* U1,
                          const double* U2, const double* G, const double* R, double* dG,
                          double* dX, double* dU1, double* dU2, void* ws, hipStream_t s) {
  // the bare entry carries one interaction: both lines read U1 (U2 may be NULL)
  if (entry == SOX_ENTRY_BARE) U2 = U1;
  const VjpLayout L = vjp_layout_for(p, entry, p.vjp_slab);
  char* base = (char*)ws;
  T* u1t = (T*)(base + L.u1t);
  T* u2t = (T*)(base + L.u2t);
  T* u2tT = (T*)(base + L.u2tT);
  double* du1t = (double*)(base + L.du1t);
  double* du2t = (double*)(base + L.du2t);
  double* mbuf = (double*)(base + L.mbuf);
  double* dGs = (double*)(base + L.dgs);
  double* dXs = (double*)(base + L.dxs);
  T* P1 = (T*)(base + L.p1);
  T* P1T = (T*)(base + L.p1t);
  T* P2T = (T*)(base + L.p2t);
  T* P2 = (T*)(base + L.p2);
  T* gbt = (T*)(base + L.gbt);
  T* A = (T*)(base + L.a);
  T* AT = (T*)(base + L.at);
  double* E2 = (double*)(base + L.e2);
  double* E3 = (double*)(base + L.e3);
  T* dD = (T*)(base + L.dd);
  T* dDT = (T*)(base + L.ddt);
  double* dA = (double*)(base + L.da);
  double* dP1 = (double*)(base + L.dp1);
  double* dP2T = (double*)(base + L.dp2t);
  T* D = (T*)(base + L.d);
  const int n = p.n, N = p.N, nP = p.nP, NP = p.NP, nt = p.n_tau;
  const long NPnP = (long)NP * nP;
  const FusedCfg& fc = kFusedCfgs[p.fused_cfg];
  if (NP % (2 * fc.wp) != 0 || NP % (2 * fc.wr) != 0 || NP % 64 != 0)
    return fail(SOX_ERR_SHAPE, "internal: padded extent does not fit the tiles");
  const int tiles_p = NP / (2 * fc.wp), tiles_r = NP / (2 * fc.wr);
  ProfScope ps(p, SOX_STAGE_VJP, s);
  sox_status st;
  if ((st = launch_fill<double>(dGs, (long)nt * n * n, s))) return st;
  if ((st = launch_fill<double>(dXs, (long)n * N, s))) return st;
  if ((st = launch_fill<double>(du1t, NPnP * nP, s))) return st;
  if ((st = launch_fill<double>(du2t, NPnP * nP, s))) return st;
  if ((st = launch_utensor<T>(p, U1, X, u1t, s))) return st;
  if (entry != SOX_ENTRY_BARE && (st = launch_utensor<T>(p, U2, X, u2t, s))) return st;
  {
    UTensorProb<T> pr{U2, X, u2tT, n, N, nP, NP, nP * nP, N, 1, NP};
    SOX_HIP((launch_gemm<UTensorProb<T>, double, 2, 2, 2, 2>(pr, 1, s)));
  }
  for (int t0 = 0; t0 < nt; t0 += p.vjp_slab) {
    const int cnt = std::min(p.vjp_slab, nt - t0);
    // forward intermediates of the slab
    ProjP1Prob<T> pr1{X, G, P1, n, N, nP, NP, t0, NP, nP, n};
    SOX_HIP((launch_gemm<ProjP1Prob<T>, double, 2, 2, 2, 2>(pr1, cnt, s)));
    ProjP2TProb<T> pr2{X, G, P2T, n, N, nP, NP, t0, NP, nP, n};
    SOX_HIP((launch_gemm<ProjP2TProb<T>, double, 2, 2, 2, 2>(pr2, cnt, s)));
    if ((st = launch_transpose<T>(P1, P1T, NP, nP, cnt, s))) return st;
    if ((st = launch_transpose<T>(P2T, P2, NP, nP, cnt, s))) return st;
    if ((st = launch_gbar_t<T>(p, G, gbt, t0, cnt, s))) return st;
    if ((st = launch_astep<T>(p, u1t, gbt, A, cnt, s))) return st;
    if ((st = launch_transpose<T>(A, AT, NP, nP, (long)cnt * n, s))) return st;
    // cotangent of D
    RXProb rx{R, X, E2, n, N, NP, t0, 0, n, N, n};
    SOX_HIP((launch_gemm<RXProb, double, 2, 2, 2, 2>(rx, cnt, s)));
    RXProb rx3{R, X, E3, n, N, NP, t0, 1, n, N, n};
    SOX_HIP((launch_gemm<RXProb, double, 2, 2, 2, 2>(rx3, cnt, s)));
    DDProb<T> ddp{X, E2, dD, dDT, n, N, NP, NP, NP, n};
    SOX_HIP((launch_gemm<DDProb<T>, double, 2, 2, 2, 2>(ddp, cnt, s)));
    // D itself (for the back-transform's dX term)
    FusedArgs<T> fa;
    fa.A = A; fa.Y = P1; fa.P2T = P2T; fa.U2 = u2t; fa.D = D;
    fa.a_tstride = (long)n * NPnP; fa.a_vstride = NPnP; fa.y_tstride = NPnP; fa.p_tstride = NPnP;
    fa.u_rstride = (long)nP * nP; fa.u_vstride = nP; fa.d_tstride = (long)NP * NP;
    fa.accumulate = 0; fa.n = n; fa.nP = nP; fa.NP = NP;
    fa.tiles_p = tiles_p; fa.tiles_r = tiles_r; fa.n_tau = cnt;
    if ((st = launch_fused_cfg<T>(p, fa, s))) return st;
    // the four Hadamard-contract adjoints
    HcArgs<T, double> h{};
    h.nz = NP; h.nk = nP; h.ny = nP;
    // dA[b][v][P][q] = sum_R dD[P,R] C[R,v,P] G_Rq[R,q]
    h.L = u2t; h.l_ld = (long)nP * nP; h.l_ts = 0; h.l_vs = nP;
    h.Rm = P2T; h.r_ld = nP; h.r_ts = NPnP; h.r_vs = 0;
    h.W = dDT; h.w_ld = NP; h.w_ts = (long)NP * NP;
    h.FT = P1T; h.f_ld = NP; h.f_ts = NPnP; h.f_vs = 0;
    h.Out = dA; h.o_ld = nP; h.o_ts = (long)n * NPnP; h.o_vs = NPnP;
    h.n_ot = cnt; h.n_ov = n; h.n_it = 1; h.n_iv = 1; h.accumulate = 0;
    if ((st = launch_hc_cfg<T>(p, h, NP, s))) return st;
    // dG_Rq[b][R][q] = sum_{P,v} dD[P,R] C[R,v,P] A[P,q,v]
    h.L = P2T; h.l_ld = nP; h.l_ts = NPnP; h.l_vs = 0;
    h.Rm = u2t; h.r_ld = (long)nP * nP; h.r_ts = 0; h.r_vs = nP;
    h.W = dD;
    h.FT = AT; h.f_ld = NP; h.f_ts = (long)n * NPnP; h.f_vs = NPnP;
    h.Out = dP1; h.o_ld = nP; h.o_ts = NPnP; h.o_vs = 0;
    h.n_ot = cnt; h.n_ov = 1; h.n_it = 1; h.n_iv = n; h.accumulate = 0;
    if ((st = launch_hc_cfg<T>(p, h, NP, s))) return st;
    // dU2[v][R][w] += sum_{tau,P} dD[P,R] B[P,R,v] G_wP[w,P]
    h.L = A; h.l_ld = nP; h.l_ts = (long)n * NPnP; h.l_vs = NPnP;
    h.Rm = P1; h.r_ld = nP; h.r_ts = NPnP; h.r_vs = 0;
    h.W = dD;
    h.FT = P2; h.f_ld = NP; h.f_ts = NPnP; h.f_vs = 0;
    h.Out = du2t; h.o_ld = nP; h.o_ts = 0; h.o_vs = NPnP;
    h.n_ot = 1; h.n_ov = n; h.n_it = cnt; h.n_iv = 1; h.accumulate = 1;
    if ((st = launch_hc_cfg<T>(p, h, NP, s))) return st;
    // dG_wP^T[b][P][w] = sum_{R,v} dD[P,R] B[P,R,v] U2[R,v,w]
    h.L = P1; h.l_ld = nP; h.l_ts = NPnP; h.l_vs = 0;
    h.Rm = A; h.r_ld = nP; h.r_ts = (long)n * NPnP; h.r_vs = NPnP;
    h.W = dDT;
    h.FT = u2tT; h.f_ld = NP; h.f_ts = 0; h.f_vs = NPnP;
    h.Out = dP2T; h.o_ld = nP; h.o_ts = NPnP; h.o_vs = 0;
    h.n_ot = cnt; h.n_ov = 1; h.n_it = 1; h.n_iv = n; h.accumulate = 0;
    if ((st = launch_hc_cfg<T>(p, h, NP, s))) return st;
    // A step adjoint: dU1t and dG(beta - tau)
    DU1tProb du{dA, G, du1t, n, nP, NP, nt, t0, (int)NPnP, nP, cnt * n};
    SOX_HIP((launch_gemm<DU1tProb, double, 2, 2, 2, 2>(du, 1, s)));
    DGbProb<T> dgb{u1t, dA, dGs, n, nP, NP, nt, t0, n, n, (int)NPnP};
    SOX_HIP((launch_gemm<DGbProb<T>, double, 2, 2, 2, 2>(dgb, cnt, s)));
    // half-projection adjoints
    DGProjProb g1{X, dP1, dGs, n, N, nP, NP, t0, 0, n, n, N};
    SOX_HIP((launch_gemm<DGProjProb, double, 2, 2, 2, 2>(g1, cnt, s)));
    DGProjProb g2{X, dP2T, dGs, n, N, nP, NP, t0, 1, n, n, N};
    SOX_HIP((launch_gemm<DGProjProb, double, 2, 2, 2, 2>(g2, cnt, s)));
    DXProjProb x1{G, dP1, dXs, n, N, nP, NP, t0, 0, n, N, cnt * nP};
    SOX_HIP((launch_gemm<DXProjProb, double, 2, 2, 2, 2>(x1, 1, s)));
    DXProjProb x2{G, dP2T, dXs, n, N, nP, NP, t0, 1, n, N, cnt * nP};
    SOX_HIP((launch_gemm<DXProjProb, double, 2, 2, 2, 2>(x2, 1, s)));
    // back-transform adjoint
    DXBackProb<T> b1{E2, D, dXs, n, N, NP, 0, n, N, cnt * NP};
    SOX_HIP((launch_gemm<DXBackProb<T>, double, 2, 2, 2, 2>(b1, 1, s)));
    DXBackProb<T> b2{E3, D, dXs, n, N, NP, 1, n, N, cnt * NP};
    SOX_HIP((launch_gemm<DXBackProb<T>, double, 2, 2, 2, 2>(b2, 1, s)));
  }
  // U-contraction adjoints
  const bool bare = entry == SOX_ENTRY_BARE;
  if (dU1) {
    DUProb a1{du1t, X, dU1, n, N, nP, NP, 0, 0, N, N, nP * nP};
    SOX_HIP((launch_gemm<DUProb, double, 2, 2, 2, 2>(a1, 1, s)));
  }
  double* dU2dst = bare ? dU1 : dU2;
  if (dU2dst) {
    DUProb a2{du2t, X, dU2dst, n, N, nP, NP, 1, bare ? 1 : 0, N, N, nP * nP};
    SOX_HIP((launch_gemm<DUProb, double, 2, 2, 2, 2>(a2, 1, s)));
  }
  const long nx = (long)n * N;
  DUMProb m1{U1, du1t, mbuf, n, N, nP, NP, 0, N, nP * nP, N};
  SOX_HIP((launch_gemm<DUMProb, double, 2, 2, 2, 2>(m1, 1, s)));
  hipLaunchKernelGGL(ut_adjoint_x_kernel, grid1d(nx), dim3(256), 0, s, mbuf,
                     X, dXs, n, N, nP);
  SOX_HIP(hipGetLastError());
  DUMProb m2{U2, du2t, mbuf, n, N, nP, NP, 1, N, nP * nP, N};
  SOX_HIP((launch_gemm<DUMProb, double, 2, 2, 2, 2>(m2, 1, s)));
  hipLaunchKernelGGL(ut_adjoint_x_kernel, grid1d(nx), dim3(256), 0, s, mbuf,
                     X, dXs, n, N, nP);
  SOX_HIP(hipGetLastError());
  if (dG) SOX_HIP(hipMemcpyAsync(dG, dGs, sizeof(double) * nt * n * n, hipMemcpyDeviceToDevice, s));
  if (dX) SOX_HIP(hipMemcpyAsync(dX, dXs, sizeof(double) * nx, hipMemcpyDeviceToDevice, s));
  return SOX_OK;
}

struct DynVjpLayout {
  size_t w2t, gg2t, daw, dawt, dw2, dgg2, dgg, dadyn, adynT, p2, xp, u2tT, dd, ddt, e2, e3;
  size_t dp1d, dp2td, dxt, du2t, mbuf, dgs, dxs, total;
  int ldk;
};

DynVjpLayout dyn_vjp_layout_for(const sox_plan& p, int vc) {
  DynVjpLayout L{};
  const size_t es = elem_size(p.precision);
  const size_t nP = p.nP, NP = p.NP, n = p.n, N = p.N, nt = p.n_tau, nw = p.n_omega;
  L.ldk = (int)round_up((long)vc * n, 16);
  const size_t ldk = L.ldk;
  Carver k;
  k.off = dyn_layout_for(p, vc, p.eslab).total;
  L.w2t = k.take(nw * 4 * NP * NP * es);
  L.gg2t = k.take(nw * 2 * NP * ldk * es);
  L.daw = k.take(nw * 2 * NP * ldk * es);
  L.dawt = k.take(nw * (size_t)vc * n * 2 * NP * es);
  L.dw2 = k.take(nw * 4 * NP * NP * 8);
  L.dgg2 = k.take(nw * (size_t)vc * n * 2 * NP * 8);
  L.dgg = k.take(nt * (size_t)vc * n * NP * 8);
  L.dadyn = k.take(nt * (size_t)vc * NP * nP * 8);
  L.adynT = k.take(nt * (size_t)vc * nP * NP * es);
  L.p2 = k.take(nt * nP * NP * es);
  L.xp = k.take(nP * NP * es);
  L.u2tT = k.take(nP * nP * NP * es);
  L.dd = k.take(nt * NP * NP * es);
  L.ddt = k.take(nt * NP * NP * es);
  L.e2 = k.take(nt * n * NP * 8);
  L.e3 = k.take(nt * n * NP * 8);
  L.dp1d = k.take(nt * NP * nP * 8);
  L.dp2td = k.take(nt * NP * nP * 8);
  L.dxt = k.take(nt * NP * nP * 8);
  L.du2t = k.take(nP * NP * nP * 8);
  L.mbuf = k.take(NP * nP * nP * 8);
  L.dgs = k.take(nt * n * n * 8);
  L.dxs = k.take(n * N * 8);
  L.total = k.off;
  return L;
}

size_t dyn_vjp_total(const sox_plan& p, int vc) { return dyn_vjp_layout_for(p, vc).total; }

template <typename T>
sox_status run_vjp_dynamic(sox_plan& p, const double* X, const double* Wtau, const double* V,
                           const double* G, const double* R, double* dG, double* dX, double* dW,
                           double* dV, void* ws, hipStream_t s) {
  const int vcw = p.vc_vjp;
  const DynLayout F = dyn_layout_for(p, vcw, p.eslab);
  const DynVjpLayout L = dyn_vjp_layout_for(p, vcw);
  char* base = (char*)ws;
  double* P1d = (double*)(base + F.p1d);
  double* P2Td = (double*)(base + F.p2td);
  T* P2T = (T*)(base + F.p2t);
  T* XT = (T*)(base + F.xt);
  T* U2 = (T*)(base + F.u2);
  T* W2 = (T*)(base + F.w2);
  T* GG2 = (T*)(base + F.gg2);
  T* AW = (T*)(base + F.aw);
  T* Adyn = (T*)(base + F.adyn);
  T* D = (T*)(base + F.d);
  T* W2T = (T*)(base + L.w2t);
  T* GG2T = (T*)(base + L.gg2t);
  T* dAW = (T*)(base + L.daw);
  T* dAWT = (T*)(base + L.dawt);
  double* dW2 = (double*)(base + L.dw2);
  double* dGG2 = (double*)(base + L.dgg2);
  double* dGG = (double*)(base + L.dgg);
  double* dAdyn = (double*)(base + L.dadyn);
  T* AdynT = (T*)(base + L.adynT);
  T* P2 = (T*)(base + L.p2);
  T* XP = (T*)(base + L.xp);
  T* u2tT = (T*)(base + L.u2tT);
  T* dD = (T*)(base + L.dd);
  T* dDT = (T*)(base + L.ddt);
  double* E2 = (double*)(base + L.e2);
  double* E3 = (double*)(base + L.e3);
  double* dP1d = (double*)(base + L.dp1d);
  double* dP2Td = (double*)(base + L.dp2td);
  double* dXT = (double*)(base + L.dxt);
  double* du2t = (double*)(base + L.du2t);
  double* mbuf = (double*)(base + L.mbuf);
  double* dGs = (double*)(base + L.dgs);
  double* dXs = (double*)(base + L.dxs);
  const int n = p.n, N = p.N, nP = p.nP, NP = p.NP, nt = p.n_tau, nw = p.n_omega;
  const long NPnP = (long)NP * nP;
  const int ldk = L.ldk;
  if (NP % 64 != 0) return fail(SOX_ERR_SHAPE, "internal: padded extent does not fit the tiles");
  sox_status st;
  if ((st = launch_fill<double>(dGs, (long)nt * n * n, s))) return st;
  if ((st = launch_fill<double>(dXs, (long)n * N, s))) return st;
  if ((st = launch_fill<double>(du2t, NPnP * nP, s))) return st;
  if ((st = launch_fill<double>(dXT, (long)nt * NPnP, s))) return st;
  if ((st = launch_fill<double>(dW2, (long)nw * 4 * NP * NP, s))) return st;
  if ((st = launch_fill<double>(dP1d, (long)nt * NPnP, s))) return st;
  if ((st = launch_fill<double>(dP2Td, (long)nt * NPnP, s))) return st;
  // forward pass: every intermediate of the plain entry, and D for all tau
  if ((st = run_dynamic<T>(p, X, Wtau, V, G, nullptr, ws, s, vcw, W2T))) return st;
  ProfScope ps(p, SOX_STAGE_VJP, s);
  {
    const long cx = (long)nP * NP;
    hipLaunchKernelGGL(xpad_kernel<T>, grid1d(cx), dim3(256), 0, s, X, XP,
                       n, N, nP, NP);
    SOX_HIP(hipGetLastError());
    UTensorProb<T> pr{V, X, u2tT, n, N, nP, NP, nP * nP, N, 1, NP};
    SOX_HIP((launch_gemm<UTensorProb<T>, double, 2, 2, 2, 2>(pr, 1, s)));
    if ((st = launch_transpose<T>(P2T, P2, NP, nP, nt, s))) return st;
  }
  // cotangent of D for all tau, and the back-transform's dX terms
  RXProb rx{R, X, E2, n, N, NP, 0, 0, n, N, n};
  SOX_HIP((launch_gemm<RXProb, double, 2, 2, 2, 2>(rx, nt, s)));
  RXProb rx3{R, X, E3, n, N, NP, 0, 1, n, N, n};
  SOX_HIP((launch_gemm<RXProb, double, 2, 2, 2, 2>(rx3, nt, s)));
  DDProb<T> ddp{X, E2, dD, dDT, n, N, NP, NP, NP, n};
  SOX_HIP((launch_gemm<DDProb<T>, double, 2, 2, 2, 2>(ddp, nt, s)));
  DXBackProb<T> b1{E2, D, dXs, n, N, NP, 0, n, N, nt * NP};
  SOX_HIP((launch_gemm<DXBackProb<T>, double, 2, 2, 2, 2>(b1, 1, s)));
  DXBackProb<T> b2{E3, D, dXs, n, N, NP, 1, n, N, nt * NP};
  SOX_HIP((launch_gemm<DXBackProb<T>, double, 2, 2, 2, 2>(b2, 1, s)));

  for (int v0 = 0; v0 < n; v0 += vcw) {
    const int vc = std::min(vcw, n - v0);
    const long vcn = (long)vc * n;
    // recompute GG(Omega) (both layouts), A(Omega), A(tau) for the slab
    if ((st = launch_fill<T>(GG2T, (long)nw * 2 * NP * ldk, s))) return st;
    if ((st = launch_fill<T>(dAW, (long)nw * 2 * NP * ldk, s))) return st;
    // the forward pass's Q-contiguous copies of P1 and P2^T are still in
    // the workspace
    FTProb<T> ft{p.d_tf2, (const double*)(base + F.p1q), (const double*)(base + F.p2q), GG2, n, nP,
                 NP, N, nw, nt, v0, vc, 2 * nw, vc * n * NP, nt, GG2T, ldk, 1};
    SOX_HIP(launch_ft<T>(ft, p.n_cu, s));
    if ((st = launch_wgg<T>(W2, GG2, AW, NP, vcn, nw, s))) return st;
    IFTProb<T> ift{p.d_tb2, AW, Adyn, n, nP, NP, nw, nt, vc, nt, NP * vc * nP, 2 * nw};
    SOX_HIP(launch_ift<T>(ift, p.n_cu, s));
    if ((st = launch_transpose<T>(Adyn, AdynT, NP, nP, (long)nt * vc, s))) return st;
    // Hadamard-contract adjoints with B^v = A^v X
    HcArgs<T, double> h{};
    h.nz = NP; h.nk = nP; h.ny = nP;
    // dAdyn[tau][vl][P][u] = sum_R dD[P,R] C[R,v,P] X[u,R]
    h.L = U2 + (long)v0 * nP; h.l_ld = (long)nP * nP; h.l_ts = 0; h.l_vs = nP;
    h.Rm = P2T; h.r_ld = nP; h.r_ts = NPnP; h.r_vs = 0;
    h.W = dDT; h.w_ld = NP; h.w_ts = (long)NP * NP;
    h.FT = XP; h.f_ld = NP; h.f_ts = 0; h.f_vs = 0;
    h.Out = dAdyn; h.o_ld = nP; h.o_ts = (long)vc * NPnP; h.o_vs = NPnP;
    h.n_ot = nt; h.n_ov = vc; h.n_it = 1; h.n_iv = 1; h.accumulate = 0;
    if ((st = launch_hc_cfg<T>(p, h, NP, s))) return st;
    // dX^T[tau][R][u] += sum_{P,v} dD[P,R] C[R,v,P] A[tau][v][P][u]
    h.L = P2T; h.l_ld = nP; h.l_ts = NPnP; h.l_vs = 0;
    h.Rm = U2 + (long)v0 * nP; h.r_ld = (long)nP * nP; h.r_ts = 0; h.r_vs = nP;
    h.W = dD;
    h.FT = AdynT; h.f_ld = NP; h.f_ts = (long)vc * NPnP; h.f_vs = NPnP;
    h.Out = dXT; h.o_ld = nP; h.o_ts = NPnP; h.o_vs = 0;
    h.n_ot = nt; h.n_ov = 1; h.n_it = 1; h.n_iv = vc; h.accumulate = 1;
    if ((st = launch_hc_cfg<T>(p, h, NP, s))) return st;
    // dU2[v][R][w] += sum_{tau,P} dD[P,R] B[P,R,v] G_wP[w,P]
    h.L = Adyn; h.l_ld = nP; h.l_ts = (long)vc * NPnP; h.l_vs = NPnP;
    h.Rm = XT; h.r_ld = nP; h.r_ts = 0; h.r_vs = 0;
    h.W = dD;
    h.FT = P2; h.f_ld = NP; h.f_ts = NPnP; h.f_vs = 0;
    h.Out = du2t + (long)v0 * NPnP; h.o_ld = nP; h.o_ts = 0; h.o_vs = NPnP;
    h.n_ot = 1; h.n_ov = vc; h.n_it = nt; h.n_iv = 1; h.accumulate = 1;
    if ((st = launch_hc_cfg<T>(p, h, NP, s))) return st;
    // dG_wP^T[tau][P][w] += sum_{R,v} dD[P,R] B[P,R,v] U2[R,v,w]
    h.L = XT; h.l_ld = nP; h.l_ts = 0; h.l_vs = 0;
    h.Rm = Adyn; h.r_ld = nP; h.r_ts = (long)vc * NPnP; h.r_vs = NPnP;
    h.W = dDT;
    h.FT = u2tT + (long)v0 * NPnP; h.f_ld = NP; h.f_ts = 0; h.f_vs = NPnP;
    h.Out = dP2Td; h.o_ld = nP; h.o_ts = NPnP; h.o_vs = 0;
    h.n_ot = nt; h.n_ov = 1; h.n_it = 1; h.n_iv = vc; h.accumulate = 1;
    if ((st = launch_hc_cfg<T>(p, h, NP, s))) return st;
    // IFT adjoint, then the adjoints of A(Omega) = W2 GG2
    IFTAdjProb<T> ia{p.d_tb2, dAdyn, dAW, dAWT, n, nP, NP, nw, nt, vc, ldk, 2 * nw,
                     NP * vc * n, nt};
    SOX_HIP((launch_gemm<IFTAdjProb<T>, double, 2, 2, 2, 2>(ia, 1, s)));
    if (sizeof(T) == 4) {
      // float32 on the LDS-staged GEMM, results stored or accumulated in float64
      DenseLdsArgs d{};
      d.A = (const float*)dAW; d.B = (const float*)GG2T; d.C64 = dW2;
      d.lda = ldk; d.ldb = ldk; d.ldc = 2L * NP;
      d.sA = 2L * NP * ldk; d.sB = 2L * NP * ldk; d.sC = 4L * NP * NP;
      d.M = 2 * NP; d.N = 2 * NP; d.K = ldk; d.accumulate = 1;
      d.rgroup = d.M; d.rvalid = d.M;
      SOX_HIP(launch_dense_lds_f32(d, nw, s));
      DenseLdsArgs e{};
      e.A = (const float*)dAWT; e.B = (const float*)W2T; e.C64 = dGG2;
      e.lda = 2L * NP; e.ldb = 2L * NP; e.ldc = 2L * NP;
      e.sA = vcn * 2 * NP; e.sB = 4L * NP * NP; e.sC = vcn * 2 * NP;
      e.M = (int)vcn; e.N = 2 * NP; e.K = 2 * NP;
      e.rgroup = e.M; e.rvalid = e.M;
      SOX_HIP(launch_dense_lds_f32(e, nw, s));
    } else {
      DenseArgs<T, double> d{};
      d.A = dAW; d.B = GG2T; d.C = dW2;
      d.lda = ldk; d.ldb = ldk; d.ldc = 2L * NP;
      d.sA = 2L * NP * ldk; d.sB = 2L * NP * ldk; d.sC = 4L * NP * NP;
      d.M = 2 * NP; d.N = 2 * NP; d.K = ldk; d.alpha = T(1); d.accumulate = 1;
      SOX_HIP((launch_dense<T, double, 2, 2, 2, 2>(d, nw, s)));
      DenseArgs<T, double> e{};
      e.A = dAWT; e.B = W2T; e.C = dGG2;
      e.lda = 2L * NP; e.ldb = 2L * NP; e.ldc = 2L * NP;
      e.sA = vcn * 2 * NP; e.sB = 4L * NP * NP; e.sC = vcn * 2 * NP;
      e.M = (int)vcn; e.N = 2 * NP; e.K = 2 * NP; e.alpha = T(1); e.accumulate = 0;
      SOX_HIP((launch_dense<T, double, 2, 2, 2, 2>(e, nw, s)));
    }
    FTAdjProb fa{p.d_tf2, dGG2, dGG, n, NP, nw, nt, vc, nt, vc * n * NP, 2 * nw};
    SOX_HIP((launch_gemm<FTAdjProb, double, 2, 2, 2, 2>(fa, 1, s)));
    {
      const long c2 = (long)nt * N * n, c1 = (long)nt * N * vc;
      hipLaunchKernelGGL(gg_adjoint_p2_kernel, grid1d(c2), dim3(256), 0, s,
                         dGG, P1d, dP2Td, n, nP, NP, N, nt, v0, vc);
      SOX_HIP(hipGetLastError());
      hipLaunchKernelGGL(gg_adjoint_p1_kernel, grid1d(c1), dim3(256), 0, s,
                         dGG, P2Td, dP1d, n, nP, NP, N, nt, v0, vc);
      SOX_HIP(hipGetLastError());
    }
  }
  if (dW) {
    DWtauProb dwp{p.d_tf2, dW2, dW, N, NP, nw, nt, nt, N * N, 2 * nw};
    SOX_HIP((launch_gemm<DWtauProb, double, 2, 2, 2, 2>(dwp, 1, s)));
  }
  if (dV) {
    DUProb a2{du2t, X, dV, n, N, nP, NP, 1, 0, N, N, nP * nP};
    SOX_HIP((launch_gemm<DUProb, double, 2, 2, 2, 2>(a2, 1, s)));
  }
  const long nx = (long)n * N;
  DUMProb m2{V, du2t, mbuf, n, N, nP, NP, 1, N, nP * nP, N};
  SOX_HIP((launch_gemm<DUMProb, double, 2, 2, 2, 2>(m2, 1, s)));
  hipLaunchKernelGGL(ut_adjoint_x_kernel, grid1d(nx), dim3(256), 0, s, mbuf,
                     X, dXs, n, N, nP);
  SOX_HIP(hipGetLastError());
  for (int t = 0; t < nt; ++t) {
    hipLaunchKernelGGL(add_transposed_kernel, grid1d(nx), dim3(256), 0, s,
                       dXT + (long)t * NPnP, dXs, n, N, nP);
    SOX_HIP(hipGetLastError());
  }
  DGProjProb g1{X, dP1d, dGs, n, N, nP, NP, 0, 0, n, n, N};
  SOX_HIP((launch_gemm<DGProjProb, double, 2, 2, 2, 2>(g1, nt, s)));
  DGProjProb g2{X, dP2Td, dGs, n, N, nP, NP, 0, 1, n, n, N};
  SOX_HIP((launch_gemm<DGProjProb, double, 2, 2, 2, 2>(g2, nt, s)));
  DXProjProb x1{G, dP1d, dXs, n, N, nP, NP, 0, 0, n, N, nt * nP};
  SOX_HIP((launch_gemm<DXProjProb, double, 2, 2, 2, 2>(x1, 1, s)));
  DXProjProb x2{G, dP2Td, dXs, n, N, nP, NP, 0, 1, n, N, nt * nP};
  SOX_HIP((launch_gemm<DXProjProb, double, 2, 2, 2, 2>(x2, 1, s)));
  if (dG) SOX_HIP(hipMemcpyAsync(dG, dGs, sizeof(double) * nt * n * n, hipMemcpyDeviceToDevice, s));
  if (dX) SOX_HIP(hipMemcpyAsync(dX, dXs, sizeof(double) * nx, hipMemcpyDeviceToDevice, s));
  return SOX_OK;
}

// Run `body` on `s`, or capture it once into a graph keyed by `key` and
// replay the graph on later calls with the same key.
template <typename F>
sox_status run_maybe_graph(sox_plan& p, const uintptr_t (&key)[9], hipStream_t s, F&& body) {
  if (!p.graph_on) return body(s);
  for (auto& g : p.graphs) {
    if (std::equal(key, key + 9, g.key)) {
      SOX_HIP(hipGraphLaunch(g.exec, s));
      return SOX_OK;
    }
  }
  if (!p.cap_stream) SOX_HIP(hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking));
  const bool prof = p.prof_on;
  p.prof_on = false;
  SOX_HIP(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
  sox_status st = body(p.cap_stream);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(p.cap_stream, &graph);
  p.prof_on = prof;
  if (st != SOX_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(SOX_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(SOX_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
  }
  if (p.graphs.size() >= 16) {
    (void)hipGraphExecDestroy(p.graphs.front().exec);
    (void)hipGraphDestroy(p.graphs.front().graph);
    p.graphs.erase(p.graphs.begin());
  }
  sox_plan::GraphEntry ge{};
  std::copy(key, key + 9, ge.key);
  ge.graph = graph;
  ge.exec = exec;
  p.graphs.push_back(ge);
  SOX_HIP(hipGraphLaunch(exec, s));
  return SOX_OK;
}

void drop_graphs(sox_plan& p) {
  for (auto& g : p.graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  p.graphs.clear();
}

// Autotuner of the fused kernel's wave tile: time every admissible shape on
// zero-filled operands of the plan's shape (up to 8 tau nodes).
template <typename T>
sox_status time_fused_cfg(sox_plan& p, int cfg, int tt, double* ms_per_tau) {
  set_fused_cfg(p, cfg);
  const FusedCfg& fc = kFusedCfgs[cfg];
  const long nP = p.nP, NP = p.NP, n = p.n;
  const size_t es = sizeof(T);
  const size_t szA = tt * n * NP * nP, szY = tt * NP * nP, szU = NP * nP * nP, szD = tt * NP * NP;
  T* buf = nullptr;
  const size_t total = szA + 2 * szY + szU + szD;
  hipError_t e = hipMalloc(&buf, total * es);
  if (e != hipSuccess) return fail(SOX_ERR_OOM, "autotune buffers: %s", hipGetErrorString(e));
  hipLaunchKernelGGL(fill_kernel<T>, grid1d(total), dim3(256), 0, nullptr,
                     buf, (long)total, T(0));
  FusedArgs<T> fa;
  fa.A = buf; fa.Y = buf + szA; fa.P2T = buf + szA + szY; fa.U2 = buf + szA + 2 * szY;
  fa.D = buf + szA + 2 * szY + szU;
  fa.a_tstride = n * NP * nP; fa.a_vstride = NP * nP; fa.y_tstride = NP * nP; fa.p_tstride = NP * nP;
  fa.u_rstride = nP * nP; fa.u_vstride = nP; fa.d_tstride = NP * NP;
  fa.accumulate = 0; fa.n = (int)n; fa.nP = (int)nP; fa.NP = (int)NP;
  fa.tiles_p = (int)(NP / (2 * fc.wp)); fa.tiles_r = (int)(NP / (2 * fc.wr)); fa.n_tau = tt;
  hipEvent_t a = nullptr, b = nullptr;
  sox_status st = SOX_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) st = SOX_ERR_HIP;
  if (!st) st = launch_fused_cfg<T>(p, fa, nullptr);
  if (!st && hipEventRecord(a, nullptr) != hipSuccess) st = SOX_ERR_HIP;
  for (int r = 0; r < 3 && !st; ++r) st = launch_fused_cfg<T>(p, fa, nullptr);
  float ms = 0.f;
  if (!st && hipEventRecord(b, nullptr) != hipSuccess) st = SOX_ERR_HIP;
  if (!st && hipEventSynchronize(b) != hipSuccess) st = SOX_ERR_HIP;
  if (!st && hipEventElapsedTime(&ms, a, b) != hipSuccess) st = SOX_ERR_HIP;
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(buf);
  if (st) return st == SOX_ERR_HIP ? fail(SOX_ERR_HIP, "autotune launch failed") : st;
  *ms_per_tau = ms / (3.0 * tt);
  return SOX_OK;
}

std::string tune_key(const sox_plan& p) {
  char k[96];
  snprintf(k, sizeof(k), "fused %d %d %d", p.precision, p.n, p.N);
  return k;
}

sox_status autotune_fused(sox_plan& p) {
  const char* cache = getenv("SOX_TUNE_CACHE");
  const std::string key = tune_key(p);
  if (cache) {
    if (FILE* f = fopen(cache, "r")) {
      char line[160];
      int found = -1;
      while (fgets(line, sizeof(line), f)) {
        int cfg;
        char k[96];
        int prec, n, N;
        if (sscanf(line, "%95s %d %d %d %d", k, &prec, &n, &N, &cfg) == 5) {
          char full[96];
          snprintf(full, sizeof(full), "%s %d %d %d", k, prec, n, N);
          if (key == full && cfg_usable(p, cfg)) found = cfg;
        }
      }
      fclose(f);
      if (found >= 0) {
        set_fused_cfg(p, found);
        p.tune_from_cache = true;
        return SOX_OK;
      }
    }
  }
  const int tt = std::min(p.n_tau, 8);
  int best = p.fused_cfg;
  double best_ms = 1e300;
  p.tune_ms.clear();
  for (int c = 0; c < kNumFusedCfgs; ++c) {
    if (!cfg_usable(p, c)) continue;
    double ms = 0;
    sox_status st = p.precision == SOX_FP64 ? time_fused_cfg<double>(p, c, tt, &ms)
                                            : time_fused_cfg<float>(p, c, tt, &ms);
    if (st) return st;
    p.tune_ms.push_back({c, ms});
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  set_fused_cfg(p, best);
  if (cache) {
    if (FILE* f = fopen(cache, "a")) {
      fprintf(f, "%s %d\n", key.c_str(), best);
      fclose(f);
    }
  }
  return SOX_OK;
}

#include "sox_solid_run.hpp"

sox_status dispatch_static(sox_plan* plan, int entry, const double* X, const double* U1,
                           const double* U2, const double* G, double* Sigma, void* ws,
                           size_t ws_bytes, void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (!X || !U1 || !G || !Sigma || (entry == SOX_ENTRY_STATIC && !U2))
    return fail(SOX_ERR_INVALID_ARG, "NULL tensor pointer");
  st = check_ws(plan, entry, ws, ws_bytes);
  if (st) return st;
  const uintptr_t key[9] = {(uintptr_t)entry, (uintptr_t)X, (uintptr_t)U1, (uintptr_t)U2,
                            (uintptr_t)G, (uintptr_t)Sigma, (uintptr_t)ws, (uintptr_t)ws_bytes, 0};
  return run_maybe_graph(*plan, key, (hipStream_t)stream, [&](hipStream_t s) -> sox_status {
    if (plan->nk > 1) {
      if (plan->precision == SOX_FP64)
        return run_solid<double>(*plan, entry, X, U1, U2, G, Sigma, ws, s);
      return run_solid<float>(*plan, entry, X, U1, U2, G, Sigma, ws, s);
    }
    switch (plan->precision) {
      case SOX_FP64: return run_static<double>(*plan, entry, X, U1, U2, G, Sigma, ws, s);
      case SOX_FP32:
      case SOX_BF16X3: return run_static<float>(*plan, entry, X, U1, U2, G, Sigma, ws, s);
      default:
        return fail(SOX_ERR_UNSUPPORTED, "unknown precision %d", plan->precision);
    }
  });
}

// -- composite vertex self-energies (fig:diag) ---------------------------------
// The composites are sums of SOX terms with one interaction per line.  The
// library runs the terms it needs and sums them on the device:
//   SOSEX_STAT   SOX(W0, V)                       one static pass
//   G3W2_STAT    SOX(W0, W0)                      one static pass
//   2SOSEX_STAT  SOX(V,V) + SOX(V,Wd0) + SOX(Wd0,V)
//                = SOX(V, W0) + SOX(W0 - V, V)    two static passes (bilinear)
//   SOSEX_DYN    SOX(V,V) + SOX(W_d(tau),V)       solids: one pass with the bare
//                term in the dynamic chain; molecules: bare + dynamic pass
//   2SOSEX_DYN   SOX(V,V) + SOX(V,W_d) + SOX(W_d,V), with SOX(V, W_d) = SOX(W_d, V)^T
//                (molecules) or ^dagger per (k, tau) (solids): the mirror image of the
//                diagram for a symmetric (Hermitian) G(tau)
// Workspace: the largest pass, then one Sigma-sized buffer and one
// interaction-sized buffer (W0 - V).
struct VertexLayout {
  size_t pass, sig, wd0, total;
};

VertexLayout vertex_layout_for(const sox_plan& p) {
  VertexLayout L{};
  size_t pass = std::max(workspace_bytes(p, SOX_ENTRY_STATIC), workspace_bytes(p, SOX_ENTRY_BARE));
  if (p.n_omega > 0) {
    pass = std::max(pass, workspace_bytes(p, SOX_ENTRY_DYNAMIC));
    if (p.nk > 1) pass = std::max(pass, solid_dyn_total(p, true));
  }
  const size_t cplx = p.nk > 1 ? 2 * (size_t)p.nk : 1;
  Carver c;
  L.pass = c.take(pass);
  L.sig = c.take(cplx * p.n_tau * p.n * p.n * sizeof(double));
  L.wd0 = c.take(cplx * p.N * p.N * sizeof(double));
  L.total = c.off;
  return L;
}

size_t vertex_workspace_bytes(const sox_plan& p) { return vertex_layout_for(p).total; }

__global__ void vertex_axpby_kernel(double* out, const double* a, double alpha, const double* b,
                                    double beta, long count) {
  SOX_FOR_FLAT(i, count) out[i] = alpha * a[i] + beta * b[i];
}

// out[z][i][j] += a[z][j][i] (real) or conj(a[z][j][i]) (complex), z < batch
__global__ void vertex_add_adjoint_kernel(double* out, const double* a, long batch, int n,
                                          int cplx) {
  const long per = (long)n * n;
  SOX_FOR_FLAT(idx, batch * per) {
    const long z = idx / per;
    const int i = (int)((idx - z * per) / n), j = (int)(idx - z * per - (long)i * n);
    const long src = z * per + (long)j * n + i;
    if (cplx) {
      out[2 * idx] += a[2 * src];
      out[2 * idx + 1] -= a[2 * src + 1];
    } else {
      out[idx] += a[src];
    }
  }
}

sox_status vertex_pass_static(sox_plan& p, int entry, const double* X, const double* U1,
                              const double* U2, const double* G, double* out, void* ws,
                              hipStream_t s) {
  if (p.nk > 1)
    return p.precision == SOX_FP64 ? run_solid<double>(p, entry, X, U1, U2, G, out, ws, s)
                                   : run_solid<float>(p, entry, X, U1, U2, G, out, ws, s);
  return p.precision == SOX_FP64 ? run_static<double>(p, entry, X, U1, U2, G, out, ws, s)
                                 : run_static<float>(p, entry, X, U1, U2, G, out, ws, s);
}

sox_status vertex_pass_dynamic(sox_plan& p, const double* X, const double* W, const double* V,
                               const double* G, double* out, void* ws, hipStream_t s,
                               bool with_bare, bool real_w) {
  if (p.nk > 1)
    return p.precision == SOX_FP64
               ? run_solid_dynamic<double>(p, X, W, V, G, out, ws, s, with_bare)
               : run_solid_dynamic<float>(p, X, W, V, G, out, ws, s, with_bare);
  return p.precision == SOX_FP64
             ? run_dynamic<double>(p, X, W, V, G, out, ws, s)
             : run_dynamic<float>(p, X, W, V, G, out, ws, s, 0, nullptr, real_w);
}

sox_status run_vertex(sox_plan& p, int kind, const double* X, const double* V, const double* W,
                      const double* G, double* Sigma, void* ws, hipStream_t s, bool real_w) {
  const VertexLayout L = vertex_layout_for(p);
  char* base = (char*)ws;
  void* pw = base + L.pass;
  double* tmp = (double*)(base + L.sig);
  double* wd0 = (double*)(base + L.wd0);
  const long cplx = p.nk > 1 ? 2L * p.nk : 1L;
  const long nsig = cplx * p.n_tau * p.n * p.n;
  const long nint = cplx * p.N * p.N;
  const long batch = (long)(p.nk > 1 ? p.nk : 1) * p.n_tau;
  sox_status st;
  auto add = [&](double* out, const double* a) -> sox_status {
    hipLaunchKernelGGL(vertex_axpby_kernel, grid1d(nsig), dim3(256), 0, s, out, out, 1.0, a, 1.0,
                       nsig);
    SOX_HIP(hipGetLastError());
    return SOX_OK;
  };
  auto add_adjoint = [&](double* out, const double* a) -> sox_status {
    hipLaunchKernelGGL(vertex_add_adjoint_kernel, grid1d(batch * p.n * p.n), dim3(256), 0, s, out,
                       a, batch, p.n, p.nk > 1 ? 1 : 0);
    SOX_HIP(hipGetLastError());
    return SOX_OK;
  };
  switch (kind) {
    case SOX_VERTEX_SOSEX_STAT:
      return vertex_pass_static(p, SOX_ENTRY_STATIC, X, W, V, G, Sigma, pw, s);
    case SOX_VERTEX_G3W2_STAT:
      return vertex_pass_static(p, SOX_ENTRY_STATIC, X, W, W, G, Sigma, pw, s);
    case SOX_VERTEX_2SOSEX_STAT: {
      // SOX(V, W0) + SOX(W0 - V, V)
      if ((st = vertex_pass_static(p, SOX_ENTRY_STATIC, X, V, W, G, Sigma, pw, s))) return st;
      hipLaunchKernelGGL(vertex_axpby_kernel, grid1d(nint), dim3(256), 0, s, wd0, W, 1.0, V, -1.0,
                         nint);
      SOX_HIP(hipGetLastError());
      if ((st = vertex_pass_static(p, SOX_ENTRY_STATIC, X, wd0, V, G, tmp, pw, s))) return st;
      return add(Sigma, tmp);
    }
    case SOX_VERTEX_SOSEX_DYN:
      if (p.nk > 1) return vertex_pass_dynamic(p, X, W, V, G, Sigma, pw, s, true, real_w);
      if ((st = vertex_pass_static(p, SOX_ENTRY_BARE, X, V, V, G, Sigma, pw, s))) return st;
      if ((st = vertex_pass_dynamic(p, X, W, V, G, tmp, pw, s, false, real_w))) return st;
      return add(Sigma, tmp);
    case SOX_VERTEX_2SOSEX_DYN:
      // SOX(W_d, V) into tmp; SOX(V, V) + SOX(W_d, V) into Sigma; then the mirror term
      if ((st = vertex_pass_dynamic(p, X, W, V, G, tmp, pw, s, false, real_w))) return st;
      if (p.nk > 1) {
        if ((st = vertex_pass_dynamic(p, X, W, V, G, Sigma, pw, s, true, real_w))) return st;
      } else {
        if ((st = vertex_pass_static(p, SOX_ENTRY_BARE, X, V, V, G, Sigma, pw, s))) return st;
        if ((st = add(Sigma, tmp))) return st;
      }
      return add_adjoint(Sigma, tmp);
    default:
      return fail(SOX_ERR_INVALID_ARG, "unknown vertex kind %d", kind);
  }
}

// -- THC-GW direct term (sox_gw.hpp) ---------------------------------------------
// Float64 buffers of one tau slab of c nodes (complex for meshes, every
// momentum): the half projection G_Rl, the second projection Gt (meshes
// only: molecules fold the elementwise product into it), M and Y = X M.
struct GwLayout {
  size_t p1, gt, m, y, total;
};

GwLayout gw_layout_for(const sox_plan& p, int c) {
  GwLayout L{};
  const size_t es = p.nk > 1 ? 16 : 8;
  const size_t nk = p.nk, n = p.n, N = p.N, cc = c;
  Carver k;
  L.p1 = k.take(nk * cc * N * n * es);
  L.gt = p.nk > 1 ? k.take(nk * cc * N * N * es) : 0;
  L.m = k.take(nk * cc * N * N * es);
  L.y = k.take(nk * cc * n * N * es);
  L.total = k.off;
  return L;
}

// tau nodes per slab: all of them if the buffers fit the workspace budget,
// else halved until they do (at least one)
int gw_slab(const sox_plan& p) {
  const size_t budget = ws_budget();
  int c = p.n_tau;
  while (c > 1 && gw_layout_for(p, c).total > budget) c = (c + 1) / 2;
  return c;
}

size_t gw_workspace_bytes(const sox_plan& p) { return gw_layout_for(p, gw_slab(p)).total; }

// the molecular chain for nodes t0 .. t0 + cnt - 1 of G and W (one slab)
sox_status gw_mol_slab(const sox_plan& p, const double* X, const double* W, const double* G,
                       double* Sigma, int t0, int cnt, double* p1, double* m, double* y,
                       hipStream_t s) {
  const int n = p.n, N = p.N;
  ProjP1Prob<double> pr1{X, G, p1, n, N, n, N, t0, N, n, n};
  SOX_HIP((launch_gemm<ProjP1Prob<double>, double, 2, 2, 2, 2>(pr1, cnt, s)));
  GwHadProb had{p1, X, W, m, n, N, t0, N, N, n};
  SOX_HIP((launch_gemm<GwHadProb, double, 2, 2, 2, 2>(had, cnt, s)));
  GwLeftProb left{X, m, y, n, N, n, N, N};
  SOX_HIP((launch_gemm<GwLeftProb, double, 2, 2, 2, 2>(left, cnt, s)));
  GwRightProb right{y, X, Sigma, n, N, t0, n, n, N};
  SOX_HIP((launch_gemm<GwRightProb, double, 2, 2, 2, 2>(right, cnt, s)));
  return SOX_OK;
}

sox_status run_gw(sox_plan& p, const double* X, const double* W, const double* G, double* Sigma,
                  void* ws, hipStream_t s) {
  const int c = gw_slab(p);
  const GwLayout L = gw_layout_for(p, c);
  char* base = (char*)ws;
  double* p1 = (double*)(base + L.p1);
  double* gt = (double*)(base + L.gt);
  double* m = (double*)(base + L.m);
  double* y = (double*)(base + L.y);
  const int n = p.n, N = p.N, nt = p.n_tau, nk = p.nk;
  ProfScope ps(p, SOX_STAGE_GW, s);
  for (int t0 = 0; t0 < nt; t0 += c) {
    const int cnt = std::min(c, nt - t0);
    if (nk == 1) {
      sox_status st = gw_mol_slab(p, X, W, G, Sigma, t0, cnt, p1, m, y, s);
      if (st) return st;
      continue;
    }
    const int nz = nk * cnt;
    const long cN = (long)c * N;
    // G_Rl^k = sum_j X^k_jR G^k_jl
    CgArgs<double, double> a = cg_args<double, double>();
    a.A = X, a.ldA = 1, a.ksA = N, a.soA = (long)n * N;
    a.B = G + 2 * (long)t0 * n * n, a.ldB = 1, a.ksB = n, a.soB = (long)nt * n * n,
    a.siB = (long)n * n;
    a.C = p1, a.ldc = n, a.soC = cN * n, a.siC = (long)N * n;
    a.M = N, a.N = n, a.K = n, a.nzi = cnt;
    sox_status st = cg_launch(a, nz, 0, s);
    if (st) return st;
    // Gt^k[R][Q] = sum_l G_Rl^k conj(X^k_lQ)
    a = cg_args<double, double>();
    a.A = p1, a.ldA = n, a.soA = cN * n, a.siA = (long)N * n;
    a.B = X, a.ldB = 1, a.ksB = N, a.soB = (long)n * N, a.conjB = 1;
    a.C = gt, a.ldc = N, a.soC = cN * N, a.siC = (long)N * N;
    a.M = N, a.N = N, a.K = n, a.nzi = cnt;
    if ((st = cg_launch(a, nz, 0, s))) return st;
    // M^k = -(1/N_k) sum_k' W^{k-k'} Gt^{k'}: registers for the meshes of the
    // templated D step, the LDS kernel for any other
    const long NN = (long)N * N;
    bool done = false;
    const int* mc = p.mesh_canon;
#define SOX_GWCONV(A_, B_, C_)                                                               \
    if (!done && mc[0] == A_ && mc[1] == B_ && mc[2] == C_) {                                \
      hipLaunchKernelGGL((gw_conv_mesh_kernel<A_, B_, C_>), grid1d(NN * cnt), dim3(256), 0, s, \
                         W, gt, m, NN, c, t0, nt, -1.0 / nk, NN * cnt);                     \
      SOX_HIP(hipGetLastError());                                                          \
      done = true;                                                                         \
    }
    SOX_GWCONV(2, 1, 1)
    SOX_GWCONV(3, 1, 1)
    SOX_GWCONV(2, 2, 1)
    SOX_GWCONV(2, 3, 1)
    SOX_GWCONV(3, 2, 1)
    SOX_GWCONV(3, 3, 1)
    SOX_GWCONV(2, 2, 2)
    SOX_GWCONV(3, 3, 3)
#undef SOX_GWCONV
    if (!done) {
      const int E = gw_conv_width(nk);
      const long nblk = (NN + E - 1) / E;
      if (!grid_fits(nblk * cnt, 256))
        return fail(SOX_ERR_SHAPE, "GW convolution grid too large");
      hipLaunchKernelGGL(gw_conv_kernel, dim3((unsigned)(nblk * cnt)), dim3(256), 0, s, W, gt, m,
                         p.d_ktab + 3 * (size_t)nk * nk, nk, E, NN, c, t0, nt, -1.0 / nk, nblk);
      SOX_HIP(hipGetLastError());
    }
    // Y^k[i][Q] = sum_R conj(X^k_iR) M^k[R][Q]
    a = cg_args<double, double>();
    a.A = X, a.ldA = N, a.soA = (long)n * N, a.conjA = 1;
    a.B = m, a.ldB = 1, a.ksB = N, a.soB = cN * N, a.siB = (long)N * N;
    a.C = y, a.ldc = N, a.soC = cN * n, a.siC = (long)n * N;
    a.M = n, a.N = N, a.K = N, a.nzi = cnt;
    if ((st = cg_launch(a, nz, 0, s))) return st;
    // Sigma^k[i][j] = sum_Q Y^k[i][Q] X^k_jQ
    a = cg_args<double, double>();
    a.A = y, a.ldA = N, a.soA = cN * n, a.siA = (long)n * N;
    a.B = X, a.ldB = N, a.soB = (long)n * N;
    a.C = Sigma + 2 * (long)t0 * n * n, a.ldc = n, a.soC = (long)nt * n * n, a.siC = (long)n * n;
    a.M = n, a.N = n, a.K = N, a.nzi = cnt;
    if ((st = cg_launch(a, nz, 0, s))) return st;
  }
  return SOX_OK;
}

// -- minimal self-consistent loop (sox_scf.hpp) -------------------------------------
sox_status queue_energy(sox_plan& p, const double* Sigma, const double* G, double* e,
                        double** slot, hipStream_t s);  // with the energy entry points

struct ScfLayout {
  size_t g, gn, sd, sd2, snu, gin, gam, shf, heff, exch, rho, v, tf, tb, tbeta, nu, bmax,
      scal, hf_p1, hf_m, hf_y, sub, total;
};
constexpr int kScfBlocks = 1024;  // blocks of the mixing reduction

size_t scf_sub_bytes(const sox_plan& p, int terms) {
  size_t b = 0;
  if (terms & 1) b = std::max(b, gw_workspace_bytes(p));
  if (terms & 2) b = std::max(b, workspace_bytes(p, SOX_ENTRY_BARE));
  return b;
}

ScfLayout scf_layout_for(const sox_plan& p, int n_nu, int terms) {
  ScfLayout L{};
  const size_t n = p.n, N = p.N, nt = p.n_tau, nn = n * n, nm = n_nu;
  Carver c;
  L.g = c.take(nt * nn * 8);
  L.gn = c.take(nt * nn * 8);
  L.sd = c.take(nt * nn * 8);
  L.sd2 = c.take(nt * nn * 8);
  L.snu = c.take(2 * nm * nn * 8);
  L.gin = c.take(2 * nm * nn * 8);
  L.gam = c.take(nn * 8);
  L.shf = c.take(nn * 8);
  L.heff = c.take(nn * 8);
  L.exch = c.take(nn * 8);
  L.rho = c.take(N * 8);
  L.v = c.take(N * 8);
  L.tf = c.take(2 * nm * nt * 8);
  L.tb = c.take(2 * nt * nm * 8);
  L.tbeta = c.take(nt * 8);
  L.nu = c.take(nm * 8);
  L.bmax = c.take(kScfBlocks * 8);
  L.scal = c.take(8 * 8);
  L.hf_p1 = c.take(N * n * 8);
  L.hf_m = c.take(N * N * 8);
  L.hf_y = c.take(n * N * 8);
  L.sub = c.take(scf_sub_bytes(p, terms));
  L.total = c.off;
  return L;
}

sox_status run_scf(sox_plan& p, const sox_scf_params& prm, const double* X, const double* V,
                   const double* W, const double* h, const double* h_start, double* Gout,
                   sox_scf_result* res, void* ws, hipStream_t s) {
  const ScfLayout L = scf_layout_for(p, prm.n_nu, prm.terms);
  char* base = (char*)ws;
  auto P = [&](size_t off) { return (double*)(base + off); };
  double *g = P(L.g), *gn = P(L.gn), *sd = P(L.sd), *sd2 = P(L.sd2), *snu = P(L.snu);
  double *gin = P(L.gin), *gam = P(L.gam), *shf = P(L.shf), *heff = P(L.heff);
  double *exch = P(L.exch), *rho = P(L.rho), *v = P(L.v), *tf = P(L.tf), *tb = P(L.tb);
  double *tbeta = P(L.tbeta), *nu = P(L.nu), *bmax = P(L.bmax), *scal = P(L.scal);
  const int n = p.n, N = p.N, nt = p.n_tau, nm = prm.n_nu;
  const long nn = (long)n * n;
  SOX_HIP(hipMemcpyAsync(tf, prm.t_fwd, sizeof(double) * 2 * nm * nt, hipMemcpyHostToDevice, s));
  SOX_HIP(hipMemcpyAsync(tb, prm.t_bwd, sizeof(double) * 2 * nt * nm, hipMemcpyHostToDevice, s));
  SOX_HIP(hipMemcpyAsync(tbeta, prm.t_beta, sizeof(double) * nt, hipMemcpyHostToDevice, s));
  SOX_HIP(hipMemcpyAsync(nu, prm.nu, sizeof(double) * nm, hipMemcpyHostToDevice, s));
  SOX_HIP(hipStreamSynchronize(s));
  double hmax = 0.0;  // host bound on |h| for the mu bracket: read h once
  {
    std::vector<double> hh(nn);
    SOX_HIP(hipMemcpy(hh.data(), h_start ? h_start : h, sizeof(double) * nn, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) {
      double row = 0.0;
      for (int j = 0; j < n; ++j) row += std::fabs(hh[(size_t)i * n + j]);
      hmax = std::max(hmax, row);
    }
  }
  const double span = hmax + 50.0;
  // the Dyson matrices in LDS when they fit (SOX_SCF_DYSON_IN_MEMORY=1: in
  // device memory at any size, the form larger n takes)
  const char* dmem = getenv("SOX_SCF_DYSON_IN_MEMORY");
  const bool dyson_lds = n <= kScfLdsN && !(dmem && atoi(dmem) == 1);
  // N(mu) for the current heff and snu, G(tau) into out
  auto dyson = [&](double mu, double* out, double* count) -> sox_status {
    if (dyson_lds)
      hipLaunchKernelGGL(scf_dyson_kernel<true>, dim3(nm), dim3(kScfThreads), 0, s, heff, snu, nu,
                         mu, n, gin);
    else
      hipLaunchKernelGGL(scf_dyson_kernel<false>, dim3(nm), dim3(kScfThreads), 0, s, heff, snu, nu,
                         mu, n, gin);
    SOX_HIP(hipGetLastError());
    hipLaunchKernelGGL(scf_ift_kernel, grid1d((long)nt * nn), dim3(256), 0, s, tb, gin, nt, nm, nn,
                       out);
    SOX_HIP(hipGetLastError());
    if (count) {
      hipLaunchKernelGGL(scf_count_kernel, dim3(1), dim3(256), 0, s, out, tbeta, n, nt, scal);
      SOX_HIP(hipGetLastError());
      SOX_HIP(hipMemcpyAsync(count, scal, sizeof(double), hipMemcpyDeviceToHost, s));
      SOX_HIP(hipStreamSynchronize(s));
    }
    return SOX_OK;
  };
  // root of f(mu) = N(mu) - n_elec (increasing) in [lo, hi] with f(lo) <= 0
  // <= f(hi): Illinois regula falsi, a bisection step every fourth
  // evaluation, until the bracket is below 1e-12 (1 + |mu|) or f vanishes;
  // G at the final mu
  auto illinois = [&](double lo, double hi, double flo, double fhi, double* out,
                      double* mu_out) -> sox_status {
    sox_status q;
    if (flo == 0.0) hi = lo;
    if (fhi == 0.0) lo = hi;
    double mu = 0.5 * (lo + hi);
    int side = 0;
    for (int it = 0; it < 200 && flo < 0.0 && fhi > 0.0; ++it) {
      if (hi - lo <= 1e-12 * (1.0 + std::fabs(mu))) break;
      mu = (it % 4 == 3) ? 0.5 * (lo + hi) : (lo * fhi - hi * flo) / (fhi - flo);
      if (!(mu > lo && mu < hi)) mu = 0.5 * (lo + hi);
      double f = 0.0;
      if ((q = dyson(mu, out, &f))) return q;
      f -= prm.n_elec;
      if (f == 0.0) {
        lo = hi = mu;
        break;
      }
      if (f < 0.0) {
        lo = mu;
        flo = f;
        if (side < 0) fhi *= 0.5;
        side = -1;
      } else {
        hi = mu;
        fhi = f;
        if (side > 0) flo *= 0.5;
        side = 1;
      }
    }
    *mu_out = 0.5 * (lo + hi);
    return dyson(*mu_out, out, nullptr);
  };
  // the root within span of mu0: f at mu0 -/+ d, the side that does not
  // bracket moved out fourfold (the other end taking its place) until the
  // signs differ or span is reached, then the search above
  auto solve_mu = [&](double mu0, double d, double* out, double* mu_out) -> sox_status {
    sox_status q;
    d = std::min(d, span);
    double lo = mu0 - d, hi = mu0 + d, flo = 0.0, fhi = 0.0;
    if ((q = dyson(lo, out, &flo))) return q;
    flo -= prm.n_elec;
    if ((q = dyson(hi, out, &fhi))) return q;
    fhi -= prm.n_elec;
    while (flo > 0.0 && lo > mu0 - span) {
      hi = lo;
      fhi = flo;
      d = std::min(4.0 * d, span);
      lo = mu0 - d;
      if ((q = dyson(lo, out, &flo))) return q;
      flo -= prm.n_elec;
    }
    while (fhi < 0.0 && hi < mu0 + span) {
      lo = hi;
      flo = fhi;
      d = std::min(4.0 * d, span);
      hi = mu0 + d;
      if ((q = dyson(hi, out, &fhi))) return q;
      fhi -= prm.n_elec;
    }
    return illinois(lo, hi, flo, fhi, out, mu_out);
  };
  // start: G0 of h_start (or h), no self-energy
  SOX_HIP(hipMemcpyAsync(heff, h_start ? h_start : h, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
  sox_status st = launch_fill<double>(snu, 2L * nm * nn, s);
  if (st) return st;
  double mu = 0.0;
  if ((st = solve_mu(0.0, span, g, &mu))) return st;
  const long cnt = (long)nt * nn;
  const int nb = (int)std::min<long>(kScfBlocks, (cnt + 255) / 256);
  void* sub = base + L.sub;
  auto self_energy = [&]() -> sox_status {
    // gamma, Sigma^HF (exchange by the GW chain with W = V, G = gamma), heff
    hipLaunchKernelGGL(scf_density_kernel, grid1d(nn), dim3(256), 0, s, g, tbeta, n, nt, gam);
    SOX_HIP(hipGetLastError());
    sox_status q = gw_mol_slab(p, X, V, gam, exch, 0, 1, P(L.hf_p1), P(L.hf_m), P(L.hf_y), s);
    if (q) return q;
    hipLaunchKernelGGL(scf_rho_kernel, dim3((N + 63) / 64), dim3(kScfThreads), 0, s, X, gam, n, N,
                       rho);
    SOX_HIP(hipGetLastError());
    hipLaunchKernelGGL(scf_matvec_kernel, dim3((N + 3) / 4), dim3(256), 0, s, V, rho, N, v);
    SOX_HIP(hipGetLastError());
    hipLaunchKernelGGL(scf_hartree_kernel, grid1d(nn), dim3(256), 0, s, X, v, exch, h, n, N, shf,
                       heff);
    SOX_HIP(hipGetLastError());
    // Sigma^dyn(tau)
    if ((q = launch_fill<double>(sd, cnt, s))) return q;
    if (prm.terms & 1) {
      if ((q = run_gw(p, X, W, g, sd, sub, s))) return q;
    }
    if (prm.terms & 2) {
      q = p.precision == SOX_FP64 ? run_static<double>(p, SOX_ENTRY_BARE, X, V, V, g, sd2, sub, s)
                                  : run_static<float>(p, SOX_ENTRY_BARE, X, V, V, g, sd2, sub, s);
      if (q) return q;
      hipLaunchKernelGGL(scf_add_kernel, grid1d(cnt), dim3(256), 0, s, sd, sd2, cnt);
      SOX_HIP(hipGetLastError());
    }
    return SOX_OK;
  };
  double delta = INFINITY, dmu = 1.0;
  int it = 0;
  for (it = 1; it <= prm.max_iter; ++it) {
    if ((st = self_energy())) return st;
    hipLaunchKernelGGL(scf_ft_kernel, grid1d((long)nm * nn), dim3(256), 0, s, tf, sd, nt, nm, nn,
                       snu);
    SOX_HIP(hipGetLastError());
    // bracket half-width: twice the last change of mu (at least 1e-6 (1 + |mu|));
    // the first iteration, where Sigma^HF enters, starts from 1
    const double mu_prev = mu;
    if ((st = solve_mu(mu, std::max(dmu, 1e-6 * (1.0 + std::fabs(mu))), gn, &mu))) return st;
    dmu = 2.0 * std::fabs(mu - mu_prev);
    hipLaunchKernelGGL(scf_mix_kernel, dim3(nb), dim3(256), 0, s, g, gn, prm.mix, cnt, bmax);
    SOX_HIP(hipGetLastError());
    hipLaunchKernelGGL(scf_reduce_kernel, dim3(1), dim3(256), 0, s, bmax, nb, h, shf, gam, nn, scal);
    SOX_HIP(hipGetLastError());
    SOX_HIP(hipMemcpyAsync(&delta, scal, sizeof(double), hipMemcpyDeviceToHost, s));
    SOX_HIP(hipStreamSynchronize(s));
    if (delta <= prm.tol) break;
  }
  if (it > prm.max_iter) it = prm.max_iter;
  // energies at the final G: E_inf (eq:E1b) and E_dyn (eq:E2b, tau form)
  if ((st = self_energy())) return st;
  hipLaunchKernelGGL(scf_reduce_kernel, dim3(1), dim3(256), 0, s, bmax, 0, h, shf, gam, nn, scal);
  SOX_HIP(hipGetLastError());
  double e_dyn = 0.0;
  if (prm.terms) {
    if ((st = queue_energy(p, sd, g, scal + 2, nullptr, s))) return st;
  } else if ((st = launch_fill<double>(scal + 2, 1, s))) {
    return st;
  }
  double host[3];
  SOX_HIP(hipMemcpyAsync(host, scal, sizeof(host), hipMemcpyDeviceToHost, s));
  SOX_HIP(hipMemcpyAsync(Gout, g, sizeof(double) * cnt, hipMemcpyDeviceToDevice, s));
  SOX_HIP(hipStreamSynchronize(s));
  e_dyn = host[2];
  res->mu = mu;
  res->e_inf = host[1];
  res->e_dyn = e_dyn;
  res->delta = delta;
  res->iterations = it;
  return SOX_OK;
}

}  // namespace

// -- the no-allocation entry point ---------------------------------------------
// sox_sigma_bare_noalloc takes its workspace from this file-scope array
// instead of a caller buffer.  Each GPU the library runs on holds its own copy
// until the process ends.  Host code never uses the array's name as an
// address: the device address is resolved per device with
// hipGetSymbolAddress (with that device current) and kept in
// g_scratch_dev[device].
constexpr size_t kNoallocScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kNoallocMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kNoallocMaxDevices] = {};

// The device address of `scratch` on the current device, resolved on the
// first call from that device.
sox_status noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kNoallocMaxDevices)
    return fail(SOX_ERR_UNSUPPORTED, "device %d: the no-allocation entry supports devices 0..%d",
                device, kNoallocMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SOX_ERR_HIP, "hipGetSymbolAddress of the static scratch array failed: %s",
                  hipGetErrorString(e));
    g_scratch_dev[device] = ptr;
  }
  *out = g_scratch_dev[device];
  return SOX_OK;
}
}  // namespace

// =============================================================================
extern "C" {

int32_t sox_abi_version(void) { return 2; }

const char* sox_last_error(void) { return g_last_error.c_str(); }

sox_status sox_plan_create(const sox_problem* pr, int32_t precision, sox_plan** out) {
  if (!out) return fail(SOX_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!pr) return fail(SOX_ERR_INVALID_ARG, "problem is NULL");
  if (precision < SOX_FP64 || precision > SOX_BF16X3)
    return fail(SOX_ERR_INVALID_ARG, "unknown precision %d", precision);
  if (pr->n_orb < 1 || pr->n_thc < 1 || pr->n_tau < 1)
    return fail(SOX_ERR_SHAPE, "n_orb, n_thc, n_tau must be >= 1 (got %d, %d, %d)", pr->n_orb,
                pr->n_thc, pr->n_tau);
  if (pr->n_orb > 4096 || pr->n_thc > 32768 || pr->n_tau > 4096)
    return fail(SOX_ERR_SHAPE, "sizes beyond the supported range");
  if (pr->kmesh[0] < 1 || pr->kmesh[1] < 1 || pr->kmesh[2] < 1)
    return fail(SOX_ERR_SHAPE, "kmesh entries must be >= 1");
  if (pr->kmesh[0] > 16 || pr->kmesh[1] > 16 || pr->kmesh[2] > 16 ||
      pr->kmesh[0] * pr->kmesh[1] * pr->kmesh[2] > 256)
    return fail(SOX_ERR_SHAPE, "k-point mesh beyond the supported range (<= 16 per axis, <= 256 points)");
  const int nk_req = pr->kmesh[0] * pr->kmesh[1] * pr->kmesh[2];
  if (nk_req > 1 && ((long)pr->n_tau * nk_req * pr->n_orb > 0x7fffffffL ||
                     (long)nk_req * nk_req * pr->n_orb > 0x7fffffffL ||
                     (long)pr->n_thc * pr->n_orb > 0x7fffffffL))
    return fail(SOX_ERR_SHAPE, "k-point problem beyond the supported range");
  if (!(pr->beta > 0.0) || !std::isfinite(pr->beta))
    return fail(SOX_ERR_INVALID_ARG, "beta must be positive and finite");
  if (!pr->tau || !pr->weights) return fail(SOX_ERR_INVALID_ARG, "tau / weights are NULL");
  const int nt = pr->n_tau;
  const double tol = 1e-12 * pr->beta;
  for (int k = 0; k < nt; ++k) {
    const double t = pr->tau[k];
    if (!std::isfinite(t) || t < -tol || t > pr->beta + tol)
      return fail(SOX_ERR_GRID, "tau[%d] = %g outside [0, beta]", k, t);
    if (k > 0 && !(t > pr->tau[k - 1])) return fail(SOX_ERR_GRID, "tau not strictly ascending");
    if (std::fabs(t + pr->tau[nt - 1 - k] - pr->beta) > tol)
      return fail(SOX_ERR_GRID, "tau grid not mirror symmetric at node %d", k);
    if (!std::isfinite(pr->weights[k])) return fail(SOX_ERR_GRID, "weight %d not finite", k);
  }
  if (pr->n_omega < 0) return fail(SOX_ERR_SHAPE, "n_omega < 0");
  if (pr->n_omega > 0 && (!pr->t_fwd || !pr->t_bwd))
    return fail(SOX_ERR_INVALID_ARG, "n_omega > 0 but transform matrices are NULL");
  if (pr->n_omega > 4096) return fail(SOX_ERR_SHAPE, "n_omega beyond the supported range");
  for (size_t i = 0; pr->n_omega > 0 && i < 2 * (size_t)pr->n_omega * nt; ++i)
    if (!std::isfinite(pr->t_fwd[i]) || !std::isfinite(pr->t_bwd[i]))
      return fail(SOX_ERR_GRID, "transform matrices hold non-finite values");

  sox_plan* p = new (std::nothrow) sox_plan();
  if (!p) return fail(SOX_ERR_OOM, "host allocation failed");
  p->n = pr->n_orb;
  p->N = pr->n_thc;
  p->n_tau = nt;
  p->precision = precision;
  p->beta = pr->beta;
  p->tau.assign(pr->tau, pr->tau + nt);
  p->weights.assign(pr->weights, pr->weights + nt);
  p->n_omega = pr->n_omega;
  if (pr->n_omega > 0) {
    p->t_fwd.assign(pr->t_fwd, pr->t_fwd + 2 * (size_t)pr->n_omega * nt);
    p->t_bwd.assign(pr->t_bwd, pr->t_bwd + 2 * (size_t)pr->n_omega * nt);
  }
  p->nP = (int)round_up(p->n, precision == SOX_BF16X3 ? 32 : 16);
  for (int i = 0; i < 3; ++i) p->kmesh[i] = pr->kmesh[i];
  p->nk = nk_req;
  if (p->nk > 1) {
    int j = 0;
    for (int i = 0; i < 3; ++i)
      if (p->kmesh[i] > 1) p->mesh_canon[j++] = p->kmesh[i];
    for (; j < 3; ++j) p->mesh_canon[j] = 1;
  }
  p->fused_cfg = default_fused_cfg(precision, p->N);
  if (const char* s = getenv("SOX_FUSED_CFG")) {
    int v = atoi(s);
    if (v >= 0 && v < kNumFusedCfgs && cfg_allowed(precision, v)) p->fused_cfg = v;
  }
  set_fused_cfg(*p, p->fused_cfg);
  if ((p->fused_cfg == 8 || p->fused_cfg == 9) && !lds_offsets_fit(*p)) {
    // the LDS-staged kernel addresses a (tau, v) panel set with 32-bit lane
    // offsets; past that size the direct-load kernel of the same precision
    set_fused_cfg(*p, p->fused_cfg == 8 ? 7 : 3);
  }
  if (const char* at = getenv("SOX_AUTOTUNE")) {
    if (atoi(at) == 1 && !getenv("SOX_FUSED_CFG") && precision != SOX_BF16X3 && p->nk == 1) {
      sox_status st = autotune_fused(*p);
      if (st) {
        sox_plan_destroy(p);
        return st;
      }
    }
  }
  if (p->nk > 1) {
    p->slab = p->vjp_slab = 1;
    p->vcs = pick_solid_vc(*p, SOX_ENTRY_STATIC);
    p->vcs_bare = pick_solid_vc(*p, SOX_ENTRY_BARE);
    if (p->n_omega > 0) pick_solid_dyn(*p);
  } else {
    p->slab = pick_slab(*p, SOX_ENTRY_STATIC);
    p->vjp_slab = pick_vjp_slab(*p, SOX_ENTRY_STATIC);
    if (p->n_omega > 0) pick_dyn(*p);
  }

  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess &&
        ncu > 0)
      p->n_cu = ncu;
    if (p->nk == 1) pick_vsplit(*p);
  }
  p->dense_wg = 2L * p->n_cu;  // two workgroups of the LDS-staged GEMM per CU
  if (const char* s = getenv("SOX_DENSE_WG")) p->dense_wg = atol(s);
  if (e == hipSuccess && p->n_omega > 0) {
    const int nw = p->n_omega;
    std::vector<double> tf2(2 * (size_t)nw * nt), tb2((size_t)nt * 2 * nw);
    for (int m = 0; m < nw; ++m)
      for (int j = 0; j < nt; ++j) {
        tf2[(size_t)m * nt + j] = p->t_fwd[2 * ((size_t)m * nt + j)];
        tf2[(size_t)(nw + m) * nt + j] = p->t_fwd[2 * ((size_t)m * nt + j) + 1];
      }
    for (int i = 0; i < nt; ++i)
      for (int m = 0; m < nw; ++m) {
        tb2[(size_t)i * 2 * nw + m] = p->t_bwd[2 * ((size_t)i * nw + m)];
        tb2[(size_t)i * 2 * nw + nw + m] = -p->t_bwd[2 * ((size_t)i * nw + m) + 1];
      }
    e = hipMalloc(&p->d_tf2, sizeof(double) * tf2.size());
    if (e == hipSuccess) e = hipMalloc(&p->d_tb2, sizeof(double) * tb2.size());
    if (e == hipSuccess)
      e = hipMemcpy(p->d_tf2, tf2.data(), sizeof(double) * tf2.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_tb2, tb2.data(), sizeof(double) * tb2.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMalloc(&p->d_tau, sizeof(double) * nt);
  if (e == hipSuccess) e = hipMalloc(&p->d_w, sizeof(double) * nt);
  if (e == hipSuccess) {
    // molecules: occupations [n_tau][n], traces [n_tau], energy; k-points:
    // occupations, their complex copy [n_tau][n_k n], traces [n_k][n_tau], energy
    const size_t nocc = (size_t)nt * p->nk * p->n;
    const size_t nsc = p->nk > 1 ? round_up(nocc, 2) + 2 * nocc + (size_t)nt * p->nk + 1
                                 : (size_t)nt * (p->n + 1) + 1;
    e = hipMalloc(&p->d_scratch, sizeof(double) * nsc);
  }
  if (e == hipSuccess && p->nk == 1 && p->n_omega > 0)
    e = hipMalloc(&p->d_wchk, sizeof(double) * 2 * kWchkBlocks);
  if (e == hipSuccess && p->nk > 1 && p->n_omega > 0) {
    const int nw = p->n_omega;
    std::vector<double> tbc((size_t)nt * 4 * nw);
    for (int i = 0; i < nt; ++i)
      for (int m = 0; m < nw; ++m) {
        const double re = p->t_bwd[2 * ((size_t)i * nw + m)], im = p->t_bwd[2 * ((size_t)i * nw + m) + 1];
        double* row = tbc.data() + (size_t)i * 4 * nw;
        row[2 * m] = 0.5 * re;
        row[2 * m + 1] = 0.5 * im;
        row[2 * (nw + m)] = 0.5 * re;
        row[2 * (nw + m) + 1] = -0.5 * im;
      }
    std::vector<double> tfs(2 * p->t_fwd.size());
    for (size_t i = 0; i < p->t_fwd.size(); i += 2) {
      tfs[i] = p->t_fwd[i];
      tfs[i + 1] = p->t_fwd[i + 1];
      tfs[p->t_fwd.size() + i] = p->t_fwd[i];
      tfs[p->t_fwd.size() + i + 1] = -p->t_fwd[i + 1];
    }
    e = hipMalloc(&p->d_tfc, sizeof(double) * tfs.size());
    if (e == hipSuccess)
      e = hipMemcpy(p->d_tfc, tfs.data(), sizeof(double) * tfs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p->d_tbc, sizeof(double) * tbc.size());
    if (e == hipSuccess)
      e = hipMemcpy(p->d_tbc, tbc.data(), sizeof(double) * tbc.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && p->nk > 1) {
    const std::vector<int> tab = solid_tables(p->mesh_canon);
    e = hipMalloc(&p->d_ktab, sizeof(int) * tab.size());
    if (e == hipSuccess)
      e = hipMemcpy(p->d_ktab, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess)
    e = hipMemcpy(p->d_tau, p->tau.data(), sizeof(double) * nt, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_w, p->weights.data(), sizeof(double) * nt, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    sox_status st = fail(e == hipErrorOutOfMemory ? SOX_ERR_OOM : SOX_ERR_HIP,
                         "plan device setup failed: %s", hipGetErrorString(e));
    sox_plan_destroy(p);
    return st;
  }
  *out = p;
  return SOX_OK;
}

sox_status sox_plan_destroy(sox_plan* p) {
  if (!p) return SOX_OK;
  drop_graphs(*p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (auto& e : p->ev_pool) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  if (p->d_tau) (void)hipFree(p->d_tau);
  if (p->d_tf2) (void)hipFree(p->d_tf2);
  if (p->d_tb2) (void)hipFree(p->d_tb2);
  if (p->d_w) (void)hipFree(p->d_w);
  if (p->d_scratch) (void)hipFree(p->d_scratch);
  if (p->d_wchk) (void)hipFree(p->d_wchk);
  if (p->d_ktab) (void)hipFree(p->d_ktab);
  if (p->d_tfc) (void)hipFree(p->d_tfc);
  if (p->d_tbc) (void)hipFree(p->d_tbc);
  delete p;
  return SOX_OK;
}

sox_status sox_workspace_size(const sox_plan* plan, int32_t entry, size_t* bytes) {
  if (!plan) return fail(SOX_ERR_INVALID_ARG, "plan is NULL");
  if (!bytes) return fail(SOX_ERR_INVALID_ARG, "bytes is NULL");
  if (entry < SOX_ENTRY_BARE || entry > SOX_ENTRY_GW)
    return fail(SOX_ERR_INVALID_ARG, "unknown entry %d", entry);
  *bytes = workspace_bytes(*plan, entry);
  return SOX_OK;
}

sox_status sox_sigma_bare(sox_plan* plan, const double* X, const double* V, const double* G,
                          double* Sigma, void* ws, size_t ws_bytes, void* stream) {
  return dispatch_static(plan, SOX_ENTRY_BARE, X, V, V, G, Sigma, ws, ws_bytes, stream);
}

sox_status sox_sigma_static(sox_plan* plan, const double* X, const double* W0, const double* V,
                            const double* G, double* Sigma, void* ws, size_t ws_bytes,
                            void* stream) {
  return dispatch_static(plan, SOX_ENTRY_STATIC, X, W0, V, G, Sigma, ws, ws_bytes, stream);
}

sox_status sox_sigma_vertex(sox_plan* plan, int32_t kind, const double* X, const double* V,
                            const double* W, const double* G, double* Sigma, void* ws,
                            size_t ws_bytes, void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (kind < SOX_VERTEX_SOSEX_STAT || kind > SOX_VERTEX_2SOSEX_DYN)
    return fail(SOX_ERR_INVALID_ARG, "unknown vertex kind %d", kind);
  if (!X || !V || !W || !G || !Sigma) return fail(SOX_ERR_INVALID_ARG, "NULL tensor pointer");
  const bool dyn = kind == SOX_VERTEX_SOSEX_DYN || kind == SOX_VERTEX_2SOSEX_DYN;
  if (dyn && plan->n_omega <= 0)
    return fail(SOX_ERR_INVALID_ARG, "plan has no transform pair (n_omega = 0)");
  if (dyn && plan->nk == 1 && plan->precision == SOX_BF16X3 && plan->fused_cfg != 8)
    return fail(SOX_ERR_UNSUPPORTED,
                "the molecular dynamic entry in bf16x3 needs the LDS-staged fused kernel, whose "
                "32-bit panel offsets overflow at this n_orb and n_thc");
  st = check_ws(plan, SOX_ENTRY_VERTEX, ws, ws_bytes);
  if (st) return st;
  bool real_w = false;
  if (dyn && (st = dynamic_w_is_real(*plan, W, (char*)ws + vertex_layout_for(*plan).pass,
                                     (hipStream_t)stream, &real_w)))
    return st;
  if (dyn && plan->nk == 1) plan->last_w_real = real_w ? 1 : 0;
  const uintptr_t key[9] = {(uintptr_t)SOX_ENTRY_VERTEX, (uintptr_t)X, (uintptr_t)V,
                            (uintptr_t)W, (uintptr_t)G, (uintptr_t)Sigma, (uintptr_t)ws,
                            (uintptr_t)ws_bytes, (uintptr_t)kind * 2 + (real_w ? 1 : 0)};
  return run_maybe_graph(*plan, key, (hipStream_t)stream, [&](hipStream_t s) -> sox_status {
    return run_vertex(*plan, kind, X, V, W, G, Sigma, ws, s, real_w);
  });
}

sox_status sox_sigma_bare_noalloc(sox_plan* plan, const double* X, const double* V,
                                  const double* G, double* Sigma, void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (!X || !V || !G || !Sigma) return fail(SOX_ERR_INVALID_ARG, "NULL tensor pointer");
  const size_t need = workspace_bytes(*plan, SOX_ENTRY_BARE);
  if (need > kNoallocScratchBytes)
    return fail(SOX_ERR_WORKSPACE,
                "the bare entry of this plan needs %zu workspace bytes, more than the %zu-byte "
                "static scratch array (a plan made under SOX_WS_BUDGET_MB=%zu picks tau slabs "
                "that fit)",
                need, kNoallocScratchBytes, kNoallocScratchBytes >> 20);
  int device = -1;
  SOX_HIP(hipGetDevice(&device));
  if (device != plan->device)
    return fail(SOX_ERR_INVALID_ARG, "current device %d is not the plan's device %d", device,
                plan->device);
  void* ws = nullptr;
  if ((st = noalloc_scratch(device, &ws))) return st;
  // no graph capture and no profiling events: nothing in this call
  // allocates (event pools grow with hipEventCreate)
  const bool prof = plan->prof_on;
  plan->prof_on = false;
  const hipStream_t s = (hipStream_t)stream;
  if (plan->nk > 1)
    st = plan->precision == SOX_FP64
             ? run_solid<double>(*plan, SOX_ENTRY_BARE, X, V, V, G, Sigma, ws, s)
             : run_solid<float>(*plan, SOX_ENTRY_BARE, X, V, V, G, Sigma, ws, s);
  else
    st = plan->precision == SOX_FP64
             ? run_static<double>(*plan, SOX_ENTRY_BARE, X, V, V, G, Sigma, ws, s)
             : run_static<float>(*plan, SOX_ENTRY_BARE, X, V, V, G, Sigma, ws, s);
  plan->prof_on = prof;
  return st;
}

sox_status sox_sigma_dynamic(sox_plan* plan, const double* X, const double* W_tau,
                             const double* V, const double* G, double* Sigma, void* ws,
                             size_t ws_bytes, void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (plan->n_omega <= 0)
    return fail(SOX_ERR_INVALID_ARG, "plan has no transform pair (n_omega = 0)");
  if (!X || !W_tau || !V || !G || !Sigma) return fail(SOX_ERR_INVALID_ARG, "NULL tensor pointer");
  st = check_ws(plan, SOX_ENTRY_DYNAMIC, ws, ws_bytes);
  if (st) return st;
  if (plan->nk == 1 && plan->precision == SOX_BF16X3 && plan->fused_cfg != 8)
    return fail(SOX_ERR_UNSUPPORTED,
                "the molecular dynamic entry in bf16x3 needs the LDS-staged fused kernel, whose "
                "32-bit panel offsets overflow at this n_orb and n_thc");
  bool real_w = false;
  if ((st = dynamic_w_is_real(*plan, W_tau, ws, (hipStream_t)stream, &real_w))) return st;
  if (plan->nk == 1) plan->last_w_real = real_w ? 1 : 0;
  const uintptr_t key[9] = {(uintptr_t)SOX_ENTRY_DYNAMIC, (uintptr_t)X, (uintptr_t)W_tau,
                            (uintptr_t)V, (uintptr_t)G, (uintptr_t)Sigma, (uintptr_t)ws,
                            (uintptr_t)ws_bytes, (uintptr_t)real_w};
  return run_maybe_graph(*plan, key, (hipStream_t)stream, [&](hipStream_t s) -> sox_status {
    if (plan->nk > 1) {
      if (plan->precision == SOX_FP64)
        return run_solid_dynamic<double>(*plan, X, W_tau, V, G, Sigma, ws, s);
      return run_solid_dynamic<float>(*plan, X, W_tau, V, G, Sigma, ws, s);
    }
    switch (plan->precision) {
      case SOX_FP64: return run_dynamic<double>(*plan, X, W_tau, V, G, Sigma, ws, s);
      case SOX_FP32:
      case SOX_BF16X3:
        return run_dynamic<float>(*plan, X, W_tau, V, G, Sigma, ws, s, 0, nullptr, real_w);
      default:
        return fail(SOX_ERR_UNSUPPORTED, "unknown precision %d", plan->precision);
    }
  });
}

sox_status sox_ir_grid(double beta, double lambda, double eps, int32_t capacity, int32_t* n_tau,
                       int32_t* n_omega, double* tau, double* weights, int64_t* omega_index,
                       double* t_fwd, double* t_bwd, double* singular_values) {
  if (!n_tau || !n_omega) return fail(SOX_ERR_INVALID_ARG, "n_tau or n_omega is NULL");
  *n_tau = 0;
  *n_omega = 0;
  if (!(beta > 0.0) || !std::isfinite(beta))
    return fail(SOX_ERR_INVALID_ARG, "beta must be positive and finite");
  if (!(lambda >= 1.0) || !(lambda <= 1e8))
    return fail(SOX_ERR_INVALID_ARG, "lambda %g outside [1, 1e8]", lambda);
  if (!(eps >= 1e-12) || !(eps <= 1e-2))
    return fail(SOX_ERR_INVALID_ARG, "eps %g outside [1e-12, 1e-2]", eps);
  if (capacity < 0) return fail(SOX_ERR_INVALID_ARG, "negative capacity");
  sox_ir::Grid g = sox_ir::build(beta, lambda, eps);
  if (!g.error.empty()) return fail(SOX_ERR_UNSUPPORTED, "IR grid: %s", g.error.c_str());
  const int L = g.L, nm = (int)g.m.size();
  *n_tau = L;
  *n_omega = nm;
  if (capacity < std::max(L, nm))
    return fail(SOX_ERR_SHAPE, "capacity %d below the grid's %d tau nodes and %d frequencies",
                capacity, L, nm);
  if (!tau || !weights || !omega_index || !t_fwd || !t_bwd || !singular_values)
    return fail(SOX_ERR_INVALID_ARG, "NULL output array");
  for (int i = 0; i < L; ++i) {
    tau[i] = g.tau[i];
    weights[i] = g.weights[i];
    singular_values[i] = g.sv[i];
  }
  for (int q = 0; q < nm; ++q) omega_index[q] = g.m[q];
  for (size_t i = 0; i < g.t_fwd.size(); ++i) {
    t_fwd[2 * i] = g.t_fwd[i].real();
    t_fwd[2 * i + 1] = g.t_fwd[i].imag();
  }
  for (size_t i = 0; i < g.t_bwd.size(); ++i) {
    t_bwd[2 * i] = g.t_bwd[i].real();
    t_bwd[2 * i + 1] = g.t_bwd[i].imag();
  }
  return SOX_OK;
}

sox_status sox_ir_grid_fermion(double beta, double lambda, double eps, int32_t capacity,
                               int32_t* n_tau, int32_t* n_nu, double* tau, int64_t* nu_index,
                               double* t_fwd, double* t_bwd, double* t_beta) {
  if (!n_tau || !n_nu) return fail(SOX_ERR_INVALID_ARG, "n_tau or n_nu is NULL");
  *n_tau = 0;
  *n_nu = 0;
  if (!(beta > 0.0) || !std::isfinite(beta))
    return fail(SOX_ERR_INVALID_ARG, "beta must be positive and finite");
  if (!(lambda >= 1.0) || !(lambda <= 1e8))
    return fail(SOX_ERR_INVALID_ARG, "lambda %g outside [1, 1e8]", lambda);
  if (!(eps >= 1e-12) || !(eps <= 1e-2))
    return fail(SOX_ERR_INVALID_ARG, "eps %g outside [1e-12, 1e-2]", eps);
  if (capacity < 0) return fail(SOX_ERR_INVALID_ARG, "negative capacity");
  sox_ir::Grid g = sox_ir::build(beta, lambda, eps, true);
  if (!g.error.empty()) return fail(SOX_ERR_UNSUPPORTED, "IR grid: %s", g.error.c_str());
  const int L = g.L, nm = (int)g.m.size();
  *n_tau = L;
  *n_nu = nm;
  if (capacity < std::max(L, nm))
    return fail(SOX_ERR_SHAPE, "capacity %d below the grid's %d tau nodes and %d frequencies",
                capacity, L, nm);
  if (!tau || !nu_index || !t_fwd || !t_bwd || !t_beta)
    return fail(SOX_ERR_INVALID_ARG, "NULL output array");
  for (int i = 0; i < L; ++i) {
    tau[i] = g.tau[i];
    t_beta[i] = g.t_beta[i];
  }
  for (int q = 0; q < nm; ++q) nu_index[q] = g.m[q];
  for (size_t i = 0; i < g.t_fwd.size(); ++i) {
    t_fwd[2 * i] = g.t_fwd[i].real();
    t_fwd[2 * i + 1] = g.t_fwd[i].imag();
  }
  for (size_t i = 0; i < g.t_bwd.size(); ++i) {
    t_bwd[2 * i] = g.t_bwd[i].real();
    t_bwd[2 * i + 1] = g.t_bwd[i].imag();
  }
  return SOX_OK;
}

sox_status sox_scf_workspace_size(const sox_plan* plan, int32_t n_nu, int32_t terms,
                                  size_t* bytes) {
  if (!plan || !bytes) return fail(SOX_ERR_INVALID_ARG, "plan or bytes is NULL");
  if (n_nu < 1) return fail(SOX_ERR_INVALID_ARG, "n_nu must be positive");
  if (terms < 0 || terms > 3) return fail(SOX_ERR_INVALID_ARG, "unknown terms %d", terms);
  *bytes = scf_layout_for(*plan, n_nu, terms).total;
  return SOX_OK;
}

sox_status sox_scf(sox_plan* plan, const sox_scf_params* prm, const double* X, const double* V,
                   const double* W_tau, const double* h, const double* h_start, double* G,
                   sox_scf_result* result, void* ws, size_t ws_bytes, void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (!prm || !result) return fail(SOX_ERR_INVALID_ARG, "params or result is NULL");
  if (plan->nk != 1)
    return fail(SOX_ERR_UNSUPPORTED, "the self-consistent loop runs on molecular plans only");
  if (plan->n > kScfMaxN)
    return fail(SOX_ERR_UNSUPPORTED, "the Dyson kernel takes at most %d orbitals", kScfMaxN);
  if (prm->terms < 0 || prm->terms > 3)
    return fail(SOX_ERR_INVALID_ARG, "unknown terms %d", prm->terms);
  if (prm->n_nu < 1 || !prm->nu || !prm->t_fwd || !prm->t_bwd || !prm->t_beta)
    return fail(SOX_ERR_INVALID_ARG, "fermionic transform pair missing");
  if (!(prm->mix > 0.0 && prm->mix <= 1.0)) return fail(SOX_ERR_INVALID_ARG, "mix outside (0, 1]");
  if (!(prm->tol > 0.0) || prm->max_iter < 1)
    return fail(SOX_ERR_INVALID_ARG, "tol must be positive and max_iter at least 1");
  if (!(prm->n_elec > 0.0 && prm->n_elec < plan->n))
    return fail(SOX_ERR_INVALID_ARG, "n_elec outside (0, n_orb)");
  if (!X || !V || !h || !G || ((prm->terms & 1) && !W_tau))
    return fail(SOX_ERR_INVALID_ARG, "NULL tensor pointer");
  const size_t need = scf_layout_for(*plan, prm->n_nu, prm->terms).total;
  if (!ws) return fail(SOX_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (((uintptr_t)ws & 255) != 0) return fail(SOX_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < need)
    return fail(SOX_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  return run_scf(*plan, *prm, X, V, W_tau, h, h_start, G, result, ws, (hipStream_t)stream);
}

sox_status sox_sigma_gw(sox_plan* plan, const double* X, const double* W_tau, const double* G,
                        double* Sigma, void* ws, size_t ws_bytes, void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (!X || !W_tau || !G || !Sigma) return fail(SOX_ERR_INVALID_ARG, "NULL tensor pointer");
  if ((st = check_ws(plan, SOX_ENTRY_GW, ws, ws_bytes))) return st;
  const uintptr_t key[9] = {(uintptr_t)SOX_ENTRY_GW, (uintptr_t)X, (uintptr_t)W_tau,
                            (uintptr_t)G, (uintptr_t)Sigma, (uintptr_t)ws, (uintptr_t)ws_bytes,
                            0, 0};
  return run_maybe_graph(*plan, key, (hipStream_t)stream, [&](hipStream_t s) -> sox_status {
    return run_gw(*plan, X, W_tau, G, Sigma, ws, s);
  });
}

sox_status sox_sigma_vjp(sox_plan* plan, int32_t entry, const double* X, const double* U1,
                         const double* U2, const double* G, const double* R, double* dG,
                         double* dX, double* dU1, double* dU2, void* ws, size_t ws_bytes,
                         void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (entry < SOX_ENTRY_BARE || entry > SOX_ENTRY_DYNAMIC)
    return fail(SOX_ERR_INVALID_ARG, "unknown entry %d", entry);
  if (plan->nk > 1)
    return fail(SOX_ERR_UNSUPPORTED, "the adjoint is not implemented for k-point meshes");
  if (!X || !U1 || !G || !R) return fail(SOX_ERR_INVALID_ARG, "NULL input pointer");
  if (entry != SOX_ENTRY_BARE && !U2) return fail(SOX_ERR_INVALID_ARG, "U2 is NULL");
  if (entry == SOX_ENTRY_BARE && dU2)
    return fail(SOX_ERR_INVALID_ARG, "bare entry: dU2 must be NULL (dU1 receives dL/dV)");
  if (entry == SOX_ENTRY_DYNAMIC && plan->n_omega <= 0)
    return fail(SOX_ERR_INVALID_ARG, "plan has no transform pair (n_omega = 0)");
  st = check_ws(plan, entry, ws, ws_bytes);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if (entry == SOX_ENTRY_DYNAMIC) {
    switch (plan->precision) {
      case SOX_FP64: return run_vjp_dynamic<double>(*plan, X, U1, U2, G, R, dG, dX, dU1, dU2, ws, s);
      case SOX_FP32: return run_vjp_dynamic<float>(*plan, X, U1, U2, G, R, dG, dX, dU1, dU2, ws, s);
      default: return fail(SOX_ERR_UNSUPPORTED, "precision %d not implemented", plan->precision);
    }
  }
  switch (plan->precision) {
    case SOX_FP64:
      return run_vjp_static<double>(*plan, entry, X, U1, U2, G, R, dG, dX, dU1, dU2, ws, s);
    case SOX_FP32:
      return run_vjp_static<float>(*plan, entry, X, U1, U2, G, R, dG, dX, dU1, dU2, ws, s);
    default: return fail(SOX_ERR_UNSUPPORTED, "precision %d not implemented", plan->precision);
  }
}

sox_status sox_build_g_tau(sox_plan* plan, const double* Q, const double* eps, double mu,
                           double* G, void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (!Q || !eps || !G) return fail(SOX_ERR_INVALID_ARG, "NULL tensor pointer");
  if (!std::isfinite(mu)) return fail(SOX_ERR_INVALID_ARG, "mu not finite");
  hipStream_t s = (hipStream_t)stream;
  if (plan->nk > 1) return solid_build_g(*plan, Q, eps, mu, G, s);
  const int n = plan->n, nt = plan->n_tau;
  double* occ = plan->d_scratch;  // [n_tau][n]
  const int tot = n * nt;
  ProfScope ps(*plan, SOX_STAGE_GBUILD, s);
  hipLaunchKernelGGL(occupation_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, eps,
                     plan->d_tau, mu, plan->beta, n, nt, occ);
  SOX_HIP(hipGetLastError());
  GBuildProb pg{Q, occ, G, n, n, n, n};
  SOX_HIP((launch_gemm<GBuildProb, double, 2, 2, 2, 2>(pg, nt, s)));
  return SOX_OK;
}

namespace {
// Queues the Galitskii-Migdal energy into e (device; null: the plan's scratch
// slot, returned in *slot).
sox_status queue_energy(sox_plan& p, const double* Sigma, const double* G, double* e,
                        double** slot, hipStream_t s) {
  if (p.nk > 1) return solid_energy(p, Sigma, G, e, slot, s);
  const int n = p.n, nt = p.n_tau;
  double* tr = p.d_scratch + (size_t)nt * n;
  if (!e) e = tr + nt;
  if (slot) *slot = e;
  ProfScope ps(p, SOX_STAGE_ENERGY, s);
  hipLaunchKernelGGL(energy_trace_kernel, dim3(nt), dim3(256), 0, s, Sigma, G, n, nt, tr);
  SOX_HIP(hipGetLastError());
  hipLaunchKernelGGL(energy_reduce_kernel, dim3(1), dim3(256), 0, s, tr, p.d_w, nt, e);
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}
}  // namespace

sox_status sox_energy_gm(sox_plan* plan, const double* Sigma, const double* G, double* E_host,
                         void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (!Sigma || !G || !E_host) return fail(SOX_ERR_INVALID_ARG, "NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  double* e = nullptr;
  if ((st = queue_energy(*plan, Sigma, G, nullptr, &e, s))) return st;
  SOX_HIP(hipMemcpyAsync(E_host, e, sizeof(double), hipMemcpyDeviceToHost, s));
  SOX_HIP(hipStreamSynchronize(s));
  return SOX_OK;
}

sox_status sox_energy_gm_device(sox_plan* plan, const double* Sigma, const double* G,
                                double* E_dev, void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (!Sigma || !G || !E_dev) return fail(SOX_ERR_INVALID_ARG, "NULL pointer");
  return queue_energy(*plan, Sigma, G, E_dev, nullptr, (hipStream_t)stream);
}

sox_status sox_profile_enable(sox_plan* plan, int32_t on) {
  sox_status st = check_plan(plan);
  if (st) return st;
  plan->prof_on = on != 0;
  return SOX_OK;
}

sox_status sox_profile_select(sox_plan* plan, uint32_t stage_mask) {
  sox_status st = check_plan(plan);
  if (st) return st;
  plan->prof_mask = stage_mask;
  return SOX_OK;
}

sox_status sox_profile_read(sox_plan* plan, double* ms, int64_t* launches, int64_t* dropped,
                            int32_t reset) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (!ms || !launches) return fail(SOX_ERR_INVALID_ARG, "NULL output");
  for (int i = 0; i < SOX_N_STAGES; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  for (size_t i = 0; i < plan->ev_used; ++i) {
    auto& e = plan->ev_pool[i];
    SOX_HIP(hipEventSynchronize(e.b));
    float t = 0.f;
    SOX_HIP(hipEventElapsedTime(&t, e.a, e.b));
    ms[e.stage] += t;
    launches[e.stage] += 1;
  }
  if (dropped) *dropped = plan->ev_dropped;
  if (reset) {
    plan->ev_used = 0;
    plan->ev_dropped = 0;
  }
  return SOX_OK;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Autotuner on the caller's operands.  A candidate is one setting of the
// plan's launch choices: molecules the fused kernel config and the split of
// its v sum; k-point meshes the tau slab of the B, C and D steps and the
// pair slab of the transforms (dynamic terms) or the v slab (static and
// bare terms).  Every candidate whose workspace fits the budget and the
// caller's buffer is timed on one call of the entry (several for calls
// under 20 ms), the fastest is kept, and the choice is cached per
// (entry, kind, precision, shape) in the file SOX_TUNE_CACHE names.
typedef sox_plan::TuneResult TuneKnobs;

TuneKnobs get_knobs(const sox_plan& p) {
  return TuneKnobs{p.fused_cfg, p.fused_vsplit, p.dyn_ts, p.dyn_ps, p.vcs, p.vcs_bare, 0.0};
}

// the plan's own picks for its current fused config (as at plan creation)
void refresh_choices(sox_plan& p) {
  if (p.nk > 1) {
    p.vcs = pick_solid_vc(p, SOX_ENTRY_STATIC);
    p.vcs_bare = pick_solid_vc(p, SOX_ENTRY_BARE);
    if (p.n_omega > 0) pick_solid_dyn(p);
  } else {
    p.slab = pick_slab(p, SOX_ENTRY_STATIC);
    p.vjp_slab = pick_vjp_slab(p, SOX_ENTRY_STATIC);
    if (p.n_omega > 0) pick_dyn(p);
    pick_vsplit(p);
  }
}

void set_knobs(sox_plan& p, const TuneKnobs& k) {
  if (k.fused_cfg != p.fused_cfg) {
    set_fused_cfg(p, k.fused_cfg);
    refresh_choices(p);
  }
  p.fused_vsplit = k.fused_vsplit;
  p.dyn_ts = k.dyn_ts;
  p.dyn_ps = k.dyn_ps;
  p.vcs = k.vcs;
  p.vcs_bare = k.vcs_bare;
}

bool entry_is_dynamic(int entry, int kind) {
  return entry == SOX_ENTRY_DYNAMIC ||
         (entry == SOX_ENTRY_VERTEX &&
          (kind == SOX_VERTEX_SOSEX_DYN || kind == SOX_VERTEX_2SOSEX_DYN));
}

// candidates within the workspace budget, the plan's own choice first
std::vector<TuneKnobs> tune_candidates(const sox_plan& p0, int entry, int kind) {
  std::vector<TuneKnobs> out;
  const size_t budget = ws_budget();
  sox_plan p = p0;  // a copy for the layout arithmetic (no resources are freed)
  auto add = [&](const TuneKnobs& k) {
    set_knobs(p, k);
    if (workspace_bytes(p, entry) > budget) return;
    for (auto& o : out)
      if (o.fused_cfg == k.fused_cfg && o.fused_vsplit == k.fused_vsplit && o.dyn_ts == k.dyn_ts &&
          o.dyn_ps == k.dyn_ps && o.vcs == k.vcs && o.vcs_bare == k.vcs_bare)
        return;
    out.push_back(k);
  };
  const TuneKnobs base = get_knobs(p0);
  add(base);
  const bool dyn = entry_is_dynamic(entry, kind);
  if (p0.nk == 1) {
    for (int c = 0; c < kNumFusedCfgs; ++c) {
      if (!cfg_usable(p0, c)) continue;
      // the split-precision dynamic entry runs on the LDS-staged kernel only
      if (dyn && p0.precision == SOX_BF16X3 && c != 8) continue;
      set_knobs(p, base);
      TuneKnobs k = base;
      k.fused_cfg = c;
      set_knobs(p, k);
      const TuneKnobs own = get_knobs(p);  // that config's own v split
      add(own);
      // the v split applies to the static entries' LDS-staged and direct-load
      // float kernels; the split-precision direct-load kernels sum all v
      if (p0.precision != SOX_BF16X3 || c == 8)
        for (int s : {1, 2, 4})
          if (s != own.fused_vsplit && (p0.n + s - 1) / s >= 8) {
            TuneKnobs ks = own;
            ks.fused_vsplit = s;
            add(ks);
          }
    }
  } else if (dyn) {
    for (int ts : {4, 8, 16})
      for (int half = 0; half < 2; ++half) {
        TuneKnobs k = base;
        k.dyn_ts = std::min(ts, p0.n_tau);
        if (half) {
          const int nq = base.dyn_ps / p0.nk;  // whole momentum transfers per slab
          if (nq < 2) continue;
          k.dyn_ps = (nq + 1) / 2 * p0.nk;
        }
        add(k);
      }
  } else {
    for (int h : {1, 2}) {
      TuneKnobs k = base;
      k.vcs = std::max(1, (base.vcs + h - 1) / h);
      k.vcs_bare = std::max(1, (base.vcs_bare + h - 1) / h);
      add(k);
    }
  }
  return out;
}

std::string autotune_key(const sox_plan& p, int entry, int kind) {
  char k[160];
  snprintf(k, sizeof(k), "auto-%d-%d %d %d %d %d %d %d %d %d", entry, kind, p.precision, p.n,
           p.N, p.n_tau, p.kmesh[0], p.kmesh[1], p.kmesh[2], p.n_omega);
  return k;
}

}  // namespace

extern "C" {

sox_status sox_autotune_workspace_size(const sox_plan* plan, int32_t entry, int32_t kind,
                                       size_t* bytes) {
  if (!plan) return fail(SOX_ERR_INVALID_ARG, "plan is NULL");
  if (!bytes) return fail(SOX_ERR_INVALID_ARG, "bytes is NULL");
  if (entry < SOX_ENTRY_BARE || entry > SOX_ENTRY_VERTEX)
    return fail(SOX_ERR_INVALID_ARG, "unknown entry %d", entry);
  sox_plan p = *plan;
  size_t need = workspace_bytes(p, entry);
  for (const TuneKnobs& k : tune_candidates(*plan, entry, kind)) {
    set_knobs(p, k);
    need = std::max(need, workspace_bytes(p, entry));
  }
  *bytes = need;
  return SOX_OK;
}

sox_status sox_autotune(sox_plan* plan, int32_t entry, int32_t kind, const double* X,
                        const double* U1, const double* U2, const double* G, double* Sigma,
                        void* ws, size_t ws_bytes, void* stream) {
  sox_status st = check_plan(plan);
  if (st) return st;
  if (entry < SOX_ENTRY_BARE || entry > SOX_ENTRY_VERTEX)
    return fail(SOX_ERR_INVALID_ARG, "unknown entry %d", entry);
  if (!X || !U1 || !G || !Sigma || (entry != SOX_ENTRY_BARE && !U2))
    return fail(SOX_ERR_INVALID_ARG, "NULL tensor pointer");
  if (!ws) return fail(SOX_ERR_WORKSPACE, "workspace is NULL");
  sox_plan& p = *plan;
  const hipStream_t s = (hipStream_t)stream;
  auto call = [&]() -> sox_status {
    switch (entry) {
      case SOX_ENTRY_BARE: return sox_sigma_bare(plan, X, U1, G, Sigma, ws, ws_bytes, stream);
      case SOX_ENTRY_STATIC:
        return sox_sigma_static(plan, X, U1, U2, G, Sigma, ws, ws_bytes, stream);
      case SOX_ENTRY_DYNAMIC:
        return sox_sigma_dynamic(plan, X, U1, U2, G, Sigma, ws, ws_bytes, stream);
      default: return sox_sigma_vertex(plan, kind, X, U1, U2, G, Sigma, ws, ws_bytes, stream);
    }
  };
  std::vector<TuneKnobs> cand = tune_candidates(p, entry, kind);
  const TuneKnobs own = get_knobs(p);
  // a cached choice (validated like any candidate) replaces the timing
  const std::string key = autotune_key(p, entry, kind);
  if (const char* cache = getenv("SOX_TUNE_CACHE")) {
    if (FILE* f = fopen(cache, "r")) {
      char line[256];
      bool found = false;
      TuneKnobs best{};
      while (fgets(line, sizeof(line), f)) {
        char k[32];
        int e, pr, n, N, nt, m0, m1, m2, nw;
        TuneKnobs t{};
        if (sscanf(line, "%31s %d %d %d %d %d %d %d %d | %d %d %d %d %d %d", k, &pr, &n, &N, &nt,
                   &m0, &m1, &m2, &nw, &t.fused_cfg, &t.fused_vsplit, &t.dyn_ts, &t.dyn_ps,
                   &t.vcs, &t.vcs_bare) != 15)
          continue;
        (void)e;
        char full[160];
        snprintf(full, sizeof(full), "%s %d %d %d %d %d %d %d %d", k, pr, n, N, nt, m0, m1, m2, nw);
        if (key != full) continue;
        for (const TuneKnobs& c : cand)
          if (c.fused_cfg == t.fused_cfg && c.fused_vsplit == t.fused_vsplit &&
              c.dyn_ts == t.dyn_ts && c.dyn_ps == t.dyn_ps && c.vcs == t.vcs &&
              c.vcs_bare == t.vcs_bare) {
            best = c;
            found = true;
          }
      }
      fclose(f);
      if (found) {
        sox_plan q = p;
        set_knobs(q, best);
        if (workspace_bytes(q, entry) <= ws_bytes) {
          drop_graphs(p);
          set_knobs(p, best);
          p.autotune.clear();
          p.autotune_cached = 1;
          return SOX_OK;
        }
      }
    }
  }
  // candidates run in the caller's mode: with graph mode on, each candidate
  // is captured once (its own launch sequence) and timed as graph replays
  const bool graph = p.graph_on, prof = p.prof_on;
  p.prof_on = false;
  drop_graphs(p);
  hipEvent_t a = nullptr, b = nullptr;
  auto finish = [&](sox_status r) {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    drop_graphs(p);  // the chosen sequence is captured again by the next call
    p.graph_on = graph;
    p.prof_on = prof;
    return r;
  };
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return finish(fail(SOX_ERR_HIP, "autotune events"));
  p.autotune.clear();
  p.autotune_cached = 0;
  // a call this long hides its launches: such candidates run eagerly, and
  // one call is their measurement
  constexpr float kLongMs = 20.f;
  bool warm = false, tune_graph = false;
  // one candidate's ms per call over about target_ms of back-to-back calls
  auto time_one = [&](const TuneKnobs& c, float target_ms, float* out) -> sox_status {
    drop_graphs(p);
    set_knobs(p, c);
    sox_status r;
    float ms = 0.f;
    if (!warm) {  // first touch of the operands and the code, eager
      p.graph_on = false;
      SOX_HIP(hipEventRecord(a, s));
      if ((r = call())) return r;
      SOX_HIP(hipEventRecord(b, s));
      SOX_HIP(hipEventSynchronize(b));
      SOX_HIP(hipEventElapsedTime(&ms, a, b));
      warm = true;
      tune_graph = graph && ms < kLongMs;
      p.graph_on = tune_graph;
    }
    if (tune_graph && (r = call())) return r;  // the capture
    // one synchronised call sizes the measurement; then the calls run back
    // to back with one synchronisation at the end, as a caller's loop (or a
    // graph replay) runs them: the host enqueues ahead, so the time is the
    // device's, not the launch overhead of a freshly synchronised stream
    SOX_HIP(hipEventRecord(a, s));
    if ((r = call())) return r;
    SOX_HIP(hipEventRecord(b, s));
    SOX_HIP(hipEventSynchronize(b));
    SOX_HIP(hipEventElapsedTime(&ms, a, b));
    if (ms >= kLongMs) {
      *out = ms;
      return SOX_OK;
    }
    const int reps = std::max(1, std::min(100, (int)std::ceil(target_ms / std::max(ms, 1e-3f))));
    SOX_HIP(hipEventRecord(a, s));
    for (int i = 0; i < reps; ++i)
      if ((r = call())) return r;
    SOX_HIP(hipEventRecord(b, s));
    SOX_HIP(hipEventSynchronize(b));
    SOX_HIP(hipEventElapsedTime(&ms, a, b));
    *out = ms / reps;
    return SOX_OK;
  };
  for (const TuneKnobs& c : cand) {
    sox_plan q = p;
    set_knobs(q, c);
    if (workspace_bytes(q, entry) > ws_bytes) continue;
    TuneKnobs r = c;
    float ms;
    if ((st = time_one(c, kLongMs, &ms))) return finish(st);
    r.ms = ms;
    p.autotune.push_back(r);
  }
  // the sweep times short calls in a fixed order, so a drift of the clocks
  // over it favours some; the three fastest are timed again, interleaved over
  // three rounds of longer runs, and each keeps its fastest time
  std::vector<size_t> top(p.autotune.size());
  for (size_t i = 0; i < top.size(); ++i) top[i] = i;
  std::sort(top.begin(), top.end(),
            [&](size_t x, size_t y) { return p.autotune[x].ms < p.autotune[y].ms; });
  top.resize(std::min<size_t>(3, top.size()));
  if (top.size() > 1 && p.autotune[top[0]].ms < kLongMs)
    for (int round = 0; round < 3; ++round)
      for (size_t i : top) {
        float ms;
        if ((st = time_one(p.autotune[i], 40.f, &ms))) return finish(st);
        p.autotune[i].ms = std::min(p.autotune[i].ms, (double)ms);
      }
  double best_ms = 1e300;
  TuneKnobs best = own;
  for (const TuneKnobs& r : p.autotune)
    if (r.ms < best_ms) {
      best_ms = r.ms;
      best = r;
    }
  set_knobs(p, best);
  if (const char* cache = getenv("SOX_TUNE_CACHE")) {
    if (FILE* f = fopen(cache, "a")) {
      fprintf(f, "%s | %d %d %d %d %d %d\n", key.c_str(), best.fused_cfg, best.fused_vsplit,
              best.dyn_ts, best.dyn_ps, best.vcs, best.vcs_bare);
      fclose(f);
    }
  }
  return finish(SOX_OK);
}

sox_status sox_plan_set_graph(sox_plan* plan, int32_t enable) {
  sox_status st = check_plan(plan);
  if (st) return st;
  plan->graph_on = enable != 0;
  if (!plan->graph_on) drop_graphs(*plan);
  return SOX_OK;
}

sox_status sox_plan_describe(const sox_plan* plan, char* buf, size_t len) {
  if (!plan) return fail(SOX_ERR_INVALID_ARG, "plan is NULL");
  if (!buf || len == 0) return fail(SOX_ERR_INVALID_ARG, "buffer is NULL or empty");
  std::string tune = "[";
  for (size_t i = 0; i < plan->tune_ms.size(); ++i) {
    char t[64];
    snprintf(t, sizeof(t), "%s[%d,%.6g]", i ? "," : "", plan->tune_ms[i].first,
             plan->tune_ms[i].second);
    tune += t;
  }
  tune += "]";
  std::string at = "[";
  for (size_t i = 0; i < plan->autotune.size(); ++i) {
    const auto& r = plan->autotune[i];
    char t[160];
    snprintf(t, sizeof(t),
             "%s{\"fused_cfg\":%d,\"fused_vsplit\":%d,\"tau_slab\":%d,\"pair_slab\":%d,"
             "\"v_slab\":%d,\"v_slab_bare\":%d,\"ms\":%.6g}",
             i ? "," : "", r.fused_cfg, r.fused_vsplit, r.dyn_ts, r.dyn_ps, r.vcs, r.vcs_bare, r.ms);
    at += t;
  }
  at += "]";
  const FusedCfg& fc = kFusedCfgs[plan->fused_cfg];
  snprintf(buf, len,
           "{\"n\":%d,\"N\":%d,\"n_tau\":%d,\"nP\":%d,\"NP\":%d,\"precision\":%d,"
           "\"fused_cfg\":%d,\"fused_wave_tile\":[%d,%d],\"tau_slab\":%d,\"vjp_tau_slab\":%d,"
           "\"v_slab\":%d,\"vjp_v_slab\":%d,\"graph\":%d,\"fused_vsplit\":%d,\"n_cu\":%d,"
           "\"tune_ms_per_tau\":%s,"
           "\"tune_from_cache\":%d,\"kmesh\":[%d,%d,%d],\"n_k\":%d,\"solid_v_slab\":%d,"
           "\"solid_v_slab_bare\":%d,\"solid_dyn_pair_slab\":%d,\"solid_dyn_tau_slab\":%d,"
           "\"solid_bare_tau_slab\":%d,\"dynamic_real_w\":%d,\"autotune\":%s,"
           "\"autotune_cached\":%d}",
           plan->n, plan->N, plan->n_tau, plan->nP, plan->NP, plan->precision, plan->fused_cfg,
           fc.wp, fc.wr, plan->slab, plan->vjp_slab, plan->vc, plan->vc_vjp, plan->graph_on ? 1 : 0,
           plan->fused_vsplit, plan->n_cu, tune.c_str(), plan->tune_from_cache ? 1 : 0, plan->kmesh[0], plan->kmesh[1],
           plan->kmesh[2], plan->nk, plan->vcs, plan->vcs_bare, plan->dyn_ps, plan->dyn_ts,
           plan->dyn_ta, plan->last_w_real, at.c_str(), plan->autotune_cached);
  return SOX_OK;
}

sox_status sox_sync(void* stream) {
  SOX_HIP(hipStreamSynchronize((hipStream_t)stream));
  SOX_HIP(hipGetLastError());
  return SOX_OK;
}

}  // extern "C"
