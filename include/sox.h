/*
 * sox.h - C ABI of the MI355X (gfx950) THC second-order-exchange library.
 *
 * Computes the second-order-exchange (SOX) self-energy of arXiv 2412.18829,
 * eq:sox, through the tensor-hypercontracted step chain the paper gives in
 * its section "THC-SOX and THC-SOSEX: algorithm and implementation details
 * for solids and molecules" (static interactions: the U-contraction
 * eq:U_contraction, the half projections G_Rq / G_wP, then A, B, C, D,
 * Sigma_RP and the back-transform; dynamic interactions: eq:GG, FT,
 * W(Omega) GG(Omega), IFT, B, C, D, Sigma).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - One spin channel per call (SOX couples only same-spin quantities).
 * - Molecules (kmesh {1,1,1}): all tensors are real float64, row-major,
 *   contiguous:
 *     X      [n_orb, n_thc]           X_iP, the THC collocation matrix
 *     V, W0  [n_thc, n_thc]           symmetric interaction in the THC basis
 *     W_tau  [n_tau, n_thc, n_thc]    dynamic part of the screened interaction
 *     G      [n_tau, n_orb, n_orb]    G[k,p,q] = G_pq(tau_k); treated as a
 *                                     general (not necessarily symmetric) matrix
 *     Sigma  [n_tau, n_orb, n_orb]    Sigma[k,t,r] = Sigma_tr(tau_k)
 * - Solids (kmesh {m0,m1,m2} with more than one point): n_k = m0 m1 m2
 *   momenta of a Gamma-centred mesh, index (a m1 + b) m2 + c for the integer
 *   vector (a, b, c); q = k_i - k_j is taken modulo the mesh.  Every tensor
 *   is complex128 (interleaved re, im doubles), row-major, contiguous:
 *     X      [n_k, n_orb, n_thc]      X^k_iP
 *     V, W0  [n_k, n_thc, n_thc]      U^q_PQ of the THC integrals
 *            (i k_i, j k_j | s k_s, r k_r) = sum_PQ conj(X^{k_i}_iP) X^{k_j}_jP
 *                                         U^q_PQ conj(X^{k_s}_sQ) X^{k_r}_rQ
 *     W_tau  [n_k, n_tau, n_thc, n_thc] W^q(tau_j) (dynamic entry)
 *     G      [n_k, n_tau, n_orb, n_orb]
 *     Sigma  [n_k, n_tau, n_orb, n_orb]
 *   The k-point form of eq:sox carries 1/N_k per momentum sum (1/N_k^2 in
 *   all), k_s = k_p + k_q - k_t, and follows the momentum-resolved chain of
 *   the paper's solids section (Sigma_RP = -D_PR / N_k).  The bare, static
 *   and dynamic entries, sox_build_g_tau and sox_energy_gm accept solids in
 *   fp64, fp32 and bf16x3 (bf16x3: the B and C products in split precision,
 *   every other step as fp32); the adjoint returns SOX_ERR_UNSUPPORTED.  The dynamic
 *   entry transforms complex functions of imaginary time at +Omega_m with
 *   t_fwd and at -Omega_m with conj(t_fwd), and inverts with
 *   f(tau) = 1/2 sum_m [t_bwd f(i Omega_m) + conj(t_bwd) f(-i Omega_m)]
 *   (the same pair, extended from real to complex functions).
 * - Every tensor pointer is a DEVICE pointer owned by the caller.  Outputs
 *   are overwritten, never accumulated into.  `stream` is a hipStream_t
 *   (NULL = the null stream); all device work of a call is ordered on it
 *   and the call returns before that work finishes, except sox_energy_gm,
 *   which synchronises the stream to return the energy to the host
 *   (sox_energy_gm_device leaves it in device memory instead).
 * - The third propagator of eq:sox is read from node n_tau-1-k, i.e. the
 *   stored G(beta - tau_k): the tau grid must be mirror symmetric,
 *   tau[k] + tau[n_tau-1-k] = beta (checked at plan creation, 1e-12 beta).
 *   eq:sox keeps its leading minus with that reading.
 * - Sign and normalisation readings: Sigma_RP = -D_PR; molecules carry no
 *   1/N_k factors.
 * - Errors are status codes.  A failed argument check returns before any
 *   device work is queued; sox_last_error() then holds a message (per
 *   thread).  Device faults surface as SOX_ERR_HIP on a later call.
 * - A plan is not thread safe; use one plan per host thread.
 */
#ifndef SOX_H
#define SOX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SOX_OK = 0,
  SOX_ERR_INVALID_ARG = 1, /* null pointer, bad enum value, bad scalar        */
  SOX_ERR_SHAPE = 2,       /* sizes out of range or inconsistent              */
  SOX_ERR_GRID = 3,        /* tau grid not ascending / not mirror symmetric   */
  SOX_ERR_WORKSPACE = 4,   /* workspace missing, misaligned or too small      */
  SOX_ERR_OOM = 5,         /* device allocation at plan creation failed       */
  SOX_ERR_HIP = 6,         /* a HIP runtime call or kernel launch failed      */
  SOX_ERR_UNSUPPORTED = 7  /* valid request this library version lacks        */
} sox_status;

/* Arithmetic of the contraction kernels (the A step and the fused B.C -> D
 * step).  G(tau) synthesis, the half projections, the back-transform to
 * orbitals and the energy are always float64.  The Matsubara transforms are
 * float64 for molecules and for SOX_FP64 plans; k-point SOX_FP32 and
 * SOX_BF16X3 plans with even n run them on float32 MFMAs in real form (the
 * other k-point float plans in float64).  The U-contraction
 * (eq:U_contraction) runs in float64 for SOX_FP64 plans and for every
 * k-point plan; molecular SOX_FP32 and SOX_BF16X3 plans run it in float32
 * (its result is stored in float32 for the A step either way).  The k-point
 * D step transforms B and C over the mesh in float32 (float64 for SOX_FP64
 * plans) and accumulates in float64.
 *   SOX_FP64    float64 MFMA (v_mfma_f64_16x16x4f64)
 *   SOX_FP32    float32 MFMA (v_mfma_f32_16x16x4f32), float32 accumulation
 *   SOX_BF16X3  each float32 operand split as hi + lo bfloat16; the products
 *               hi*hi + hi*lo + lo*hi run on bf16 MFMA with float32
 *               accumulation.  Molecules: the bare and static entries (the
 *               A step and the fused B, C -> D contraction in split
 *               precision, the other steps in float32) and the dynamic
 *               entry (the fused contraction in split precision, A(tau)
 *               written by the inverse transform as hi + lo planes, the
 *               other steps in float32); the adjoint returns
 *               SOX_ERR_UNSUPPORTED for a bf16x3 plan.  The molecular
 *               dynamic entry needs the LDS-staged fused kernel, whose
 *               panel offsets are 32-bit: with n_thc * n_orb^2 * 2 bytes at
 *               or past 2^32 (after padding) it returns SOX_ERR_UNSUPPORTED
 *               before any device work (the bare and static entries fall
 *               back to the direct-load kernel there).                      */
typedef enum { SOX_FP64 = 0, SOX_FP32 = 1, SOX_BF16X3 = 2 } sox_precision;

/* Entry kinds, for sox_workspace_size and sox_sigma_vjp. */
typedef enum {
  SOX_ENTRY_BARE = 0,    /* SOX(V, V)                                        */
  SOX_ENTRY_STATIC = 1,  /* SOX(W0, V), W0 = W(Omega = 0)                    */
  SOX_ENTRY_DYNAMIC = 2, /* SOX(W_d(tau), V)                                 */
  SOX_ENTRY_VERTEX = 3,  /* sox_sigma_vertex, every kind (workspace only)    */
  SOX_ENTRY_GW = 4       /* sox_sigma_gw (workspace only)                    */
} sox_entry;

/* Composite vertex self-energies of the paper's diagram family (fig:diag;
 * the G3W2stat decomposition in "Total energies and self-energies"), W =
 * V + W_d split into its bare and dynamic parts:
 *   SOX_VERTEX_SOSEX_STAT   SOX(W0, V)                   statically screened SOSEX
 *   SOX_VERTEX_2SOSEX_STAT  SOX(V,V) + SOX(V,Wd0) + SOX(Wd0,V), Wd0 = W0 - V
 *   SOX_VERTEX_G3W2_STAT    SOX(W0, W0)                  both lines screened
 *   SOX_VERTEX_SOSEX_DYN    SOX(V,V) + SOX(W_d(tau),V) = SOX(V + W_d, V)
 *   SOX_VERTEX_2SOSEX_DYN   SOX(V,V) + SOX(V,W_d(tau)) + SOX(W_d(tau),V)       */
typedef enum {
  SOX_VERTEX_SOSEX_STAT = 0,
  SOX_VERTEX_2SOSEX_STAT = 1,
  SOX_VERTEX_G3W2_STAT = 2,
  SOX_VERTEX_SOSEX_DYN = 3,
  SOX_VERTEX_2SOSEX_DYN = 4
} sox_vertex;

typedef struct sox_plan sox_plan;

typedef struct {
  int32_t n_orb;          /* n, orbitals (>= 1)                                */
  int32_t n_thc;          /* N, THC interpolation points (>= 1)                */
  int32_t n_tau;          /* imaginary-time nodes (>= 1)                       */
  int32_t kmesh[3];       /* {1,1,1}: molecule; else a k-point mesh, each entry
                             1..16, at most 256 points                         */
  double beta;            /* inverse temperature (> 0)                         */
  const double* tau;      /* HOST [n_tau], ascending in [0, beta], mirror
                             symmetric; copied at plan creation                */
  const double* weights;  /* HOST [n_tau], quadrature weights on [0, beta]
                             (used by sox_energy_gm); copied                   */
  int32_t n_omega;        /* dynamic entry only: number of non-negative bosonic
                             Matsubara samples Omega_m; 0 disables the dynamic
                             entry                                             */
  const double* t_fwd;    /* HOST complex128 interleaved [n_omega, n_tau]:
                             f(i Omega_m) = sum_j t_fwd[m,j] f(tau_j); copied  */
  const double* t_bwd;    /* HOST complex128 interleaved [n_tau, n_omega]:
                             f(tau_i) = Re sum_m t_bwd[i,m] f(i Omega_m) for a
                             function real in imaginary time; copied           */
} sox_problem;

/* Create a plan: validates the problem, copies the grid, uploads the
 * quadrature weights and transform pair to the current HIP device and picks
 * the tile shapes and the tau-slab width.  The environment variable
 * SOX_WS_BUDGET_MB (default 65536) caps the workspace the plan asks for
 * (when even the smallest slabs exceed it, the plan asks for those).
 * With SOX_AUTOTUNE=1 the plan times every wave-tile shape of the fused
 * B, C -> D kernel on the device (zero-filled operands of the plan's shape,
 * up to 8 tau nodes) and keeps the fastest; SOX_TUNE_CACHE=<file> stores and
 * reuses those choices per (precision, n, N) across processes.
 * precision is a sox_precision value.  On success *out owns device memory
 * until sox_plan_destroy. */
sox_status sox_plan_create(const sox_problem* problem, int32_t precision, sox_plan** out);

/* Free a plan and its device memory.  NULL is accepted. */
sox_status sox_plan_destroy(sox_plan* plan);

/* Bytes of device workspace the entry `entry` (a sox_entry) needs for this
 * plan; sox_sigma_vjp uses the same value.  The workspace must be 256-byte
 * aligned. */
sox_status sox_workspace_size(const sox_plan* plan, int32_t entry, size_t* bytes);

/* Sigma = SOX(U1 = V, U2 = V): eq:sox with the bare interaction on both
 * lines and the static time relations (tau_wp = tau_uq = tau, the third line
 * at beta - tau).  X [n,N], V [N,N] symmetric, G [n_tau,n,n] -> Sigma
 * [n_tau,n,n]. */
sox_status sox_sigma_bare(sox_plan* plan, const double* X, const double* V, const double* G,
                          double* Sigma, void* workspace, size_t workspace_bytes, void* stream);

/* sox_sigma_bare without a caller workspace, for callers that cannot
 * allocate device memory around the call: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The call itself
 * allocates nothing (no hipMalloc / hipFree, no graph, no profiling events;
 * profiling records nothing for it).  Its workspace is a file-scope device
 * array of 256 MiB that every GPU the library runs on holds from the first
 * such call until the process ends.  Arguments, result and errors as
 * sox_sigma_bare, plus:
 *   - SOX_ERR_WORKSPACE when the plan's bare-entry workspace
 *     (sox_workspace_size) exceeds 256 MiB; a plan created with
 *     SOX_WS_BUDGET_MB=256 or less picks tau slabs that fit;
 *   - SOX_ERR_INVALID_ARG when the current device is not the plan's.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (nothing in it must start at zero): calls that overlap in time on
 * one GPU (several streams or host threads) race, so the caller serialises
 * them. */
sox_status sox_sigma_bare_noalloc(sox_plan* plan, const double* X, const double* V,
                                  const double* G, double* Sigma, void* stream);

/* Sigma = SOX(U1 = W0, U2 = V): the statically screened interaction W0 =
 * W(Omega = 0) (bare part included) on line 1 of eq:sox, the bare V on line
 * 2.  Shapes as sox_sigma_bare; W0 [N,N] symmetric. */
sox_status sox_sigma_static(sox_plan* plan, const double* X, const double* W0, const double* V,
                            const double* G, double* Sigma, void* workspace,
                            size_t workspace_bytes, void* stream);

/* Sigma = SOX(U1 = W_d(tau), U2 = V): line 1 carries the dynamic part of the
 * screened interaction W_tau [n_tau,N,N] (each slice symmetric), evaluated
 * with the paper's eq:GG scheme: GG -> FT -> W(Omega) GG(Omega) -> IFT ->
 * B, C, D -> Sigma, using the plan's transform pair.  The plan must have
 * n_omega > 0.  Solids: W_tau, V, X, G, Sigma complex128 as listed above. */
sox_status sox_sigma_dynamic(sox_plan* plan, const double* X, const double* W_tau, const double* V,
                             const double* G, double* Sigma, void* workspace,
                             size_t workspace_bytes, void* stream);

/* Composite vertex self-energy `kind` (a sox_vertex), assembled on the
 * device from the SOX terms above (the caller does no arithmetic):
 *   W  the full screened interaction W0 = W(Omega = 0) [N,N] for the *_STAT
 *      kinds; the dynamic part W_d(tau) [n_tau,N,N] for the *_DYN kinds
 *      (plan with n_omega > 0).  Solids: complex128 with the leading n_k
 *      axis, as for the other entries.
 *   V  the bare interaction; X, G, Sigma as sox_sigma_bare.
 * SOSEX_DYN on a k-point plan runs as one pass: both terms share line 2, so
 * the bare term enters the dynamic chain's A(tau) and the B, C, D steps and
 * the back-transform run once.  2SOSEX_DYN takes SOX(V, W_d) as the mirror
 * image of SOX(W_d, V) (transpose for molecules, conjugate transpose per k
 * and tau for solids), which holds when every G(tau) is symmetric
 * (Hermitian per k), as for a G built by sox_build_g_tau; for a general G
 * that term is not SOX(V, W_d).  2SOSEX_STAT is SOX(V, W0) + SOX(W0 - V, V)
 * (bilinearity) and needs no such condition.  Workspace:
 * sox_workspace_size(plan, SOX_ENTRY_VERTEX).  Errors as the other entries
 * (SOX_ERR_INVALID_ARG for an unknown kind or a *_DYN kind without a
 * transform pair). */
sox_status sox_sigma_vertex(sox_plan* plan, int32_t kind, const double* X, const double* V,
                            const double* W, const double* G, double* Sigma, void* workspace,
                            size_t workspace_bytes, void* stream);

/* The THC-GW direct term: the GW self-energy of fig:diag (the dynamic
 * part: the propagator and the screened line W_d join the same two points),
 *   Sigma_ij(tau) = - sum_kl (ik|lj)_{W_d(tau)} G_kl(tau)
 *                 = - sum_PQ X_iP [Gt_PQ(tau) W_PQ(tau)] X_jQ,
 *   Gt_PQ(tau) = sum_kl X_kP G_kl(tau) X_lQ,
 * with the interaction in the THC form of section "THC-SOX and THC-SOSEX"
 * (Gt starts from the SOX chain's half projection G_Rq).  Local in tau: no
 * transform pair is needed, and W_tau is sampled on the plan's tau grid.
 * Molecules: X [n,N], W_tau [n_tau,N,N], G, Sigma [n_tau,n,n], float64.
 * Solids (complex128, leading n_k axis; W_tau indexed by the transfer q):
 *   Sigma^k_ij(tau) = -(1/N_k) sum_k' sum_PQ conj(X^k_iP) W^{k-k'}_PQ(tau)
 *                     Gt^{k'}_PQ(tau) X^k_jQ,
 *   Gt^{k'}_PQ = sum_ls X^{k'}_lP G^{k'}_ls conj(X^{k'}_sQ).
 * Every step runs in float64 whatever the plan's precision (the term costs
 * O(n_tau N^2 n) per momentum pair, a factor n below the SOX chain).
 * Workspace: sox_workspace_size(plan, SOX_ENTRY_GW).  Errors: NULL pointers
 * (SOX_ERR_INVALID_ARG), workspace (SOX_ERR_WORKSPACE), launch failures
 * (SOX_ERR_HIP). */
sox_status sox_sigma_gw(sox_plan* plan, const double* X, const double* W_tau, const double* G,
                        double* Sigma, void* workspace, size_t workspace_bytes, void* stream);

/* An IR (intermediate representation) imaginary-time grid built in-house,
 * the sparse grid of the paper's computational details (beta, Lambda = beta
 * omega_max): the singular value expansion of the logistic kernel
 * K(x, y) = exp(-Lambda y (x + 1) / 2) / (1 + exp(-Lambda y)) (x = 2 tau /
 * beta - 1, y = beta omega / Lambda), truncated at s_l >= eps s_0 (L basis
 * functions); tau nodes at the L roots of the first function left out
 * (ascending, mirror symmetric: usable as sox_problem.tau); quadrature
 * weights of int_0^beta for sox_problem.weights; bosonic Matsubara samples
 * Omega_m = 2 pi m / beta (m = omega_index[q] >= 0: m = 0 and the sign
 * changes of the first even and odd functions left out); and the transform
 * pair in the layout of sox_problem.t_fwd / t_bwd: f(i Omega_m) =
 * sum_j t_fwd[q,j] f(tau_j), f(tau_i) = Re sum_q t_bwd[i,q] f(i Omega_q) for
 * a function real in imaginary time.  Host code, no device work; float64.
 *   beta > 0; 1 <= lambda <= 1e8; 1e-12 <= eps <= 1e-2 (float64 resolves
 *   the basis there);
 *   capacity: the length the caller's arrays allow: tau, weights,
 *   singular_values (s_l / s_0) hold L values, omega_index n_omega, t_fwd
 *   2 n_omega L doubles (complex interleaved [n_omega][L]) and t_bwd
 *   2 L n_omega ([L][n_omega]): allocate capacity, capacity, capacity and
 *   2 capacity^2 doubles.
 * *n_tau = L and *n_omega are written on success and when capacity is too
 * small (SOX_ERR_SHAPE, nothing else written: call again with a larger
 * capacity).  SOX_ERR_INVALID_ARG for parameters out of range or NULL
 * arrays; SOX_ERR_UNSUPPORTED when the root count of the first omitted
 * function shows the basis unresolved. */
sox_status sox_ir_grid(double beta, double lambda, double eps, int32_t capacity, int32_t* n_tau,
                       int32_t* n_omega, double* tau, double* weights, int64_t* omega_index,
                       double* t_fwd, double* t_bwd, double* singular_values);

/* The fermionic counterpart of sox_ir_grid on the same basis and tau nodes:
 * odd Matsubara samples nu_n = (2n + 1) pi / beta (n = nu_index[q] >= 0: n = 0
 * and the sign changes of the first omitted even function's Im U^ and odd
 * function's Re U^), the pair f(i nu_n) = sum_j t_fwd[q,j] f(tau_j),
 * f(tau_i) = Re sum_q t_bwd[i,q] f(i nu_q) (complex interleaved, layouts as
 * sox_ir_grid) and t_beta [n_tau] with f(beta^-) = sum_i t_beta[i] f(tau_i).
 * Arguments, capacity protocol and errors as sox_ir_grid.  Host code. */
sox_status sox_ir_grid_fermion(double beta, double lambda, double eps, int32_t capacity,
                               int32_t* n_tau, int32_t* n_nu, double* tau, int64_t* nu_index,
                               double* t_fwd, double* t_bwd, double* t_beta);

/* A minimal self-consistent Dyson loop (section "Definitions": eq:Dyson,
 * eq:G0 with an orthonormal basis S = I, the chemical potential updated
 * every iteration for the target electron count, energies eq:E1b and
 * eq:E2b) for one spin channel of a molecule, float64:
 *   Sigma[G] = Sigma^HF[gamma] + Sigma^dyn[G](tau),
 *   Sigma^HF_ij = sum_kl [(ij|kl) gamma_lk - (ik|lj) gamma_kl] with V,
 *   Sigma^dyn = the THC-GW direct term with the fixed W_tau (terms bit 0; a
 *   stand-in for the screened interaction, not rebuilt from G) plus SOX(V,
 *   V) (bit 1, in the plan's precision);
 *   gamma_pq = -G_qp(beta^-); each iteration transforms Sigma^dyn to the
 *   fermionic samples, solves G(i nu) = [(i nu + mu) I - h - Sigma^HF -
 *   Sigma^dyn(i nu)]^-1 (batched in-place Gauss-Jordan inversions with
 *   partial pivoting, in LDS for n_orb <= 96 unless
 *   SOX_SCF_DYSON_IN_MEMORY=1) for the mu that holds n_elec (the root of N(mu) =
 *   -Tr G(beta^-) by Illinois regula falsi, to 1e-12 (1 + |mu|), inside a
 *   bracket about the previous mu of twice its last change, widened
 *   fourfold until it holds the root), returns to tau, and mixes
 *   G <- (1 - mix) G + mix G_new until max |G_new - G| <= tol or max_iter.
 *   E_inf = sum_pq (h + Sigma^HF / 2)_pq gamma_pq; E_dyn = -1/2 sum_j w_j
 *   Tr[Sigma^dyn(tau_j) G(beta - tau_j)] (the plan's weights).
 * The plan: a molecular plan on the IR tau grid of sox_ir_grid_fermion
 * (with its sox_ir_grid weights), n_orb <= 1024.  Device inputs X [n,N], V
 * [N,N], W_tau [n_tau,N,N] (may be NULL without bit 0), h [n,n] (the one-body
 * H0 of eq:G0), h_start [n,n] or NULL (the H0 of the starting G0; default
 * h); output G [n_tau,n,n] device.  The host arrays of the fermionic pair
 * are copied at the call.  Workspace: sox_scf_workspace_size.  Errors:
 * SOX_ERR_UNSUPPORTED for k-point plans or n_orb > 1024, SOX_ERR_INVALID_ARG
 * for parameters out of range.  The call synchronises the stream (the loop
 * control runs on the host). */
typedef struct {
  double n_elec;        /* target electrons of the channel, 0 < n_elec < n_orb */
  double mix;           /* 0 < mix <= 1 */
  double tol;           /* > 0: stop at max |G_new - G| <= tol */
  int32_t max_iter;     /* >= 1 */
  int32_t terms;        /* bit 0: GW with W_tau; bit 1: SOX(V, V)          */
  int32_t n_nu;         /* fermionic samples of the pair                  */
  const double* nu;     /* HOST [n_nu] nu_n = (2n + 1) pi / beta           */
  const double* t_fwd;  /* HOST complex [n_nu][n_tau]                      */
  const double* t_bwd;  /* HOST complex [n_tau][n_nu]                      */
  const double* t_beta; /* HOST [n_tau]                                    */
} sox_scf_params;

typedef struct {
  double mu, e_inf, e_dyn, delta;  /* converged mu, eq:E1b, eq:E2b, last max |dG| */
  int32_t iterations;
} sox_scf_result;

sox_status sox_scf_workspace_size(const sox_plan* plan, int32_t n_nu, int32_t terms,
                                  size_t* bytes);
sox_status sox_scf(sox_plan* plan, const sox_scf_params* params, const double* X, const double* V,
                   const double* W_tau, const double* h, const double* h_start, double* G,
                   sox_scf_result* result, void* workspace, size_t workspace_bytes, void* stream);

/* Vector-Jacobian product of L = sum(Sigma * R) for the entry `entry`:
 *   R [n_tau,n,n] cotangent;  dG [n_tau,n,n], dX [n,N], dU1, dU2 outputs.
 * For SOX_ENTRY_BARE, U1 = U2 = V is passed as U1 (U2 ignored) and dU1
 * receives the total dL/dV; dU2 must be NULL.  For SOX_ENTRY_STATIC dU1 =
 * dL/dW0, dU2 = dL/dV.  For SOX_ENTRY_DYNAMIC U1 = W_tau, dU1 = dL/dW_tau
 * [n_tau,N,N], dU2 = dL/dV.  Any output may be NULL (not computed).
 * Gradients are with respect to every entry of the (general) matrices, not
 * symmetrised. */
sox_status sox_sigma_vjp(sox_plan* plan, int32_t entry, const double* X, const double* U1,
                         const double* U2, const double* G, const double* R, double* dG,
                         double* dX, double* dU1, double* dU2, void* workspace,
                         size_t workspace_bytes, void* stream);

/* G(tau_k) = -Q diag(n(eps, tau_k)) Q^T on the plan's grid (eq:G_def for a
 * one-body Hamiltonian F = Q diag(eps) Q^T, chemical potential mu), with
 * n(e,tau) = e^{-(e-mu)tau} / (1 + e^{-beta(e-mu)}) for e >= mu and the
 * equal form e^{(beta-tau)(e-mu)} / (1 + e^{beta(e-mu)}) for e < mu, so no
 * exponential overflows.  Q [n,n] device (eigenvectors in columns), eps [n]
 * device, G [n_tau,n,n] device output.  float64 throughout.
 * Solids: G^k(tau) = -Q_k diag(n(eps_k, tau)) Q_k^dagger with Q complex128
 * [n_k,n,n], eps float64 [n_k,n], G complex128 [n_k,n_tau,n,n]. */
sox_status sox_build_g_tau(sox_plan* plan, const double* Q, const double* eps, double mu,
                           double* G, void* stream);

/* Galitskii-Migdal energy of a SOX self-energy (eq:E2b in imaginary time):
 * E = -1/2 sum_k w_k sum_tr Sigma_tr(tau_k) G_rt(beta - tau_k), float64.
 * Sigma, G device [n_tau,n,n]; *E_host written after the stream is
 * synchronised.  Solids: E = -1/2 (1/N_k) sum_k sum_j w_j
 * Re Tr[Sigma^k(tau_j) G^k(beta - tau_j)], Sigma and G complex128
 * [n_k,n_tau,n,n]. */
sox_status sox_energy_gm(sox_plan* plan, const double* Sigma, const double* G, double* E_host,
                         void* stream);

/* The same energy (eq:E2b) stored in DEVICE memory: E_dev is one float64
 * owned by the caller, written on `stream`; the call returns before it is
 * written and does not synchronise, so a loop of sweeps can queue the
 * energy of every iteration and read the values later.  Arguments and
 * errors as for sox_energy_gm. */
sox_status sox_energy_gm_device(sox_plan* plan, const double* Sigma, const double* G,
                                double* E_dev, void* stream);

/* Per-stage device-time accounting.  While enabled, every kernel launch of
 * the plan's entry points is bracketed by HIP events recorded on the call's
 * stream; sox_profile_read synchronises those events and returns, per
 * stage, the summed elapsed milliseconds and the number of launches since
 * the last reset.  Used by the benchmark to time the dominant kernel on the
 * stream it runs on.  At most 65536 launches are recorded between resets;
 * later ones are counted in `dropped`. */
typedef enum {
  SOX_STAGE_GBUILD = 0,   /* G(tau) synthesis                               */
  SOX_STAGE_UTENSOR = 1,  /* U-contraction (eq:U_contraction)               */
  SOX_STAGE_PROJECT = 2,  /* half projections G_Rq, G_wP                    */
  SOX_STAGE_ASTEP = 3,    /* A step                                         */
  SOX_STAGE_FUSED = 4,    /* fused B, C -> D contraction                    */
  SOX_STAGE_BACK = 5,     /* back-transform to orbitals                     */
  SOX_STAGE_ENERGY = 6,   /* Galitskii-Migdal energy                        */
  SOX_STAGE_GG_FT = 7,    /* dynamic: GG formation + forward transform      */
  SOX_STAGE_WGEMM = 8,    /* dynamic: W(Omega) GG(Omega)                    */
  SOX_STAGE_IFT = 9,      /* dynamic: inverse transform                     */
  SOX_STAGE_SPLIT = 10,   /* bf16 hi/lo split                               */
  SOX_STAGE_VJP = 11,     /* adjoint kernels                                */
  SOX_STAGE_KBC = 12,     /* solids: B and C products of every momentum pair */
  SOX_STAGE_KD = 13,      /* solids: the n_k^3 D step                        */
  SOX_STAGE_GW = 14,      /* sox_sigma_gw, the whole chain                   */
  SOX_N_STAGES = 15
} sox_stage;

sox_status sox_profile_enable(sox_plan* plan, int32_t on);

/* Bit s of stage_mask selects stage s (sox_stage) for recording while
 * profiling is enabled; the other stages launch without events.  Default:
 * every stage.  Each recorded stage adds two event records per launch
 * group to the stream, so timing one stage perturbs the rest least. */
sox_status sox_profile_select(sox_plan* plan, uint32_t stage_mask);

/* ms[SOX_N_STAGES], launches[SOX_N_STAGES]; `dropped` may be NULL.  reset != 0
 * clears the accounting afterwards. */
sox_status sox_profile_read(sox_plan* plan, double* ms, int64_t* launches, int64_t* dropped,
                            int32_t reset);

/* Replay whole sweeps as HIP graphs.  When enabled, the first
 * sox_sigma_bare / sox_sigma_static / sox_sigma_dynamic call with a given set
 * of pointers (inputs, output, workspace) captures its launch sequence on a
 * plan-owned stream into a graph; later calls with the same pointers launch
 * that graph on `stream` (one launch per sweep).  The graph reads the
 * buffers' current contents, so only the pointers, not the values, must
 * match.  Up to 16 graphs are kept per plan (the oldest is dropped).  Kernel
 * timing (sox_profile_*) records nothing for replayed sweeps. */
sox_status sox_plan_set_graph(sox_plan* plan, int32_t enable);

/* Autotuner on the caller's operands (the batching of all tau nodes and,
 * for k-point plans, all momentum pairs into few launches whose shapes are
 * the plan's choices; see the THC section's step lists for the steps).
 * Times `entry` for every candidate setting of the plan's launch choices
 * and keeps the fastest: one synchronised call sizes the measurement and,
 * when it is shorter than 20 ms, calls filling about 20 ms (up to 100) run
 * back to back with a single synchronisation, so the time is the device's
 * per call as in a caller's loop, not the launch overhead of an idle
 * stream.  With the plan's graph mode on (sox_plan_set_graph) and calls
 * shorter than 20 ms, each candidate is captured once and timed as graph
 * replays, the mode such a caller runs in.  For such short calls the three
 * fastest candidates are then timed again, interleaved over three rounds of
 * about 40 ms each, and keep their fastest time (the sweep's fixed order
 * would otherwise favour candidates timed after the clocks have settled).
 * The choices:
 *   molecules        the fused B, C -> D kernel's configuration (wave tile,
 *                    direct-load or LDS-staged, of the plan's precision)
 *                    and the split of its v sum over workgroups;
 *   k-point, dynamic the tau slab of the B, C and D steps (4, 8, 16 nodes)
 *                    and the momentum-pair slab of the transforms (the
 *                    plan's and half of it);
 *   k-point, static / bare  the v slab of the B, C and D steps (the plan's
 *                    and half of it).
 * Candidates whose workspace exceeds SOX_WS_BUDGET_MB or workspace_bytes
 * are skipped; sox_autotune_workspace_size gives the size that admits every
 * candidate.  Operands as the entry takes them: BARE U1 = V, U2 = NULL;
 * STATIC U1 = W0, U2 = V; DYNAMIC U1 = W_tau, U2 = V; VERTEX U1 = V,
 * U2 = W with vertex kind `kind` (ignored otherwise).  Sigma receives the
 * result of the last candidate timed (every candidate computes the same
 * Sigma).  With SOX_TUNE_CACHE=<file> the choice is appended to the file,
 * keyed by entry, kind, precision and shape, and a later call with the same
 * key takes it from there without timing.  The plan's graphs are dropped
 * (its launch sequence may change; the next call captures the chosen one);
 * the plan's graph mode is kept.  Results
 * appear under "autotune" in sox_plan_describe.  Errors: those of the entry
 * (the first failing candidate's status is returned). */
sox_status sox_autotune(sox_plan* plan, int32_t entry, int32_t kind, const double* X,
                        const double* U1, const double* U2, const double* G, double* Sigma,
                        void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes that admit every sox_autotune candidate of `entry`
 * (`kind` as for sox_autotune). */
sox_status sox_autotune_workspace_size(const sox_plan* plan, int32_t entry, int32_t kind,
                                       size_t* bytes);

/* A one-line JSON description of the plan's decisions: padded extents, the
 * fused kernel's wave tile, tau-slab and v-slab widths, and the autotuners'
 * timings when they ran.  Writes at most `len` bytes including the NUL. */
sox_status sox_plan_describe(const sox_plan* plan, char* buf, size_t len);

/* Synchronise `stream` and report any pending device error. */
sox_status sox_sync(void* stream);

/* Message for the last non-OK status on this host thread ("" if none). */
const char* sox_last_error(void);

/* ABI version of this library (increments on incompatible changes). */
int32_t sox_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SOX_H */
