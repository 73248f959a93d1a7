"""FP64 CPU oracle for the THC second-order-exchange (SOX) self-energy.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the GPU path: the two meet only
at the seeded synthetic inputs.

Every function is written from the paper (arXiv 2412.18829), section
"THC-SOX and THC-SOSEX: algorithm and implementation details for solids and
molecules", equation eq:sox and the two step lists that follow it, plus the
Galitskii-Migdal energy eq:E2b and the Green's function definition eq:G_def.

Readings of the paper used here (also listed in the design notes):

* Sign.  eq:sox carries a leading minus and the third propagator at -tau.
  We keep the minus and take the third propagator as the stored G(beta-tau)
  (G(-tau) = -G(beta-tau) for fermions).  This makes the SOX energy opposite
  in sign to the direct second-order term (as the paper states in its
  discussion of the molecular couplings) and makes the one-electron Pauli
  cancellation exact.
* The garbled summation labels of the half projections read
  G_Rq = sum_u X_uR G_uq and G_wP = sum_p G_wp X*_pP.
* The momentum label of G_Rq / X_uR in the B steps reads k_v - q1 (the same
  label as the U-contraction and eq:GG).
* 1/N_k appears once in D and once in Sigma_RP: 1/N_k^2 overall.
* Energy: E = -1/2 sum_k w_k Tr[Sigma(tau_k) G(beta - tau_k)] per spin
  channel (the tau form of eq:E2b with the Galitskii-Migdal one half).
* Dynamic interaction: U(1) = W_d(tau) (dynamic part only), U(2) static; the
  convolution variable sits on the G_uq G_sv pair (eq:GG) and the transform
  pair (T_fwd, T_bwd) is an input.

Modules:
  sox_mol    molecules: brute force over the 4-index integrals, the paper's
             THC step chain (static and dynamic), the auxiliary-space route,
             Green's function and energy.
  sox_solid  k-point solids: brute force and the THC step chain.
  sox_vjp    reference vector-Jacobian products (torch CPU float64 autograd
             of the THC chain).
  sox_gw     the THC-GW direct term Sigma^GW = -G W_d of fig:diag (molecules
             and k-point meshes): 4-index brute force and THC chain.
  ir_grid    an in-house IR grid (singular value expansion of the logistic
             kernel): tau sampling points, quadrature weights, the bosonic
             and the fermionic transform pairs.
  scf        a minimal self-consistent Dyson loop (Sigma^HF + Sigma^GW with a
             fixed W_d, optionally SOX(V,V); mu search; E_inf, E_dyn).
  sox_vertex the composite vertex self-energies (SOSEX, 2SOSEX, G3W2stat of
             fig:diag) as sums of SOX terms; SOX(V, W_d) with the dynamic
             interaction on line 2 has its own brute force in sox_mol /
             sox_solid.
"""
