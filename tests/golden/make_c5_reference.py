"""Writes c5_sosex_dyn_support8.npz: oracle reference values of the
benchmarked solid step, SOX(V,V) + SOX(W_d(tau),V) (SOSEX_dyn, fig:diag;
the THC section's k-point static chain plus its momentum-resolved eq:GG
chain), on the 3x3x3, n = 52, N = 400, 100-node, beta = 100 workload with
the collocation matrix restricted to an 8-column support.

The benchmark runs its full launch configuration on that input and compares
these samples (3 momenta x a mirror pair of nodes) element by element, which
gives its max_rel_err against the oracle.  Every input comes from the seeded
generators (synth), every value from oracle/; nothing here touches the GPU
library.  Run from the repository root:  python tests/golden/make_c5_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import sox_solid as osd  # noqa: E402
from paper_2412_18829_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_sosex_dyn_support8.npz")
SUPPORT = dict(per_band=1, seed=502)        # synth.column_support(N, ...)
K_SAMPLES = (0, 5, 22)
NODES = (3, 96)                             # a mirror pair: tau_3 + tau_96 = beta
OMEGA_MAX = 14.0


def main():
    wl = synth.workload(5)
    poles = synth.solid_screening_poles(wl)
    cols = synth.column_support(wl["N"], **SUPPORT)
    tp = synth.bosonic_transform_pair(wl["tau"], wl["beta"], omega_max=OMEGA_MAX, tol=1e-10)
    G = osd.g_tau_k(wl["eps"], wl["Q"], wl["mu"], wl["beta"], wl["tau"])
    tb = (wl["kvecs"], wl["kdiff"], wl["ksum"], wl["kneg"])
    Xs = wl["X"][:, :, cols]
    Vs = wl["V"][:, cols][:, :, cols]
    Ws = sum(a * pole[None, :, None, None] * S[:, None][:, :, cols][:, :, :, cols]
             for a, pole, S in poles)
    t0 = time.perf_counter()
    dyn = 0
    for v0 in range(0, wl["n"], 13):
        dyn = dyn + osd.sigma_solid_dynamic_thc(Xs, Ws, Vs, G, tp["T_fwd"], tp["T_bwd"], tb,
                                                v_subset=range(v0, min(wl["n"], v0 + 13)))
        print(f"dynamic chain: orbitals v < {min(wl['n'], v0 + 13)} ({time.perf_counter() - t0:.0f} s)",
              flush=True)
    bare = osd.sigma_solid_thc(Xs, Vs, Vs, G[:, list(NODES)], tb)
    ref = bare + dyn[:, list(NODES)]
    ks = list(K_SAMPLES)
    np.savez(OUT, sigma=ref[ks], k=np.array(ks), nodes=np.array(NODES), cols=cols,
             n_omega=len(tp["m"]), omega_max=OMEGA_MAX)
    print(f"wrote {OUT}: sigma {ref[ks].shape}, max |sigma| {np.abs(ref[ks]).max():.6e}")


if __name__ == "__main__":
    main()
