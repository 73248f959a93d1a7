"""Composite vertex self-energies built from SOX terms (oracle; test
infrastructure only).

The paper's diagram family (fig:diag) and its G3W2stat decomposition
(section "Total energies and self-energies") write the vertex corrections as
sums of SOX terms with one interaction per line, W = V + W_d split into its
bare part and the rest:

  SOSEX_stat   = SOX(W0, V)
  2SOSEX_stat  = SOX(V,V) + SOX(V,Wd0) + SOX(Wd0,V),      Wd0 = W0 - V
  G3W2_stat    = SOX(W0, W0) = 2SOSEX_stat + SOX(Wd0, Wd0)
  SOSEX_dyn    = SOX(V,V) + SOX(W_d(tau), V)
  2SOSEX_dyn   = SOX(V,V) + SOX(V, W_d(tau)) + SOX(W_d(tau), V)

Each function here is that definition written out term by term with the
oracle's own chains: the static chain for SOX(U1, U2), the eq:GG chain for
SOX(W_d, V), and for SOX(V, W_d) either the line-2 brute force or (line2 =
"mirror") the mirror image of SOX(W_d, V) — transpose for molecules,
conjugate transpose per (k, tau) for solids — which equals it for a
symmetric (Hermitian) G (pinned in tests/test_oracle_vertex.py).
"""
from __future__ import annotations

import numpy as np

from oracle import sox_mol as om
from oracle import sox_solid as osd

KINDS = ("sosex_stat", "2sosex_stat", "g3w2_stat", "sosex_dyn", "2sosex_dyn")


def vertex_mol(kind, X, V, W, G, T_fwd=None, T_bwd=None, line2="mirror"):
    """Molecule: W is W0 [N, N] for the *_stat kinds, W_d(tau) [n_tau, N, N]
    for the *_dyn kinds."""
    Gb = G[::-1]

    def sox(U1, U2):
        return om.sigma_static_thc(X, U1, U2, G, Gb)

    if kind == "sosex_stat":
        return sox(W, V)
    if kind == "2sosex_stat":
        Wd0 = W - V
        return sox(V, V) + sox(V, Wd0) + sox(Wd0, V)
    if kind == "g3w2_stat":
        return sox(W, W)
    dyn = om.sigma_dynamic_thc(X, W, V, G, Gb, T_fwd, T_bwd)          # SOX(W_d, V)
    if kind == "sosex_dyn":
        return sox(V, V) + dyn
    if kind == "2sosex_dyn":
        if line2 == "mirror":
            l2 = dyn.transpose(0, 2, 1)
        else:
            l2 = om.sigma_dynamic_line2_eri(X, V, W, G, Gb, T_fwd, T_bwd)   # SOX(V, W_d)
        return sox(V, V) + l2 + dyn
    raise ValueError(kind)


def vertex_solid(kind, X, V, W, G, tables, T_fwd=None, T_bwd=None, line2="mirror",
                 dyn=None):
    """k-point mesh: W is W0^q [n_k, N, N] for the *_stat kinds and W^q(tau)
    [n_k, n_tau, N, N] for the *_dyn kinds.  `dyn` may hold a precomputed
    SOX(W_d, V) (the eq:GG chain) to reuse across kinds."""

    def sox(U1, U2):
        return osd.sigma_solid_thc(X, U1, U2, G, tables)

    if kind == "sosex_stat":
        return sox(W, V)
    if kind == "2sosex_stat":
        Wd0 = W - V
        return sox(V, V) + sox(V, Wd0) + sox(Wd0, V)
    if kind == "g3w2_stat":
        return sox(W, W)
    if dyn is None:
        dyn = osd.sigma_solid_dynamic_thc(X, W, V, G, T_fwd, T_bwd, tables)
    if kind == "sosex_dyn":
        return sox(V, V) + dyn
    if kind == "2sosex_dyn":
        if line2 == "mirror":
            l2 = np.conj(np.swapaxes(dyn, 2, 3))
        else:
            l2 = osd.sigma_solid_dynamic_line2_eri(X, V, W, G, T_fwd, T_bwd, tables)
        return sox(V, V) + l2 + dyn
    raise ValueError(kind)
