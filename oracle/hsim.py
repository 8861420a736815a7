"""The Hierarchical Subspace Iteration Method (Algorithm 2), on the CPU.

1. build the hierarchy (vertex sets, prolongations, Galerkin operators);
2. q = max(ceil(1.5 p), p + 8);
3. solve the coarsest dense problem completely and keep its first q pairs;
4. for tau = T-2 down to 0: prolong Phi <- U^tau Phi, set the shift
   mu = Lambda^{tau+1}_j with j = floor(p/10), run SIM (Algorithm 1) with the
   Section 4.2 refinements (two inverse iterations per Rayleigh-Ritz step,
   locking at eps/10) and the Euclidean-norm test on the coarse levels;
5. return the first p pairs of level 0.

Reading: when the selected Ritz value is (numerically) the zero eigenvalue of
the constant mode, S - mu M would be singular; the shift then becomes
-1e-3 times the first non-zero Ritz value.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .hierarchy import build_hierarchy, shift_index
from .jacobi import jacobi_gep
from .sim import sim, subspace_size


def choose_shift(lam, p, alpha=0.1):
    j = shift_index(p, alpha)
    mu = float(lam[j])
    if mu <= 1e-12 * float(lam[-1]):
        nz = lam[lam > 1e-12 * lam[-1]]
        mu = -1e-3 * float(nz[0])
    return mu


def hsim(V, F, S0, m0, p, eps=1e-2, levels=0, n_coarsest=0, sigma=7.0, seed=0,
         alpha=0.1, max_iter=200, hierarchy=None):
    """Returns (lam[p], X[n, p], info) with info = dict(iters=[...] coarsest
    first as in the paper's "F|a|b" notation, mu=[...], hierarchy)."""
    lv = hierarchy or build_hierarchy(V, F, S0, m0, p, levels, n_coarsest, sigma, seed)
    T = len(lv)
    q = subspace_size(p)
    top = lv[T - 1]
    Sd = top["S"].toarray() if sp.issparse(top["S"]) else np.asarray(top["S"])
    Md = top["M"].toarray() if sp.issparse(top["M"]) else np.diag(top["M"])
    lam_all, X_all = jacobi_gep(Sd, Md)
    lam, Phi = lam_all[:q], X_all[:, :q]
    iters, mus = ["F"], []
    for tau in range(T - 2, -1, -1):
        Phi = lv[tau]["U"] @ Phi
        mu = choose_shift(lam, p, alpha)
        mus.append(mu)
        lam, Phi, it, r = sim(lv[tau]["S"], lv[tau]["M"], Phi, p, eps, mu,
                              max_iter=max_iter, inverse_iterations=2, lock=True,
                              norm="minv" if tau == 0 else "l2")
        iters.append(it)
    return lam[:p], Phi[:, :p], dict(iters=iters, mu=mus, resid=r[:p], hierarchy=lv)
