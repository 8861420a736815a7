"""Write the stored reference eigenpairs of the large workloads.

Runs the oracle only: FP64 assembly (Section 3.1, eq. massStiffMatrices) and
plain subspace iteration (Algorithm 1, with two inverse iterations per
Rayleigh-Ritz step as in Section 4.2, no locking, no hierarchy) from a seeded
random start, with the constant negative shift of ``oracle.sim.sim_lowest``
and a SuperLU factorisation, until every stored pair has a floored relative
residual (M^-1-norm form of eq. conv2) below ``--eps`` (1e-10).  Stored pairs:
the first p plus the rest of the eigenvalue cluster (relative gaps < 1e-2)
that holds pair p-1, so the cluster-aware eigenvector comparison always has
the whole cluster.

The result is pinned to something other than the iteration itself:
  * Sylvester inertia: the number of eigenvalues below lambda_{k-1}(1 + 1e-7)
    is at least k and below lambda_{k-1}(1 - 1e-7) at most k - 1 (sign count
    of the pivots of a symmetric-ordering factorisation without off-diagonal
    pivoting), so no eigenvalue below the last stored one is missed;
  * the residual bound itself, re-evaluated after the run;
  * M-orthonormality of the stored vectors.

Eigenvectors of a 1M-vertex mesh are too large to keep, so a sketch is stored:
Z = G^T (M^{1/2} Y) for the seeded Gaussian G = synth.gaussian_matrix(n, r,
seed) (see oracle.metrics).  Output, next to this script:
  <workload>_p<p>.json   eigenvalues, residuals, clusters, run and check data,
                         and the largest residual of the tested pairs after every
                         Rayleigh-Ritz step (the oracle's convergence history)
  <workload>_p<p>_sketch.npy   Z (r x k), float64

Usage: python tests/golden/make_golden.py torus100k 100 [--q 200] [--threads 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import assembly, metrics, sim  # noqa: E402

SKETCH_ROWS = 64
SKETCH_SEED = 20211117


def negative_count(S, m, sigma):
    """Eigenvalues of S x = lambda M x below sigma, by Sylvester's law of
    inertia on a factorisation with static diagonal pivots."""
    A = (S - sigma * sp.diags(m)).tocsc()
    lu = spla.splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    if not np.array_equal(lu.perm_r, lu.perm_c):
        raise RuntimeError("symmetric permutation expected")
    return int(np.sum(lu.U.diagonal() < 0))


class _Progress(list):
    def __init__(self, t0):
        super().__init__()
        self.t0 = t0

    def append(self, x):
        super().append(x)
        print(f"  iteration {len(self)}: max residual of the tested pairs {x:.3e} "
              f"({time.perf_counter() - self.t0:.0f} s)", flush=True)


def stored_count(lam, p):
    """p plus the rest of the cluster that holds pair p-1."""
    for a, b in metrics.clusters(lam):
        if a <= p - 1 < b:
            return b
    return p


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("p", type=int)
    ap.add_argument("--q", type=int, default=0, help="subspace size (default 2p)")
    ap.add_argument("--eps", type=float, default=1e-10)
    ap.add_argument("--seed", type=int, default=0, help="mesh seed")
    ap.add_argument("--start-seed", type=int, default=7, help="seed of the random start block")
    ap.add_argument("--threads", type=int, default=1)
    ap.add_argument("--max-iter", type=int, default=400)
    a = ap.parse_args()

    t0 = time.perf_counter()
    V, F, dens = synth.config_mesh(a.workload, seed=a.seed)
    S, m = assembly.assemble(V, F, density=dens)
    n = len(m)
    q = a.q or 2 * a.p
    mu = -1e-6 * S.diagonal().sum() / m.sum()
    print(f"[golden] {a.workload}: n={n}, p={a.p}, q={q}, mu={mu:.3e} ({time.perf_counter() - t0:.0f} s)", flush=True)
    solver = sim.ShiftedSolver(S, m, mu, symmetric=True, threads=a.threads)
    print(f"[golden] factorised ({time.perf_counter() - t0:.0f} s)", flush=True)
    Phi = np.random.default_rng(a.start_seed).standard_normal((n, q))
    k = a.p
    total_it = 0
    hist = _Progress(t0)
    while True:
        lam, Phi, it, r = sim.sim(S, m, Phi, k, a.eps, mu, max_iter=a.max_iter - total_it,
                                  inverse_iterations=2, history=hist, solver=solver)
        total_it += it
        k_new = stored_count(lam, a.p)
        if k_new > q - 8:
            raise RuntimeError(f"cluster of pair p-1 reaches {k_new}: increase q")
        if np.all(r[:k_new] < a.eps) or total_it >= a.max_iter:
            k = k_new
            break
        k = k_new
    if not np.all(r[:k] < a.eps):
        raise RuntimeError(f"not converged after {total_it} iterations: {r[:k].max():.3e}")
    lam, Y, r = lam[:k], Phi[:, :k], r[:k]
    print(f"[golden] converged: {total_it} iterations, {k} pairs stored ({time.perf_counter() - t0:.0f} s)", flush=True)
    del solver, Phi

    # checks that do not come from the iteration
    r_chk = sim.residual(S, m, Y, lam)
    orth = metrics.m_orthonormality(Y, m)
    top = float(lam[k - 1])
    below_hi = negative_count(S, m, top * (1 + 1e-7))
    below_lo = negative_count(S, m, top * (1 - 1e-7))
    print(f"[golden] residual {r_chk.max():.2e}, M-orthonormality {orth:.2e}, "
          f"inertia {below_lo} < {k} <= {below_hi} ({time.perf_counter() - t0:.0f} s)", flush=True)
    if not (r_chk.max() < a.eps and orth < 1e-10 and below_hi >= k and below_lo <= k - 1):
        raise RuntimeError("oracle result failed its checks")

    G = synth.gaussian_matrix(n, SKETCH_ROWS, SKETCH_SEED)
    Z = metrics.sketch(Y, m, G)
    base = os.path.join(HERE, f"{a.workload}_p{a.p}")
    np.save(base + "_sketch.npy", Z)
    out = dict(
        workload=a.workload, mesh_seed=a.seed, n=n, p=a.p, stored=k,
        eigenvalues=[float(x) for x in lam], residuals=[float(x) for x in r_chk],
        clusters=[[int(x), int(y)] for x, y in metrics.clusters(lam)],
        sketch=dict(file=os.path.basename(base + "_sketch.npy"), rows=SKETCH_ROWS, seed=SKETCH_SEED,
                    definition="Z = G^T (sqrt(m) * Y), G = synth.gaussian_matrix(n, rows, seed)"),
        oracle=dict(method="plain subspace iteration (Algorithm 1), two inverse iterations per "
                           "Rayleigh-Ritz step, SuperLU factor of S - mu M, seeded random start",
                    q=q, mu=mu, eps=a.eps, iterations=total_it, start_seed=a.start_seed),
        history=[float(x) for x in hist],
        checks=dict(max_residual=float(r_chk.max()), m_orthonormality=orth,
                    inertia_below_upper=below_hi, inertia_below_lower=below_lo),
        seconds=round(time.perf_counter() - t0, 1),
    )
    with open(base + ".json", "w") as f:
        json.dump(out, f, indent=1)
    print(f"[golden] wrote {base}.json ({out['seconds']} s)", flush=True)


if __name__ == "__main__":
    main()
