"""The Subspace Iteration Method (Algorithm 1) and its convergence test.

Algorithm 1 (Section 3.2): factor S - mu M once, then repeat
    solve (S - mu M) Psi = M Phi           (inverse iteration)
    Sbar = Psi^T S Psi, Mbar = Psi^T M Psi (reduced matrices)
    Sbar Phibar = Mbar Phibar Lambdabar    (dense eigenproblem)
    Phi <- Psi Phibar                      (update)
until the first p pairs pass the convergence test eq. (conv2):
    ||S phi_i - lambda_i M phi_i||_{M^-1} / ||S phi_i||_{M^-1} < eps.

Section 4.2 adds two refinements used by the hierarchical solver: two inverse
iterations before each Rayleigh-Ritz step, and locking of the lowest
converged vectors once their residual is below eps/10 (they are not
inverse-iterated any more).  Section 5 (termination criterion) replaces the
M^-1-norm by the Euclidean norm on the coarse levels, where M is not diagonal.

Readings
--------
* eq. (conv2) is 0/0 for the constant eigenvector (lambda = 0).  Since
  ||S phi||_{M^-1} = |lambda| ||phi||_M for an eigenpair, the floored form
  r_i = ||S phi_i - lambda_i M phi_i||_{M^-1} / (max(|lambda_i|, lambda_c) ||phi_i||_M)
  is used for the test, with lambda_c the first Ritz value above
  1e-8 * lambda_{q-1}.  ``residual_conv2`` gives the paper's form as well.
* Locking takes the longest prefix of pairs with r_i < eps/10.
* The direct solver is a library sparse LU (SuperLU); the paper uses a
  sparse LDL^T.  Both solve the same linear systems.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .jacobi import jacobi_gep


def mass_operator(M):
    """Sparse matrix for M given either as a diagonal vector or a matrix."""
    if sp.issparse(M):
        return M.tocsr()
    M = np.asarray(M, dtype=np.float64)
    if M.ndim == 1:
        return sp.diags(M).tocsr()
    return sp.csr_matrix(M)


def subspace_size(p):
    """q = max(ceil(1.5 p), p + 8) (Section 3.2 subspace dimension; Alg. 2)."""
    return max(int(math.ceil(1.5 * p)), p + 8)


def _minv_norm_cols(R, m):
    return np.sqrt(np.sum(R * R / m[:, None], axis=0))


def residual_conv2(S, M, X, lam):
    """Paper form of eq. (conv2) in the M^-1-norm (M diagonal)."""
    m = np.asarray(M.diagonal() if sp.issparse(M) else M, dtype=np.float64)
    SX = S @ X
    R = SX - (m[:, None] * X) * lam[None, :]
    den = _minv_norm_cols(SX, m)
    with np.errstate(divide="ignore", invalid="ignore"):
        return _minv_norm_cols(R, m) / den


def lambda_floor(lam):
    """First Ritz value above 1e-8 * (largest Ritz value)."""
    lam = np.asarray(lam)
    top = np.max(np.abs(lam))
    above = lam[lam > 1e-8 * top]
    return float(above[0]) if len(above) else float(top if top > 0 else 1.0)


def residual(S, M, X, lam, lam_c=None, norm="minv"):
    """Floored relative residual (see module readings).

    norm = "minv": M^-1-norm of the residual over max(|lam|, lam_c) ||x||_M,
    M diagonal (finest level).  norm = "l2": Euclidean norms,
    ||S x - lam M x||_2 / (max(|lam|, lam_c) ||M x||_2) (coarse levels)."""
    lam = np.asarray(lam, dtype=np.float64)
    if lam_c is None:
        lam_c = lambda_floor(lam)
    Mop = mass_operator(M)
    SX = S @ X
    MX = Mop @ X
    R = SX - MX * lam[None, :]
    scale = np.maximum(np.abs(lam), lam_c)
    if norm == "minv":
        m = Mop.diagonal()
        num = _minv_norm_cols(R, m)
        xm = np.sqrt(np.sum(X * MX, axis=0))
        return num / (scale * xm)
    num = np.linalg.norm(R, axis=0)
    return num / (scale * np.linalg.norm(MX, axis=0))


def rayleigh_ritz(S, M, Psi, dense=jacobi_gep):
    """Reduced matrices, dense eigenproblem and update (Algorithm 1).  Returns (lam, Phi, Phibar, Sbar, Mbar)."""
    Mop = mass_operator(M)
    Sbar = Psi.T @ (S @ Psi)
    Mbar = Psi.T @ (Mop @ Psi)
    Sbar = 0.5 * (Sbar + Sbar.T)
    Mbar = 0.5 * (Mbar + Mbar.T)
    lam, Phibar = dense(Sbar, Mbar)
    return lam, Psi @ Phibar, Phibar, Sbar, Mbar


class ShiftedSolver:
    """(S - mu M)^-1 applied to blocks, by one sparse factorisation
    (the factorisation of Algorithm 1).

    ``symmetric=True`` factors with a symmetric fill-reducing ordering of
    A + A^T and without off-diagonal pivoting (SuperLU's symmetric mode):
    for mu below the spectrum A = S - mu M is symmetric positive definite,
    so static diagonal pivots are stable and the LU is an LDL^T in disguise
    (U = D L^T), with far less fill than the default column ordering.
    ``threads`` > 1 splits the right-hand sides into column chunks solved
    concurrently (the library releases the interpreter lock inside its solve
    for part of the work)."""

    def __init__(self, S, M, mu, symmetric=False, threads=1):
        self.mu = float(mu)
        A = (S - self.mu * mass_operator(M)).tocsc()
        if symmetric:
            self.lu = spla.splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                                options=dict(SymmetricMode=True))
        else:
            self.lu = spla.splu(A)
        self.threads = max(1, int(threads))

    def solve(self, B):
        B = np.asarray(B, dtype=np.float64)
        if self.threads == 1 or B.ndim == 1 or B.shape[1] < 2 * self.threads:
            return self.lu.solve(np.asfortranarray(B))
        from concurrent.futures import ThreadPoolExecutor
        cols = np.array_split(np.arange(B.shape[1]), self.threads)
        X = np.empty(B.shape, dtype=np.float64, order="F")

        def one(c):
            X[:, c[0]:c[-1] + 1] = self.lu.solve(np.asfortranarray(B[:, c[0]:c[-1] + 1]))
        with ThreadPoolExecutor(self.threads) as ex:
            list(ex.map(one, cols))
        return X


def sim(S, M, Phi0, p, eps, mu, max_iter=500, inverse_iterations=1, lock=False,
        norm="minv", history=None, solver=None):
    """Algorithm 1 with optional Section 4.2 refinements.

    Returns (lam[q], Phi[n, q], iterations, resid[q]); the first p pairs have
    passed the test (unless max_iter was hit: then resid shows it)."""
    Mop = mass_operator(M)
    Phi = np.array(Phi0, dtype=np.float64, copy=True)
    q = Phi.shape[1]
    solver = solver or ShiftedSolver(S, Mop, mu)
    locked = 0
    it = 0
    lam = np.zeros(q)
    r = np.full(q, np.inf)
    for it in range(1, max_iter + 1):
        Psi = Phi.copy()
        act = slice(locked, q)
        for _ in range(inverse_iterations):
            Psi[:, act] = solver.solve(Mop @ Psi[:, act])
        lam, Phi, _, _, _ = rayleigh_ritz(S, Mop, Psi)
        r = residual(S, Mop, Phi, lam, norm=norm)
        if history is not None:
            history.append(r[:p].max())
        if np.all(r[:p] < eps):
            break
        if lock:
            ok = r < eps / 10.0
            locked = int(np.argmin(ok)) if not ok.all() else q
            locked = min(locked, p)
    return lam, Phi, it, r


def sim_lowest(S, M, p, eps=1e-10, seed=0, mu=None, q=None, max_iter=500):
    """Plain SIM from a seeded random start (the oracle's large-mesh path).

    mu defaults to a small negative shift -1e-6 * tr(S)/tr(M), which makes
    S - mu M positive definite on closed meshes.  Returns the first p pairs,
    ascending, and the iteration count."""
    Mop = mass_operator(M)
    n = S.shape[0]
    q = q or subspace_size(p)
    if mu is None:
        mu = -1e-6 * S.diagonal().sum() / Mop.diagonal().sum()
    rng = np.random.default_rng(seed)
    Phi0 = rng.standard_normal((n, q))
    lam, Phi, it, r = sim(S, Mop, Phi0, p, eps, mu, max_iter=max_iter)
    return lam[:p], Phi[:, :p], it, r[:p]
