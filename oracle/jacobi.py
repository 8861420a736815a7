"""Dense symmetric (generalized) eigensolver by the cyclic Jacobi method.

The paper solves the dense eigenproblems (the coarsest level of Algorithm 2
and the reduced q x q problem of Algorithm 1) with a library direct solver;
the oracle uses the classical two-sided Jacobi method instead, which is short
and obviously correct:

* each rotation J(p, q, theta) zeroes the (p, q) entry of C <- J^T C J
  (angle from the symmetric 2x2 Schur decomposition: tau = (c_qq - c_pp) /
  (2 c_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)), c = 1/sqrt(1+t^2),
  s = t c);
* a sweep visits every pair once in round-robin (tournament) order, n/2
  disjoint pairs per round, so the rotations of one round commute and are
  applied together;
* sweeps repeat until every off-diagonal entry is below tol * ||C||_F.

The generalized problem S x = lambda M x (M symmetric positive definite) is
reduced with the Cholesky factor M = R^T R: C = R^-T S R^-1, x = R^-1 y.
"""
from __future__ import annotations

import numpy as np


def _round_robin(n):
    """n-1 rounds of n/2 disjoint pairs (n even) covering every pair once."""
    players = list(range(n))
    rounds = []
    for _ in range(n - 1):
        a = np.array(players[: n // 2])
        b = np.array(players[n // 2:][::-1])
        rounds.append((np.minimum(a, b), np.maximum(a, b)))
        players = [players[0]] + [players[-1]] + players[1:-1]
    return rounds


def jacobi_eigh(C, tol=1e-15, max_sweeps=60):
    """All eigenpairs of the symmetric matrix C, ascending.

    Returns (lam, V, sweeps) with C V = V diag(lam), V orthogonal."""
    C = np.array(C, dtype=np.float64, copy=True)
    n = C.shape[0]
    if n == 1:
        return C.diagonal().copy(), np.ones((1, 1)), 0
    if not np.allclose(C, C.T, rtol=0, atol=1e-12 * max(1.0, np.abs(C).max())):
        raise ValueError("jacobi_eigh: matrix is not symmetric")
    C = 0.5 * (C + C.T)
    m = n + (n % 2)
    if m != n:  # pad with an isolated dummy row/column
        Cp = np.zeros((m, m))
        Cp[:n, :n] = C
        C = Cp
    Vt = np.eye(m)          # V^T, so that every update is a row update
    rounds = _round_robin(m)
    norm = np.linalg.norm(C)
    thresh = tol * (norm if norm > 0 else 1.0)
    sweeps = 0

    def rotate_rows(A, p, q, c, s):
        Ap, Aq = A[p, :], A[q, :]
        A[p, :], A[q, :] = c[:, None] * Ap - s[:, None] * Aq, s[:, None] * Ap + c[:, None] * Aq

    for sweeps in range(1, max_sweeps + 1):
        rotated = False
        for p, q in rounds:
            apq = C[p, q]
            act = np.abs(apq) > thresh
            if not act.any():
                continue
            rotated = True
            app, aqq = C[p, p], C[q, q]
            with np.errstate(divide="ignore", invalid="ignore"):
                tau = np.where(act, (aqq - app) / (2.0 * np.where(act, apq, 1.0)), 0.0)
            sgn = np.where(tau >= 0, 1.0, -1.0)
            t = np.where(act, sgn / (np.abs(tau) + np.sqrt(1.0 + tau * tau)), 0.0)
            c = 1.0 / np.sqrt(1.0 + t * t)
            s = t * c
            # C <- J^T C J: rotate the rows, then (C symmetric) the rows of
            # the transpose; V <- V J is a row rotation of V^T.
            rotate_rows(C, p, q, c, s)
            C = np.ascontiguousarray(C.T)
            rotate_rows(C, p, q, c, s)
            rotate_rows(Vt, p, q, c, s)
        if not rotated:
            break
    V = Vt.T
    lam = np.diag(C)[:n].copy()
    V = V[:n, :n]
    order = np.argsort(lam, kind="stable")
    return lam[order], V[:, order], sweeps


def cholesky_upper(M):
    """Upper Cholesky factor R of an SPD matrix, M = R^T R (column-by-column
    definition, no library call)."""
    M = np.array(M, dtype=np.float64)
    n = M.shape[0]
    R = np.zeros_like(M)
    for j in range(n):
        s = M[j, j] - R[:j, j] @ R[:j, j]
        if s <= 0:
            raise np.linalg.LinAlgError("cholesky_upper: matrix is not positive definite")
        R[j, j] = np.sqrt(s)
        R[j, j + 1:] = (M[j, j + 1:] - R[:j, j] @ R[:j, j + 1:]) / R[j, j]
    return R


def jacobi_gep(S, M, tol=1e-15):
    """All eigenpairs of S x = lambda M x (S symmetric, M SPD), ascending,
    eigenvectors M-orthonormal (X^T M X = I)."""
    S = np.asarray(S, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    R = cholesky_upper(M)
    Rinv = np.linalg.solve(R, np.eye(len(R)))      # R^-1 (triangular)
    C = Rinv.T @ S @ Rinv
    C = 0.5 * (C + C.T)
    lam, Y, _ = jacobi_eigh(C, tol=tol)
    return lam, Rinv @ Y


def jacobi_gep_diag(S, m, tol=1e-15):
    """Generalized problem with a diagonal mass matrix given as the vector m:
    C = M^-1/2 S M^-1/2, x = M^-1/2 y."""
    S = np.asarray(S.todense() if hasattr(S, "todense") else S, dtype=np.float64)
    r = 1.0 / np.sqrt(np.asarray(m, dtype=np.float64))
    C = r[:, None] * S * r[None, :]
    lam, Y, _ = jacobi_eigh(0.5 * (C + C.T), tol=tol)
    return lam, r[:, None] * Y


def sign_fix(X):
    """Make every column deterministic: its largest-magnitude entry positive
    (lowest index on ties)."""
    X = np.array(X, copy=True)
    idx = np.argmax(np.abs(X), axis=0)
    s = np.sign(X[idx, np.arange(X.shape[1])])
    s[s == 0] = 1.0
    return X * s[None, :]
