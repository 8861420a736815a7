"""Error measures for computed eigenpairs against reference eigenpairs.

Eigenvectors of (near-)degenerate eigenvalues are defined only up to a
rotation inside their cluster (the sphere's 2l+1-fold eigenvalues, the torus's
+-m pairs), so eigenvectors are compared cluster-wise: a cluster is a maximal
run of reference eigenvalues with relative gaps below ``gap``, and the error
of a computed vector x_i is its M-norm distance to the span of the reference
cluster containing index i, ||x_i - Y_C Y_C^T M x_i||_M (Y_C M-orthonormal).
The paper measures eigenvector differences by the relative L2 norm (Section 5,
termination criterion); with ||x_i||_M = 1 this is the same quantity.

Sketches (for meshes whose reference eigenvectors are too large to keep)
-----------------------------------------------------------------------
With a fixed Gaussian matrix G (n x r) and M diagonal, the sketch of a block X
is W = G^T (M^{1/2} X) (r x k).  For an M-orthonormal reference cluster Y_C,
Z_C = G^T M^{1/2} Y_C, and a vector x = Y_C c + e with e M-orthogonal to Y_C
has sketch Z_C c + G^T M^{1/2} e, whose second part is independent of Z_C and
Gaussian with variance ||e||_M^2 per entry.  Removing the least-squares fit on
the columns of Z_C therefore leaves a residual whose squared norm has expected
value (r - |C|) ||e||_M^2: ``sketch_vector_err`` returns that estimate of the
cluster-aware error of ``eigenvector_err`` (a chi-square estimate with
r - |C| degrees of freedom).  ``sketch_projector_diff`` compares the
rotation-invariant sketches W W^T and Z_C Z_C^T of two bases of a whole
cluster.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def clusters(lam, gap=1e-2):
    """List of index ranges [a, b) grouping eigenvalues whose consecutive
    relative gap (lam[i+1]-lam[i])/lam[i+1] is below ``gap``."""
    lam = np.asarray(lam)
    out, a = [], 0
    for i in range(len(lam) - 1):
        den = abs(lam[i + 1]) if lam[i + 1] != 0 else 1.0
        if (lam[i + 1] - lam[i]) / den >= gap:
            out.append((a, i + 1))
            a = i + 1
    out.append((a, len(lam)))
    return out


def eigenvalue_rel_err(lam, lam_ref, floor=None):
    lam, lam_ref = np.asarray(lam), np.asarray(lam_ref)
    den = np.abs(lam_ref)
    if floor is not None:
        den = np.maximum(den, floor)
    return np.abs(lam - lam_ref) / den


def eigenvector_err(X, Y, M, lam_ref, gap=1e-2):
    """Cluster-aware M-norm error of each column of X against the reference
    basis Y (which must hold every cluster that the columns of X touch)."""
    Mop = sp.diags(M) if not sp.issparse(M) and np.ndim(M) == 1 else M
    err = np.empty(X.shape[1])
    MX = Mop @ X
    for a, b in clusters(lam_ref, gap):
        if a >= X.shape[1]:
            break
        Yc = Y[:, a:b]
        for i in range(a, min(b, X.shape[1])):
            c = Yc.T @ MX[:, i]
            d = X[:, i] - Yc @ c
            err[i] = np.sqrt(max(d @ (Mop @ d), 0.0)) / np.sqrt(max(X[:, i] @ MX[:, i], 1e-300))
    return err


def m_orthonormality(X, M):
    Mop = sp.diags(M) if not sp.issparse(M) and np.ndim(M) == 1 else M
    G = X.T @ (Mop @ X)
    return float(np.abs(G - np.eye(G.shape[0])).max())


def sketch(X, m, G):
    """W = G^T (m^{1/2} * X) for a diagonal mass m (see the module notes)."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    return G.T @ (np.sqrt(np.asarray(m, dtype=np.float64))[:, None] * X)


def sketch_vector_err(w, Zc, xnorm=None):
    """Estimate of ||x - Y_C Y_C^T M x||_M / ||x||_M from the sketch w of x
    (length r) and the sketch Zc (r x |C|) of the M-orthonormal reference
    cluster Y_C.  ``xnorm`` = ||x||_M if known (else estimated as |w|/sqrt(r),
    since E|w|^2 = r ||x||_M^2)."""
    w = np.asarray(w, dtype=np.float64)
    r, c = Zc.shape
    if c >= r:
        raise ValueError("sketch has too few rows for this cluster")
    coef, *_ = np.linalg.lstsq(Zc, w, rcond=None)
    res = w - Zc @ coef
    out = np.sqrt(float(res @ res) / (r - c))
    if xnorm is None:
        xnorm = np.sqrt(float(w @ w) / r)
    return out / max(float(xnorm), 1e-300)


def sketch_projector_diff(W, Zc):
    """|| W W^T - Zc Zc^T ||_F / || Zc Zc^T ||_F for the sketches of two bases
    of the same cluster (invariant to rotations and signs inside the cluster)."""
    A = W @ W.T
    B = Zc @ Zc.T
    return float(np.linalg.norm(A - B) / np.linalg.norm(B))
