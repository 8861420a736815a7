"""Derivatives of eigenpairs of S x = lambda M x with respect to the vertex
positions (dense FP64 reference for the adjoint).

Plain definitions, written with PyTorch CPU autograd for the assembly part:

* a^T S(V) b = sum over triangles and corners of cot(theta)/2 (a_i - a_j)(b_i - b_j)
  over the edge (i, j) opposite the corner (eq. massStiffMatrices with the
  cotangent formula);
* a^T M(V) b = sum_i m_i(V) a_i b_i, m_i = rho_i sum_{t containing i} area(t)/3
  (barycentric lumping), or rho_i times the circumcentric dual area (each
  corner's cot(theta) |e|^2 / 8 over its opposite edge e, to both ends of e).

Eigenvalue derivative (simple eigenvalue, x^T M x = 1):
    d lambda_k = x_k^T (dS - lambda_k dM) x_k.
Eigenvector part of a loss with gradient g_k = dL/dx_k: with all n eigenpairs,
    w_k = sum_{j not in cluster(k)} x_j (x_j^T g_k) / (lambda_j - lambda_k),
    dL = -sum_k w_k^T (dS - lambda_k dM) x_k - 1/2 sum_{j,k in one cluster} G_jk x_j^T dM x_k,
with G_jk the symmetrised x_j^T g_k.  The cluster form is exact for losses
that do not change under rotations inside a cluster (the reading taken for
near-degenerate eigenvalues, e.g. the sphere's 2l+1 multiplets); for simple
eigenvalues it equals the textbook formula.

Dirichlet condition (Section 5, surfaces with boundary): the problem keeps the
interior rows and columns of S and M, so for vectors extended by zero to the
boundary vertices a^T S_II b = a~^T S b~ and a^T M_II b = a~^T M b~.  The
derivatives above therefore hold unchanged with every vector (x_k, w_k and the
cluster terms) extended by zero; only the eigenpairs come from the interior
problem, and dL/dx_k is read on the interior rows.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl
import torch

from .assembly import assemble, dirichlet


def _corner_terms(Vt, Ft):
    """cot of the angle at each corner and the opposite edge (i, j)."""
    out = []
    for c in range(3):
        i, j = (c + 1) % 3, (c + 2) % 3
        P = Vt[Ft[:, c]]
        u = Vt[Ft[:, i]] - P
        w = Vt[Ft[:, j]] - P
        cot = (u * w).sum(1) / torch.linalg.norm(torch.cross(u, w, dim=1), dim=1)
        out.append((cot, Ft[:, i], Ft[:, j]))
    return out


def bilinear_S(Vt, Ft, A, B):
    """sum_k a_k^T S(V) b_k for the columns of A and B (torch, n x k)."""
    tot = 0.0
    for cot, i, j in _corner_terms(Vt, Ft):
        tot = tot + (0.5 * cot[:, None] * (A[i] - A[j]) * (B[i] - B[j])).sum()
    return tot


def lumped_mass_torch(Vt, Ft, rho=None, lumping="barycentric"):
    """Lumped masses as a function of the positions: barycentric (area / 3 per
    corner) or circumcentric (each corner's cot times its opposite edge's
    squared length / 8, to both ends of that edge)."""
    m = torch.zeros(Vt.shape[0], dtype=Vt.dtype)
    if lumping == "barycentric":
        a, b, c = Vt[Ft[:, 0]], Vt[Ft[:, 1]], Vt[Ft[:, 2]]
        area = 0.5 * torch.linalg.norm(torch.cross(b - a, c - a, dim=1), dim=1)
        for k in range(3):
            m = m.index_add(0, Ft[:, k], area / 3.0)
    elif lumping == "voronoi":
        for cot, i, j in _corner_terms(Vt, Ft):
            t = cot * ((Vt[i] - Vt[j]) ** 2).sum(1) / 8.0
            m = m.index_add(0, i, t).index_add(0, j, t)
    else:
        raise ValueError(lumping)
    if rho is not None:
        m = m * torch.as_tensor(rho, dtype=Vt.dtype)
    return m


def clusters_of(lam, gap=1e-2):
    """Cluster id per eigenvalue: a new cluster starts at a relative gap >= gap."""
    cl = np.zeros(len(lam), dtype=np.int64)
    for j in range(1, len(lam)):
        den = abs(lam[j]) if lam[j] != 0 else 1.0
        cl[j] = cl[j - 1] + (1 if (lam[j] - lam[j - 1]) / den >= gap else 0)
    return cl


def reference_gradient(V, F, p, grad_lam=None, grad_X=None, density=None, gap=1e-2, boundary="neumann",
                       lumping="barycentric"):
    """dL/dV (n x 3) for L with dL/dlambda = grad_lam(lam[:p]) and
    dL/dX = grad_X(X[:, :p]) at the exact eigenpairs (dense, all pairs of the
    problem; the dense generalized eigensolver is a library routine).
    boundary="dirichlet" takes the eigenpairs of the interior problem, the
    eigenvectors extended by zero to the whole mesh.  Returns
    (grad, lam[:p], X[:, :p]) with X over all mesh vertices."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    S, m = assemble(V, F, lumping=lumping, density=density)
    if boundary == "dirichlet":
        Si, mi, interior = dirichlet(S, m, F)
        lam, Xi = sl.eigh(Si.toarray(), np.diag(mi))
        X = np.zeros((len(V), len(lam)))
        X[interior] = Xi
    elif boundary == "neumann":
        lam, X = sl.eigh(S.toarray(), np.diag(m))
    else:
        raise ValueError("boundary must be 'neumann' or 'dirichlet'")
    n = len(lam)
    nv = len(V)
    x = X[:, :p]
    gl = np.zeros(p) if grad_lam is None else np.asarray(grad_lam(lam[:p]), dtype=np.float64)
    W = np.zeros((nv, p))
    Gam = np.zeros((n, p))
    if grad_X is not None:
        gX = np.asarray(grad_X(x), dtype=np.float64)
        C = X.T @ gX                                  # x_j^T g_k, all j
        cl = clusters_of(lam, gap)
        for k in range(p):
            for j in range(n):
                if cl[j] != cl[k]:
                    W[:, k] += X[:, j] * (C[j, k] / (lam[j] - lam[k]))
                else:
                    ckj = C[k, j] if j < p else 0.0
                    Gam[j, k] = C[j, k] if j == k else 0.5 * (C[j, k] + ckj)
    Vt = torch.tensor(V, requires_grad=True)
    Ft = torch.tensor(F)
    xt = torch.tensor(x)
    lt = torch.tensor(lam[:p])
    m_t = lumped_mass_torch(Vt, Ft, density, lumping)
    # eigenvalue part: sum_k gl_k x_k^T (S - lam_k M) x_k
    phi = bilinear_S(Vt, Ft, xt * torch.tensor(gl)[None, :], xt)
    phi = phi - (m_t[:, None] * xt * xt * (torch.tensor(gl) * lt)[None, :]).sum()
    # eigenvector part
    Wt = torch.tensor(W)
    phi = phi - bilinear_S(Vt, Ft, Wt, xt) + (m_t[:, None] * Wt * xt * lt[None, :]).sum()
    Yt = torch.tensor(X @ Gam)                         # sum_j x_j G_jk
    phi = phi - 0.5 * (m_t[:, None] * Yt * xt).sum()
    phi.backward()
    return Vt.grad.numpy(), lam[:p], x
