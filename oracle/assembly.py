"""Stiffness and mass matrices of the P1 finite element discretisation.

Section 3.1, eq. (massStiffMatrices): S_ij = int grad(phi_i) . grad(phi_j) dA
and M_ij = int phi_i phi_j dA over the piecewise-linear hat functions phi_i of
the triangle mesh; the discrete eigenproblem is S Phi = lambda M Phi
(eq. eigenProb).  The paper uses a diagonal (lumped) mass matrix on the finest
level (Section 5, termination criterion paragraph).

Readings
--------
* The explicit P1 formulas are the classical ones the paper cites: on a
  triangle t with angle theta_k opposite the edge (i, j),
  S_ij += -cot(theta_k)/2 and S_ii = -sum_{j != i} S_ij.
* Lumping (formula deferred by the paper): ``"barycentric"`` is the row-sum of
  the consistent P1 mass matrix, m_i = sum_{t containing i} area(t)/3;
  ``"voronoi"`` is the circumcentric dual-cell area
  m_i = sum_t (|e_ij|^2 cot(theta_k) + |e_ik|^2 cot(theta_j)) / 8, exact for the
  flat grid pin (it assumes non-obtuse triangles).
* An optional per-vertex density multiplies m_i.
* Surfaces with boundary (Section 5, paragraph "Surface with boundary"): the
  natural (Neumann) condition needs nothing beyond the assembly above; the
  Dirichlet condition u = 0 on the boundary keeps the interior vertices only,
  i.e. the principal submatrix of S and the lumped masses there.  Boundary
  vertices are the endpoints of edges that belong to exactly one triangle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def triangle_areas(V, F):
    """Area of every triangle: |(b - a) x (c - a)| / 2 with the products and
    sums taken in a fixed order (x, y, z)."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    e1 = b - a
    e2 = c - a
    cx = e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1]
    cy = e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2]
    cz = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    return 0.5 * np.sqrt(cx * cx + cy * cy + cz * cz)


def surface_area(V, F):
    """Total area, summed sequentially in triangle order."""
    return float(np.cumsum(triangle_areas(V, F))[-1])


def _cot_at(V, F, k):
    """cot of the angle at corner k of every triangle (opposite edge = the
    other two corners)."""
    i, j = (k + 1) % 3, (k + 2) % 3
    p = V[F[:, k]]
    u = V[F[:, i]] - p
    w = V[F[:, j]] - p
    dot = np.sum(u * w, axis=1)
    cr = np.cross(u, w)
    return dot / np.linalg.norm(cr, axis=1)


def stiffness(V, F):
    """Cotangent stiffness matrix S (n x n CSR, symmetric positive semi-definite,
    S @ 1 = 0)."""
    n = len(V)
    rows, cols, vals = [], [], []
    for k in range(3):
        i, j = F[:, (k + 1) % 3], F[:, (k + 2) % 3]
        w = -0.5 * _cot_at(V, F, k)           # contribution to S_ij and S_ji
        rows += [i, j, i, j]
        cols += [j, i, i, j]
        vals += [w, w, -w, -w]
    S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    return S


def lumped_mass(V, F, lumping="barycentric", density=None):
    """Diagonal of the lumped mass matrix M (length-n vector)."""
    n = len(V)
    if lumping == "barycentric":
        A = triangle_areas(V, F)
        m = np.zeros(n)
        for k in range(3):
            np.add.at(m, F[:, k], A / 3.0)
    elif lumping == "voronoi":
        m = np.zeros(n)
        for k in range(3):
            # vertex k gets (|e_ki|^2 cot(theta_j) + |e_kj|^2 cot(theta_i)) / 8
            i, j = (k + 1) % 3, (k + 2) % 3
            eki = np.sum((V[F[:, i]] - V[F[:, k]]) ** 2, axis=1)
            ekj = np.sum((V[F[:, j]] - V[F[:, k]]) ** 2, axis=1)
            np.add.at(m, F[:, k], (eki * _cot_at(V, F, j) + ekj * _cot_at(V, F, i)) / 8.0)
    else:
        raise ValueError(lumping)
    if density is not None:
        m = m * np.asarray(density, dtype=np.float64)
    return m


def assemble(V, F, lumping="barycentric", density=None):
    """(S, m): cotangent stiffness (CSR) and lumped mass diagonal."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    return stiffness(V, F), lumped_mass(V, F, lumping, density)


def consistent_mass(V, F):
    """Consistent P1 mass matrix M_ij = int phi_i phi_j (area/6 on the diagonal,
    area/12 off the diagonal per triangle); used only to check the lumping."""
    n = len(V)
    A = triangle_areas(V, F)
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(F[:, a])
            cols.append(F[:, b])
            vals.append(A / 6.0 if a == b else A / 12.0)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def boundary_vertices(F, nv):
    """Boolean mask of the vertices on the mesh boundary (endpoints of edges
    that belong to exactly one triangle)."""
    F = np.asarray(F, dtype=np.int64)
    E = np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), axis=1)
    edges, count = np.unique(E, axis=0, return_counts=True)
    on = np.zeros(nv, dtype=bool)
    on[edges[count == 1].ravel()] = True
    return on


def dirichlet(S, m, F):
    """(S_II, m_I, interior): the Dirichlet problem on the interior vertices
    (ascending mesh indices) of the mesh with triangles F."""
    interior = np.flatnonzero(~boundary_vertices(F, S.shape[0]))
    S = sp.csr_matrix(S)
    return S[interior][:, interior].tocsr(), np.asarray(m)[interior], interior
