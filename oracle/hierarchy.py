"""Hierarchy of nested function spaces (Section 4.1) and the parameter rules of
Algorithm 2.

* Level sizes: n^{T-1} = max(ceil(1.5 p), 1000) (eq. nT-1) and
  n^tau = g n^{tau+1} (eq. growthRate).
* Vertex hierarchy: farthest point sampling, Algorithm 3, with the distance
  field kept up to date locally around each inserted vertex; distances are
  Dijkstra distances on the edge graph weighted by Euclidean edge length.
* Prolongation U^tau (eq. radius, eq. basis and the row normalisation):
  weights (1 - d/rho)_+ between a fine vertex and the coarse vertices within
  the radius rho, normalised to sum to one.
* Galerkin operators S^{tau+1} = U^T S^tau U, M^{tau+1} = U^T M^tau U
  (Algorithm 2, the restriction loop).

Readings (the paper is garbled or silent here)
---------------------------------------------
* Growth rate: eq. (growthRate) writes the T-th root, which does not reach
  n^0 from n^{T-1} in T-1 steps; the default is the (T-1)-th root and
  n^tau = round(g^(T-1-tau) n^{T-1}); ``growth_mode=1`` keeps the literal
  T-th root (levels then stop short of n^0, as printed).
* Number of levels: 2 when p <= 200, else 3 (Section 4.1, number of levels).
* Index convention of U^tau: rows are the fine vertices j of level tau,
  columns the coarse vertices i of level tau+1 (so that U^tau maps coarse to
  fine as the text says and U 1 = 1 makes constants representable).  The
  radius is computed from the coarse count n^{tau+1}, so that every disk
  holds about sigma coarse samples.  A fine vertex with no coarse vertex
  inside the radius takes weight 1 on its nearest coarse vertex.
* The random start vertex of Algorithm 3 is ``seed mod n``; farthest-point
  ties go to the lowest vertex index; nearest-vertex ties to the lowest coarse
  index.
* Level-local vertex order: level 0 keeps the mesh order; every coarser
  level lists its vertices in insertion order, so V^{tau+1} is a prefix of
  V^tau for tau >= 1.
"""
from __future__ import annotations

import heapq
import math

import numpy as np
import scipy.sparse as sp

from .assembly import surface_area


def num_levels(p):
    """Two levels when p <= 200, three otherwise (Section 4.1)."""
    return 2 if p <= 200 else 3


def coarsest_size(p):
    """n^{T-1} = max(ceil(1.5 p), 1000) (eq. nT-1)."""
    return max(int(math.ceil(1.5 * p)), 1000)


def level_sizes(n0, T, n_coarsest, growth_mode=0):
    """[n^0, n^1, ..., n^{T-1}]."""
    if T < 1:
        raise ValueError("T >= 1")
    if T == 1:
        return [n0]
    nc = min(n_coarsest, n0)
    root = (T - 1) if growth_mode == 0 else T
    g = (n0 / nc) ** (1.0 / root)
    sizes = [n0]
    for tau in range(1, T - 1):
        sizes.append(int(min(n0, max(nc, round(g ** (T - 1 - tau) * nc)))))
    sizes.append(nc)
    return sizes


def shift_index(p, alpha=0.1):
    """j = floor(alpha p), 0-based on the ascending Ritz values (Alg. 2)."""
    return int(math.floor(alpha * p + 1e-12))


def edge_graph(V, F):
    """Undirected edge graph in CSR form with Euclidean edge lengths
    (squared length summed x, y, z in order, then the square root)."""
    n = len(V)
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]).astype(np.int64)
    e = np.unique(np.sort(e, axis=1), axis=0)
    i = np.concatenate([e[:, 0], e[:, 1]])
    j = np.concatenate([e[:, 1], e[:, 0]])
    order = np.lexsort((j, i))
    i, j = i[order], j[order]
    d = V[i] - V[j]
    w = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, i + 1, 1)
    indptr = np.cumsum(indptr)
    return indptr, j, w


def _relax_from(src, dist, indptr, nbr, w):
    """Lower ``dist`` to min(dist, graph distance from src) by Dijkstra,
    visiting only vertices whose distance improves."""
    dist[src] = 0.0
    heap = [(0.0, src)]
    while heap:
        dv, v = heapq.heappop(heap)
        if dv > dist[v]:
            continue
        for k in range(indptr[v], indptr[v + 1]):
            u = nbr[k]
            nd = dv + w[k]
            if nd < dist[u]:
                dist[u] = nd
                heapq.heappush(heap, (nd, u))


def farthest_point_sampling(V, F, sizes, seed=0, graph=None):
    """Algorithm 3.  ``sizes`` = [n^0, ..., n^{T-1}].  Returns the insertion
    order ``order`` (length n^1, or n^0 if T == 1) so that
    V^tau = order[:n^tau] for tau >= 1."""
    n = len(V)
    T = len(sizes)
    if T == 1:
        return np.arange(n)
    indptr, nbr, w = graph or edge_graph(V, F)
    dist = np.full(n, np.inf)
    start = int(seed % n)
    order = [start]
    _relax_from(start, dist, indptr, nbr, w)
    target = sizes[1]
    while len(order) < target:
        s = int(np.argmax(dist))          # farthest; lowest index on ties
        if not dist[s] > 0:
            raise ValueError("farthest point sampling: mesh is disconnected or too small")
        order.append(s)
        _relax_from(s, dist, indptr, nbr, w)
    return np.asarray(order, dtype=np.int64)


def _ball(src, rho, n, indptr, nbr, w):
    """Graph distances from src to every vertex closer than rho."""
    dist = {src: 0.0}
    done = {}
    heap = [(0.0, src)]
    while heap:
        dv, v = heapq.heappop(heap)
        if v in done:
            continue
        if dv >= rho:
            break
        done[v] = dv
        for k in range(indptr[v], indptr[v + 1]):
            u = nbr[k]
            nd = dv + w[k]
            if nd < dist.get(u, np.inf):
                dist[u] = nd
                heapq.heappush(heap, (nd, u))
    return done


def _nearest_coarse(coarse, n, indptr, nbr, w):
    """For every vertex: the coarse sample at the smallest graph distance,
    lowest coarse index on ties (lexicographic (distance, index) Dijkstra)."""
    key = [(np.inf, np.inf)] * n
    heap = []
    for ci, g in enumerate(coarse):
        key[g] = (0.0, ci)
        heap.append((0.0, ci, g))
    heapq.heapify(heap)
    lab = np.full(n, -1, dtype=np.int64)
    while heap:
        dv, ci, v = heapq.heappop(heap)
        if (dv, ci) > key[v]:
            continue
        lab[v] = ci
        for k in range(indptr[v], indptr[v + 1]):
            u = nbr[k]
            cand = (dv + w[k], ci)
            if cand < key[u]:
                key[u] = cand
                heapq.heappush(heap, (cand[0], ci, u))
    return lab


def prolongation(V, F, fine_verts, coarse_verts, sigma=7.0, area=None, graph=None):
    """U^tau (n^tau x n^{tau+1} CSR): rows = fine level vertices (level-local
    order), columns = coarse level vertices.  eq. (radius) with the coarse
    count, eq. (basis), row normalisation."""
    n = len(V)
    indptr, nbr, w = graph or edge_graph(V, F)
    A = surface_area(V, F) if area is None else area
    nc = len(coarse_verts)
    rho = math.sqrt(sigma * A / (nc * math.pi))
    pos = np.full(n, -1, dtype=np.int64)
    pos[np.asarray(fine_verts)] = np.arange(len(fine_verts))
    rows, cols, vals = [], [], []
    for ci, g in enumerate(coarse_verts):
        for v, d in _ball(int(g), rho, n, indptr, nbr, w).items():
            j = pos[v]
            if j >= 0:
                wt = 1.0 - d / rho
                if wt > 0.0:
                    rows.append(j)
                    cols.append(ci)
                    vals.append(wt)
    Ut = sp.csr_matrix((vals, (rows, cols)), shape=(len(fine_verts), nc))
    Ut.sum_duplicates()
    rs = np.asarray(Ut.sum(axis=1)).ravel()
    empty = np.nonzero(rs == 0)[0]
    if len(empty):
        lab = _nearest_coarse(np.asarray(coarse_verts), n, indptr, nbr, w)
        fv = np.asarray(fine_verts)[empty]
        extra = sp.csr_matrix((np.ones(len(empty)), (empty, lab[fv])), shape=Ut.shape)
        Ut = Ut + extra
        rs = np.asarray(Ut.sum(axis=1)).ravel()
    U = sp.diags(1.0 / rs) @ Ut
    U = U.tocsr()
    U.sort_indices()
    return U, rho


def build_hierarchy(V, F, S0, m0, p, levels=0, n_coarsest=0, sigma=7.0, seed=0, growth_mode=0):
    """Levels 0..T-1 with their vertex sets, prolongations and Galerkin
    operators.  Returns a list of dicts: verts (mesh ids in level order),
    S, M (level 0: the diagonal vector m0; coarser: CSR), U (tau < T-1), rho."""
    n = len(V)
    T = levels or num_levels(p)
    nc = n_coarsest or coarsest_size(p)
    sizes = level_sizes(n, T, nc, growth_mode)
    graph = edge_graph(V, F)
    order = farthest_point_sampling(V, F, sizes, seed=seed, graph=graph)
    area = surface_area(V, F)
    lv = [dict(verts=np.arange(n), S=S0.tocsr(), M=np.asarray(m0, dtype=np.float64))]
    for tau in range(1, T):
        lv.append(dict(verts=order[: sizes[tau]]))
    for tau in range(T - 1):
        U, rho = prolongation(V, F, lv[tau]["verts"], lv[tau + 1]["verts"], sigma, area, graph)
        lv[tau]["U"], lv[tau]["rho"] = U, rho
        Mt = lv[tau]["M"]
        Mop = sp.diags(Mt) if not sp.issparse(Mt) else Mt
        lv[tau + 1]["S"] = (U.T @ lv[tau]["S"] @ U).tocsr()
        lv[tau + 1]["M"] = (U.T @ Mop @ U).tocsr()
    return lv
