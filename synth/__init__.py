"""Seeded synthetic triangle meshes shaped like the paper's workloads.

This module only generates inputs (vertex positions, triangles, per-vertex
densities and random target fields).  It holds none of the eigensolver's
arithmetic: no stiffness or mass assembly, no hierarchy, no solver.  Both the
oracle tests and the GPU path draw their inputs from here.

The paper evaluates on scanned and CAD meshes of 85k-820k vertices and on
regular spheres of 10k-1M vertices (Section 5, Fig. error); those meshes are
not available, so noisy spheres and tori of the same sizes stand in for them.

Every generator is deterministic given its arguments and ``seed``
(``numpy.random.default_rng(seed)``).  Triangles are returned as int32
``(nf, 3)`` arrays with counter-clockwise orientation seen from outside,
vertices as float64 ``(nv, 3)`` arrays.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "icosahedron", "icosphere", "geodesic_icosphere", "torus", "rectangle_grid",
    "radial_jitter", "isotropic_noise", "gaussian_bumps", "random_density", "gaussian_matrix", "batch_mesh",
    "mean_edge_length", "config_mesh", "CONFIGS",
]


def icosahedron():
    """Unit icosahedron: 12 vertices, 20 outward-oriented faces."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int32)
    return v, f


def icosphere(k: int):
    """4:1 subdivided icosahedron projected to the unit sphere.

    ``k`` subdivisions give 10*4**k + 2 vertices and 20*4**k faces.
    """
    v, f = icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(k):
        cache = {}
        new_f = np.empty((4 * len(f), 3), dtype=np.int32)
        vv = list(verts)

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = np.add(vv[a], vv[b]) * 0.5
                p = p / np.linalg.norm(p)
                idx = len(vv)
                vv.append(tuple(p))
                cache[key] = idx
            return idx

        for i, (a, b, c) in enumerate(f):
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_f[4 * i + 0] = (a, ab, ca)
            new_f[4 * i + 1] = (b, bc, ab)
            new_f[4 * i + 2] = (c, ca, bc)
            new_f[4 * i + 3] = (ab, bc, ca)
        verts, f = vv, new_f
    return np.asarray(verts, dtype=np.float64), np.asarray(f, dtype=np.int32)


def geodesic_icosphere(nu: int):
    """Frequency-``nu`` geodesic sphere: every icosahedron face is split into
    nu*nu triangles and all points are projected to the unit sphere.

    Gives 10*nu**2 + 2 vertices and 20*nu**2 faces (nu = 324: 1,049,762
    vertices, 2,099,520 faces).
    """
    if nu < 1:
        raise ValueError("nu must be >= 1")
    v0, f0 = icosahedron()
    # global ids: 12 corners, then (nu-1) interior points per edge, then the
    # (nu-1)(nu-2)/2 interior points per face.
    edges = {}
    for a, b, c in f0:
        for x, y in ((a, b), (b, c), (c, a)):
            key = (min(x, y), max(x, y))
            if key not in edges:
                edges[key] = len(edges)
    assert len(edges) == 30
    n_edge_int = nu - 1
    n_face_int = (nu - 1) * (nu - 2) // 2
    nv = 12 + 30 * n_edge_int + 20 * n_face_int
    V = np.empty((nv, 3), dtype=np.float64)
    V[:12] = v0
    F = np.empty((20 * nu * nu, 3), dtype=np.int32)
    ii, jj = np.meshgrid(np.arange(nu + 1), np.arange(nu + 1), indexing="ij")
    mask = ii + jj <= nu
    I, J = ii[mask], jj[mask]
    face_base = 12 + 30 * n_edge_int
    for fi, (a, b, c) in enumerate(f0):
        # point (i, j) = A + (B-A) i/nu + (C-A) j/nu ; grid id map
        gid = np.full((nu + 1, nu + 1), -1, dtype=np.int64)
        gid[0, 0], gid[nu, 0], gid[0, nu] = a, b, c

        def edge_ids(x, y):
            e = edges[(min(x, y), max(x, y))]
            ids = 12 + e * n_edge_int + np.arange(n_edge_int)
            return ids if x < y else ids[::-1]   # ordered from x to y
        t = np.arange(1, nu)
        gid[t, 0] = edge_ids(a, b)           # along A->B (i)
        gid[0, t] = edge_ids(a, c)           # along A->C (j)
        gid[nu - t, t] = edge_ids(b, c)      # along B->C
        interior = (I > 0) & (J > 0) & (I + J < nu)
        gid[I[interior], J[interior]] = face_base + fi * n_face_int + np.arange(n_face_int)
        P = (v0[a][None, :] + (v0[b] - v0[a])[None, :] * (I[:, None] / nu)
             + (v0[c] - v0[a])[None, :] * (J[:, None] / nu))
        V[gid[I, J]] = P
        # triangles: up (i,j),(i+1,j),(i,j+1) and down (i+1,j),(i+1,j+1),(i,j+1)
        iu, ju = np.nonzero((ii + jj <= nu - 1))
        up = np.stack([gid[iu, ju], gid[iu + 1, ju], gid[iu, ju + 1]], axis=1)
        idn, jdn = np.nonzero((ii + jj <= nu - 2))
        dn = np.stack([gid[idn + 1, jdn], gid[idn + 1, jdn + 1], gid[idn, jdn + 1]], axis=1)
        tri = np.concatenate([up, dn], axis=0)
        F[fi * nu * nu:(fi + 1) * nu * nu] = tri
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    # orient outward (the icosahedron faces are outward, the sub-triangles
    # inherit it; keep an explicit check so a mistake fails loudly)
    e1 = V[F[:, 1]] - V[F[:, 0]]
    e2 = V[F[:, 2]] - V[F[:, 0]]
    s = np.einsum("ij,ij->i", np.cross(e1, e2), V[F[:, 0]])
    if not np.all(s > 0):
        raise AssertionError("geodesic_icosphere orientation")
    return V, F


def torus(nu: int, nv: int, R: float = 1.0, r: float = 0.3):
    """Regular ``nu`` x ``nv`` torus grid (nu around the big circle), each quad
    split into two triangles.  nu*nv vertices, 2*nu*nv faces."""
    u = 2 * np.pi * np.arange(nu) / nu
    w = 2 * np.pi * np.arange(nv) / nv
    U, W = np.meshgrid(u, w, indexing="ij")
    X = (R + r * np.cos(W)) * np.cos(U)
    Y = (R + r * np.cos(W)) * np.sin(U)
    Z = r * np.sin(W)
    V = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    i, j = i.ravel(), j.ravel()
    a = i * nv + j
    b = ((i + 1) % nu) * nv + j
    c = ((i + 1) % nu) * nv + (j + 1) % nv
    d = i * nv + (j + 1) % nv
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)]).astype(np.int32)
    return V, F


def rectangle_grid(nx: int, ny: int, h: float = 1.0):
    """Flat ``nx`` x ``ny`` vertex grid with spacing ``h`` in the z=0 plane;
    every square is split by the same diagonal (lower-left to upper-right)."""
    x = h * np.arange(nx)
    y = h * np.arange(ny)
    X, Y = np.meshgrid(x, y, indexing="ij")
    V = np.stack([X.ravel(), Y.ravel(), np.zeros(nx * ny)], axis=1)
    i, j = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="ij")
    i, j = i.ravel(), j.ravel()
    a = i * ny + j
    b = (i + 1) * ny + j
    c = (i + 1) * ny + j + 1
    d = i * ny + j + 1
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)]).astype(np.int32)
    return V, F


def mean_edge_length(V, F):
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.linalg.norm(V[e[:, 0]] - V[e[:, 1]], axis=1).mean())


def radial_jitter(V, sigma, rng):
    """Scale every vertex radially by (1 + N(0, sigma^2))."""
    return V * (1.0 + rng.normal(0.0, sigma, size=(len(V), 1)))


def _min_angle_deg(V, F):
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]

    def ang(p, q, r):
        u, w = q - p, r - p
        cosv = np.einsum("ij,ij->i", u, w) / (np.linalg.norm(u, axis=1) * np.linalg.norm(w, axis=1))
        return np.degrees(np.arccos(np.clip(cosv, -1.0, 1.0)))
    return np.minimum(np.minimum(ang(a, b, c), ang(b, c, a)), ang(c, a, b))


def isotropic_noise(V, F, sigma, rng, min_angle=1.0, max_rounds=50):
    """Add isotropic 3-D N(0, sigma^2) noise; vertices of triangles that end up
    with an angle below ``min_angle`` degrees (or flipped) are redrawn."""
    V0 = V.copy()
    W = V0 + rng.normal(0.0, sigma, size=V.shape)
    n0 = np.cross(V0[F[:, 1]] - V0[F[:, 0]], V0[F[:, 2]] - V0[F[:, 0]])
    for _ in range(max_rounds):
        n1 = np.cross(W[F[:, 1]] - W[F[:, 0]], W[F[:, 2]] - W[F[:, 0]])
        bad = (_min_angle_deg(W, F) < min_angle) | (np.einsum("ij,ij->i", n0, n1) <= 0)
        if not bad.any():
            return W
        vb = np.unique(F[bad].ravel())
        W[vb] = V0[vb] + rng.normal(0.0, sigma, size=(len(vb), 3))
    # give up on the remaining ones: put them back to the clean position
    n1 = np.cross(W[F[:, 1]] - W[F[:, 0]], W[F[:, 2]] - W[F[:, 0]])
    bad = (_min_angle_deg(W, F) < min_angle) | (np.einsum("ij,ij->i", n0, n1) <= 0)
    W[np.unique(F[bad].ravel())] = V0[np.unique(F[bad].ravel())]
    return W


def gaussian_bumps(V, rng, count=50, amplitude=0.05, width=(0.1, 0.3)):
    """Radial bumps on a unit sphere: r(x) = 1 + sum_k a exp(-|x-c_k|^2/(2 s_k^2)),
    c_k uniform on the sphere, s_k ~ U(width)."""
    c = rng.normal(size=(count, 3))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    s = rng.uniform(width[0], width[1], size=count)
    U = V / np.linalg.norm(V, axis=1, keepdims=True)
    r = np.ones(len(V))
    for k in range(count):
        d2 = np.sum((U - c[k]) ** 2, axis=1)
        r += amplitude * np.exp(-d2 / (2.0 * s[k] ** 2))
    return U * r[:, None]


def random_density(n, rng, lo=0.7, hi=1.3):
    return rng.uniform(lo, hi, size=n)


def gaussian_matrix(n, r, seed):
    """Seeded n x r matrix of independent N(0, 1) entries (row-major), used as
    the random test matrix of eigenvector sketches and as random directions."""
    return np.random.default_rng(seed).standard_normal((n, r))


def batch_mesh(i, seed=0, count=256, lo=2000, hi=50000):
    """Mesh i of a batch of ``count`` seeded meshes (noisy geodesic spheres for
    even i, noisy tori for odd i) whose vertex counts are log-uniform in
    [lo, hi].  Each mesh has its own generator (seed, i), so any subset of the
    batch can be made on its own."""
    if not 0 <= i < count:
        raise IndexError(i)
    rng = np.random.default_rng([seed, i])
    n = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
    if i % 2 == 0:
        nu = max(4, int(round(np.sqrt((n - 2) / 10))))
        V, F = geodesic_icosphere(nu)
        V = radial_jitter(V, 0.05 / nu, rng)
    else:
        a = max(8, int(round(np.sqrt(1.6 * n))))
        b = max(6, int(round(n / a)))
        V, F = torus(a, b)
        V = isotropic_noise(V, F, 0.2 * mean_edge_length(V, F), rng)
    return V, F


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------
CONFIGS = {
    # plain method, small: icosphere k=4, radial jitter N(0, 1e-3), p=20, 3 levels
    "sphere2k": dict(p=20, levels=3),
    # torus 400x250 (100k), noise 0.2*h, density U(0.7,1.3), p=100, 5 levels
    "torus100k": dict(p=100, levels=5),
    # geodesic icosphere nu=324 (1,049,762 V), 50 bumps + radial noise, p=100, 2 levels
    "sphere1m": dict(p=100, levels=2),
    # torus 500x400 (200k) perturbed, p=64, 2 levels (adjoint workload)
    "torus200k": dict(p=64, levels=2),
    # 50x40 copy of the adjoint torus (2k vertices)
    "torus2k": dict(p=64, levels=2),
}


def config_mesh(name: str, seed: int = 0, nu: int | None = None):
    """Return (V, F, density-or-None) for a named workload.

    ``nu`` overrides the geodesic frequency of ``sphere1m`` (for scaled-down
    runs of the same recipe)."""
    rng = np.random.default_rng(seed)
    if name == "sphere2k":
        V, F = icosphere(4)
        return radial_jitter(V, 1e-3, rng), F, None
    if name == "torus100k":
        V, F = torus(400, 250)
        h = mean_edge_length(V, F)
        V = isotropic_noise(V, F, 0.2 * h, rng)
        return V, F, random_density(len(V), rng)
    if name == "sphere1m":
        V, F = geodesic_icosphere(324 if nu is None else nu)
        V = gaussian_bumps(V, rng)
        h = mean_edge_length(V, F)
        V = radial_jitter(V, 0.015 * h, rng)
        return V, F, None
    if name == "torus200k":
        V, F = torus(500, 400)
        h = mean_edge_length(V, F)
        return isotropic_noise(V, F, 0.2 * h, rng), F, None
    if name == "torus2k":
        V, F = torus(50, 40)
        h = mean_edge_length(V, F)
        return isotropic_noise(V, F, 0.2 * h, rng), F, None
    raise KeyError(name)
