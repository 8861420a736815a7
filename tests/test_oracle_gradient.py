"""Pins of the dense reference gradient (oracle/gradient.py) against central
finite differences of library eigensolves and exact invariances."""
import numpy as np
import scipy.linalg as sl

import synth
from oracle import assembly, gradient


def _mesh(seed=0):
    rng = np.random.default_rng(seed)
    V, F = synth.torus(14, 9)
    V = synth.isotropic_noise(V, F, 0.15 * synth.mean_edge_length(V, F), rng)
    return V, F, synth.random_density(len(V), rng)


def _eig(V, F, d):
    S, m = assembly.assemble(V, F, density=d)
    return sl.eigh(S.toarray(), np.diag(m))


def _loss_parts(p, seed=1):
    rng = np.random.default_rng(seed)
    wl = rng.uniform(0.5, 2.0, p)
    T = rng.standard_normal((0, p))  # placeholder
    return wl


def test_eigenvalue_gradient_matches_fd():
    V, F, d = _mesh()
    p = 8
    wl = np.random.default_rng(1).uniform(0.5, 2.0, p)
    loss = lambda lam: np.sum(wl * lam[:p] ** 2)
    g, lam, X = gradient.reference_gradient(V, F, p, grad_lam=lambda l: 2 * wl * l, density=d)
    rng = np.random.default_rng(2)
    for _ in range(4):
        D = rng.standard_normal(V.shape)
        h = 1e-6
        fd = (loss(_eig(V + h * D, F, d)[0]) - loss(_eig(V - h * D, F, d)[0])) / (2 * h)
        assert abs(fd - np.sum(g * D)) <= 1e-6 * abs(fd)


def test_eigenvector_gradient_matches_fd():
    V, F, d = _mesh(3)
    p = 10
    lam0, X0 = _eig(V, F, d)
    cl = gradient.clusters_of(lam0, 1e-2)
    T = np.random.default_rng(4).standard_normal((len(V), p))

    def loss_of(X):
        # sum over clusters of ||X_C^T T_C||_F^2: invariant to signs and rotations in a cluster
        tot = 0.0
        for c in np.unique(cl[:p]):
            idx = np.nonzero(cl[:p] == c)[0]
            tot += np.sum((X[:, idx].T @ T[:, idx]) ** 2)
        return tot

    def grad_X(X):
        G = np.zeros_like(X)
        for c in np.unique(cl[:p]):
            idx = np.nonzero(cl[:p] == c)[0]
            A = X[:, idx].T @ T[:, idx]
            G[:, idx] = 2 * T[:, idx] @ A.T
        return G

    g, lam, X = gradient.reference_gradient(V, F, p, grad_X=grad_X, density=d)
    rng = np.random.default_rng(5)
    for _ in range(4):
        D = rng.standard_normal(V.shape)
        h = 1e-6
        fd = (loss_of(_eig(V + h * D, F, d)[1][:, :p]) - loss_of(_eig(V - h * D, F, d)[1][:, :p])) / (2 * h)
        assert abs(fd - np.sum(g * D)) <= 1e-5 * max(abs(fd), 1e-8)


def test_gradient_invariances():
    """Translation and rotation invariance; scaling: sum_v x_v . grad lambda_k = -2 lambda_k."""
    V, F, d = _mesh(6)
    p = 6
    for k in range(1, p):
        e = np.zeros(p)
        e[k] = 1.0
        g, lam, _ = gradient.reference_gradient(V, F, p, grad_lam=lambda l, e=e: e, density=d)
        assert np.abs(g.sum(axis=0)).max() < 1e-10 * np.abs(g).max()
        assert np.abs(np.cross(V, g).sum(axis=0)).max() < 1e-9 * np.abs(g).max()
        assert abs(np.sum(V * g) + 2 * lam[k]) < 1e-10 * lam[k]


def _open_mesh(seed=6):
    # open sheet with an out-of-plane bump: a surface with boundary that is not flat
    rng = np.random.default_rng(seed)
    V, F = synth.rectangle_grid(14, 10, 0.1)
    V = synth.isotropic_noise(V, F, 0.15 * synth.mean_edge_length(V, F), rng)
    V[:, 2] += 0.2 * np.exp(-((V[:, 0] - 0.6) ** 2 + (V[:, 1] - 0.45) ** 2) / 0.1)
    return V, F, synth.random_density(len(V), rng)


def _eig_dirichlet(V, F, d):
    S, m = assembly.assemble(V, F, density=d)
    Si, mi, interior = assembly.dirichlet(S, m, F)
    lam, Xi = sl.eigh(Si.toarray(), np.diag(mi))
    X = np.zeros((len(V), len(lam)))
    X[interior] = Xi
    return lam, X, interior


def test_dirichlet_gradient_matches_fd():
    # Dirichlet condition: eigenvalue and eigenvector losses against central
    # differences of the interior problem's eigenpairs
    V, F, d = _open_mesh()
    p = 8
    lam0, X0, interior = _eig_dirichlet(V, F, d)
    on = np.setdiff1d(np.arange(len(V)), interior)
    wl = np.random.default_rng(1).uniform(0.5, 2.0, p)
    cl = gradient.clusters_of(lam0, 1e-2)
    T = np.random.default_rng(7).standard_normal((len(V), p))

    def loss_of(lam, X):
        tot = np.sum(wl * lam[:p] ** 2)
        for c in np.unique(cl[:p]):
            idx = np.nonzero(cl[:p] == c)[0]
            tot += np.sum((X[:, idx].T @ T[:, idx]) ** 2)
        return tot

    def grad_X(X):
        G = np.zeros_like(X)
        for c in np.unique(cl[:p]):
            idx = np.nonzero(cl[:p] == c)[0]
            G[:, idx] = 2 * T[:, idx] @ (X[:, idx].T @ T[:, idx]).T
        return G

    g, lam, X = gradient.reference_gradient(V, F, p, grad_lam=lambda l: 2 * wl * l, grad_X=grad_X, density=d,
                                            boundary="dirichlet")
    assert np.array_equal(lam, lam0[:p]) and (X[on] == 0).all()
    rng = np.random.default_rng(8)
    for _ in range(4):
        D = rng.standard_normal(V.shape)
        h = 1e-6
        lp, Xp, _ = _eig_dirichlet(V + h * D, F, d)
        lm, Xm, _ = _eig_dirichlet(V - h * D, F, d)
        fd = (loss_of(lp, Xp[:, :p]) - loss_of(lm, Xm[:, :p])) / (2 * h)
        assert abs(fd - np.sum(g * D)) <= 1e-5 * abs(fd), (fd, np.sum(g * D))
    # the boundary vertices still move the interior problem (their cotangent
    # weights and masses): the gradient does not vanish there
    assert np.abs(g[on]).max() > 1e-3 * np.abs(g).max()


def test_dirichlet_gradient_differs_from_neumann():
    # the two conditions give different problems, so a reference that ignored
    # the condition would fail here
    V, F, d = _open_mesh()
    p = 6
    gl = lambda l: np.ones(p)
    gd, ld, _ = gradient.reference_gradient(V, F, p, grad_lam=gl, density=d, boundary="dirichlet")
    gn, ln, _ = gradient.reference_gradient(V, F, p, grad_lam=gl, density=d)
    assert ld[0] > 1.0 and abs(ln[0]) < 1e-8
    assert np.linalg.norm(gd - gn) > 0.1 * np.linalg.norm(gd)


def test_circumcentric_mass_torch_matches_assembly():
    # the differentiable masses equal the assembly's circumcentric masses
    import torch
    V, F, d = _mesh(9)
    m = assembly.lumped_mass(V, F, lumping="voronoi", density=d)
    mt = gradient.lumped_mass_torch(torch.tensor(V), torch.tensor(F.astype(np.int64)), d, "voronoi").numpy()
    assert np.abs(mt - m).max() <= 1e-14 * np.abs(m).max()
    assert np.abs(m - assembly.lumped_mass(V, F, density=d)).max() > 1e-3 * m.max()


def test_circumcentric_gradient_matches_fd():
    # circumcentric lumping: eigenvalue and eigenvector losses against central
    # differences of the dense eigenpairs of that lumping
    V, F, d = _mesh(10)
    p = 8

    def eig(Vx):
        S, m = assembly.assemble(Vx, F, lumping="voronoi", density=d)
        assert m.min() > 0
        return sl.eigh(S.toarray(), np.diag(m))

    lam0, X0 = eig(V)
    cl = gradient.clusters_of(lam0, 1e-2)
    wl = np.random.default_rng(1).uniform(0.5, 2.0, p)
    T = np.random.default_rng(11).standard_normal((len(V), p))

    def loss_of(lam, X):
        tot = np.sum(wl * lam[:p] ** 2)
        for c in np.unique(cl[:p]):
            idx = np.nonzero(cl[:p] == c)[0]
            tot += np.sum((X[:, idx].T @ T[:, idx]) ** 2)
        return tot

    def grad_X(X):
        G = np.zeros_like(X)
        for c in np.unique(cl[:p]):
            idx = np.nonzero(cl[:p] == c)[0]
            G[:, idx] = 2 * T[:, idx] @ (X[:, idx].T @ T[:, idx]).T
        return G

    g, lam, X = gradient.reference_gradient(V, F, p, grad_lam=lambda l: 2 * wl * l, grad_X=grad_X, density=d,
                                            lumping="voronoi")
    gb, _, _ = gradient.reference_gradient(V, F, p, grad_lam=lambda l: 2 * wl * l, grad_X=grad_X, density=d)
    assert np.linalg.norm(g - gb) > 1e-3 * np.linalg.norm(g)
    rng = np.random.default_rng(12)
    for _ in range(4):
        D = rng.standard_normal(V.shape)
        h = 1e-6
        lp, Xp = eig(V + h * D)
        lm, Xm = eig(V - h * D)
        fd = (loss_of(lp, Xp[:, :p]) - loss_of(lm, Xm[:, :p])) / (2 * h)
        assert abs(fd - np.sum(g * D)) <= 1e-5 * abs(fd), (fd, np.sum(g * D))
