"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test targets a plausible mistake: a sign or index error in the cotangent
formula, a wrong lumping, a wrong rotation angle in Jacobi, a dropped
normalisation in the prolongation, a wrong Galerkin product, a wrong
subspace-size or level rule.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import synth
from oracle import assembly, hierarchy, hsim, jacobi, metrics, sim


# ---------------------------------------------------------------- assembly
def test_stiffness_kernel_symmetry_psd():
    V, F, _ = synth.config_mesh("sphere2k", seed=1)
    S, m = assembly.assemble(V, F)
    assert abs(S - S.T).max() == 0.0
    assert np.abs(S @ np.ones(len(V))).max() < 1e-13 * abs(S).max()
    ev = sl.eigh(S.toarray(), eigvals_only=True, subset_by_index=[0, 2])
    assert ev[0] > -1e-12 and ev[1] > 1e-6          # PSD, one-dimensional kernel


def test_lumping_is_row_sum_of_consistent_mass_and_area():
    V, F = synth.torus(20, 12)
    m = assembly.lumped_mass(V, F)
    Mc = assembly.consistent_mass(V, F)
    assert np.allclose(np.asarray(Mc.sum(axis=1)).ravel(), m, rtol=1e-14, atol=0)
    assert math.isclose(m.sum(), assembly.surface_area(V, F), rel_tol=1e-13)
    # consistent mass integrates 1*1 to the area
    assert math.isclose(np.ones(len(V)) @ Mc @ np.ones(len(V)), m.sum(), rel_tol=1e-13)


def test_torus_area_closed_form():
    # smooth torus area 4 pi^2 R r; the fine polyhedral torus converges O(h^2)
    V, F = synth.torus(400, 120)
    A = assembly.surface_area(V, F)
    assert abs(A / (4 * np.pi ** 2 * 0.3) - 1) < 1e-3


def test_rigid_motion_and_scaling():
    rng = np.random.default_rng(3)
    V, F = synth.icosphere(2)
    V = synth.radial_jitter(V, 1e-2, rng)
    S, m = assembly.assemble(V, F)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    S2, m2 = assembly.assemble(V @ Q.T + np.array([1.0, -2.0, 0.5]), F)
    assert abs(S - S2).max() < 1e-12 * abs(S).max()
    assert np.abs(m - m2).max() < 1e-13 * m.max()
    # lambda(c V) = lambda(V) / c^2 : S is scale-invariant, M scales by c^2
    S3, m3 = assembly.assemble(2.5 * V, F)
    assert abs(S - S3).max() < 1e-12 * abs(S).max()
    assert np.allclose(m3, 6.25 * m, rtol=1e-13)


def test_cotan_of_equilateral_and_right_triangle():
    # single right isoceles triangle: the two acute angles have cot 1, the
    # right angle cot 0 -> S = 1/2 [[1,-1/2... ]] explicit
    V = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0]])
    F = np.array([[0, 1, 2]])
    S = assembly.stiffness(V, F).toarray()
    expect = 0.5 * np.array([[2.0, -1, -1], [-1, 1, 0], [-1, 0, 1]])
    assert np.allclose(S, expect, atol=1e-15)
    Ve = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.5, math.sqrt(3) / 2, 0]])
    Se = assembly.stiffness(Ve, F).toarray()
    c = 0.5 / math.sqrt(3)      # cot(60 deg)/2
    assert np.allclose(Se, np.array([[2 * c, -c, -c], [-c, 2 * c, -c], [-c, -c, 2 * c]]), atol=1e-15)


# ------------------------------------------------------------------ Jacobi
@pytest.mark.parametrize("n", [1, 2, 3, 8, 31])
def test_jacobi_matches_lapack(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    A = A + A.T
    lam, V, _ = jacobi.jacobi_eigh(A)
    ref = np.linalg.eigvalsh(A)       # library special case
    assert np.allclose(lam, ref, atol=1e-13 * max(1, np.abs(ref).max()))
    assert np.allclose(V.T @ V, np.eye(n), atol=1e-13)
    assert np.allclose(A @ V, V * lam[None, :], atol=1e-12 * max(1, np.abs(ref).max()))


def test_jacobi_2x2_closed_form():
    a, b, c = 2.0, 0.7, -1.3
    lam, V, _ = jacobi.jacobi_eigh(np.array([[a, b], [b, c]]))
    d = math.sqrt(((a - c) / 2) ** 2 + b * b)
    assert np.allclose(lam, [(a + c) / 2 - d, (a + c) / 2 + d], atol=1e-15)


def test_jacobi_gep_and_cholesky():
    rng = np.random.default_rng(7)
    n = 24
    B = rng.standard_normal((n, n))
    M = B @ B.T + n * np.eye(n)
    S = rng.standard_normal((n, n))
    S = S + S.T
    R = jacobi.cholesky_upper(M)
    assert np.allclose(R.T @ R, M, atol=1e-12)
    assert np.allclose(R, np.triu(R))
    lam, X = jacobi.jacobi_gep(S, M)
    ref = sl.eigh(S, M, eigvals_only=True)
    assert np.allclose(lam, ref, atol=1e-12)
    assert np.allclose(X.T @ M @ X, np.eye(n), atol=1e-12)
    assert np.allclose(S @ X, M @ X * lam[None, :], atol=1e-11)


def test_brute_force_small_meshes():
    """P4: every eigenpair of meshes under 500 vertices, own Jacobi vs LAPACK."""
    meshes = [synth.icosphere(2), synth.torus(20, 12), synth.rectangle_grid(16, 20, 0.1)]
    for V, F in meshes:
        S, m = assembly.assemble(V, F)
        lam, X = jacobi.jacobi_gep_diag(S, m)
        ref = sl.eigh(S.toarray(), np.diag(m), eigvals_only=True)
        assert np.abs(lam - ref).max() < 1e-12 * ref.max()
        assert metrics.m_orthonormality(X, m) < 1e-12


# ------------------------------------------------------- analytic spectra
def test_constant_mode_P1():
    V, F, _ = synth.config_mesh("sphere2k", seed=0)
    S, m = assembly.assemble(V, F)
    lam, X, it, r = sim.sim_lowest(S, m, 6, eps=1e-11)
    assert abs(lam[0]) <= 1e-12 * lam[1]
    x0 = X[:, 0] * np.sign(X[0, 0])
    assert np.abs(x0 - 1 / math.sqrt(m.sum())).max() < 1e-9


def test_sphere_spectrum_P2():
    V, F, _ = synth.config_mesh("sphere2k", seed=0)
    S, m = assembly.assemble(V, F)
    lam, X, it, r = sim.sim_lowest(S, m, 25, eps=1e-10)
    sizes = [b - a for a, b in metrics.clusters(lam[1:], gap=2e-2)]
    assert sizes[:3] == [3, 5, 7] and sum(sizes) == 24
    ell = np.repeat(np.arange(5), [1, 3, 5, 7, 9])[1:25]
    rel = np.abs(lam[1:] - ell * (ell + 1)) / (ell * (ell + 1))
    assert rel.max() < 2.5e-2
    # O(h^2): the l = 2..4 error shrinks by about 4 per subdivision
    ell = np.repeat(np.arange(5), [1, 3, 5, 7, 9])
    errs = []
    for k in (3, 4):
        Vk, Fk = synth.icosphere(k)
        Sk, mk = assembly.assemble(Vk, Fk)
        lk, *_ = sim.sim_lowest(Sk, mk, 25, eps=1e-10)
        errs.append((np.abs(lk[4:] - ell[4:] * (ell[4:] + 1)) / (ell[4:] * (ell[4:] + 1))).max())
    assert 3.5 < errs[0] / errs[1] < 4.5


@pytest.mark.parametrize("nx,ny", [(9, 6), (13, 10)])
def test_neumann_rectangle_P3(nx, ny):
    h = 0.37
    V, F = synth.rectangle_grid(nx, ny, h)
    S, m = assembly.assemble(V, F, lumping="voronoi")
    k, l = np.arange(nx), np.arange(ny)
    exact = np.sort(((4 / h ** 2) * (np.sin(k[:, None] * np.pi / (2 * (nx - 1))) ** 2
                                     + np.sin(l[None, :] * np.pi / (2 * (ny - 1))) ** 2)).ravel())
    lam, X = jacobi.jacobi_gep_diag(S, m)
    assert np.abs(lam - exact).max() < 1e-12 * exact.max()
    lam2, *_ = sim.sim_lowest(S, m, 10, eps=1e-11)
    assert np.abs(lam2 - exact[:10]).max() < 1e-9 * exact[9]
    # barycentric lumping breaks the closed form (the pin notices a lumping mix-up)
    Sb, mb = assembly.assemble(V, F, lumping="barycentric")
    lb, _ = jacobi.jacobi_gep_diag(Sb, mb)
    assert np.abs(lb - exact).max() > 1e-3 * exact.max()


@pytest.mark.parametrize("nx,ny", [(9, 6), (13, 10)])
def test_dirichlet_rectangle(nx, ny):
    # Dirichlet on the flat grid: the interior block of the cotangent matrix is
    # the 5-point Laplacian and the circumcentric masses are h^2, so the
    # spectrum is (4/h^2)(sin^2(k pi / 2(nx-1)) + sin^2(l pi / 2(ny-1))),
    # k = 1..nx-2, l = 1..ny-2, with eigenvectors sin(k pi i/(nx-1)) sin(l pi j/(ny-1))
    h = 0.37
    V, F = synth.rectangle_grid(nx, ny, h)
    S, m = assembly.assemble(V, F, lumping="voronoi")
    on = assembly.boundary_vertices(F, len(V))
    assert on.sum() == 2 * (nx + ny) - 4
    Si, mi, interior = assembly.dirichlet(S, m, F)
    assert len(interior) == (nx - 2) * (ny - 2) and not on[interior].any()
    k, l = np.arange(1, nx - 1), np.arange(1, ny - 1)
    exact = np.sort(((4 / h ** 2) * (np.sin(k[:, None] * np.pi / (2 * (nx - 1))) ** 2
                                     + np.sin(l[None, :] * np.pi / (2 * (ny - 1))) ** 2)).ravel())
    lam, X = jacobi.jacobi_gep_diag(Si, mi)
    assert np.abs(lam - exact).max() < 1e-12 * exact.max()
    # the lowest mode is the product of the two lowest sines on the interior
    xy = V[interior, :2] / h
    mode = np.sin(np.pi * np.round(xy[:, 0]) / (nx - 1)) * np.sin(np.pi * np.round(xy[:, 1]) / (ny - 1))
    c = abs(mode @ (mi * X[:, 0])) / np.sqrt(mode @ (mi * mode))
    assert abs(c - 1.0) < 1e-12
    # a closed surface has no boundary
    Vs, Fs = synth.icosphere(2)
    assert not assembly.boundary_vertices(Fs, len(Vs)).any()


# ---------------------------------------------------------- SIM / residual
def test_sim_matches_dense_and_residual_forms():
    V, F = synth.torus(24, 14)
    rng = np.random.default_rng(0)
    V = synth.isotropic_noise(V, F, 0.02, rng)
    S, m = assembly.assemble(V, F, density=synth.random_density(len(V), rng))
    ref, Y = sl.eigh(S.toarray(), np.diag(m))
    lam, X, it, r = sim.sim_lowest(S, m, 12, eps=1e-11)
    assert np.abs(lam - ref[:12])[1:].max() < 1e-10 * ref[11]
    assert metrics.eigenvector_err(X, Y[:, :20], m, ref[:20]).max() < 1e-8
    # paper form and floored form agree away from lambda = 0
    r1 = sim.residual_conv2(S, m, X, lam)
    r2 = sim.residual(S, m, X, lam)
    assert np.allclose(r1[1:], r2[1:], rtol=1e-6, atol=1e-14)
    # a perturbed vector has a large residual
    Xp = X + 1e-3 * rng.standard_normal(X.shape)
    assert sim.residual(S, m, Xp, lam)[1:].min() > 1e-6


def test_subspace_and_level_rules():
    assert [sim.subspace_size(p) for p in (20, 50, 64, 100, 200)] == [30, 75, 96, 150, 300]
    assert [hierarchy.shift_index(p) for p in (20, 50, 64, 100, 200)] == [2, 5, 6, 10, 20]
    assert hierarchy.coarsest_size(100) == 1000 and hierarchy.coarsest_size(1000) == 1500
    assert hierarchy.num_levels(200) == 2 and hierarchy.num_levels(201) == 3
    assert hierarchy.level_sizes(2562, 3, 1000) == [2562, 1601, 1000]
    assert hierarchy.level_sizes(100000, 5, 1000) == [100000, 31623, 10000, 3162, 1000]
    assert hierarchy.level_sizes(1049762, 2, 1000) == [1049762, 1000]


# --------------------------------------------------------------- hierarchy
@pytest.fixture(scope="module")
def small_hierarchy():
    rng = np.random.default_rng(5)
    V, F = synth.icosphere(3)
    V = synth.radial_jitter(V, 1e-2, rng)
    S, m = assembly.assemble(V, F)
    lv = hierarchy.build_hierarchy(V, F, S, m, p=10, levels=3, n_coarsest=120, seed=17)
    return V, F, S, m, lv


def test_fps_is_farthest_point_sampling(small_hierarchy):
    """Every inserted vertex is the farthest (graph distance, by the library
    Dijkstra) from the vertices inserted before it; ties to the lowest index."""
    V, F, S, m, lv = small_hierarchy
    ip, nb, w = hierarchy.edge_graph(V, F)
    G = sp.csr_matrix((w, nb, ip), shape=(len(V), len(V)))
    order = lv[1]["verts"]
    assert order[0] == 17 % len(V)
    D = csg.dijkstra(G, indices=order)
    for k in range(1, len(order)):
        d = D[:k].min(axis=0)
        assert order[k] == int(np.argmax(d))
    # nested prefixes
    assert np.array_equal(lv[2]["verts"], order[: len(lv[2]["verts"])])


def test_prolongation_definition(small_hierarchy):
    """U^tau against eq. (basis) evaluated with library graph distances."""
    V, F, S, m, lv = small_hierarchy
    ip, nb, w = hierarchy.edge_graph(V, F)
    G = sp.csr_matrix((w, nb, ip), shape=(len(V), len(V)))
    A = assembly.surface_area(V, F)
    for tau in range(2):
        fine, coarse = lv[tau]["verts"], lv[tau + 1]["verts"]
        rho = math.sqrt(7.0 * A / (len(coarse) * math.pi))
        assert math.isclose(lv[tau]["rho"], rho, rel_tol=1e-15)
        D = csg.dijkstra(G, indices=coarse)[:, fine].T          # fine x coarse
        Ut = np.where(D < rho, 1.0 - D / rho, 0.0)
        rs = Ut.sum(axis=1)
        assert (rs > 0).all()
        U = lv[tau]["U"].toarray()
        assert np.abs(U - Ut / rs[:, None]).max() < 1e-14
        assert (U >= 0).all() and np.abs(U.sum(axis=1) - 1).max() < 1e-14


def test_galerkin_operators(small_hierarchy):
    V, F, S, m, lv = small_hierarchy
    area = m.sum()
    for tau in (1, 2):
        St, Mt = lv[tau]["S"], lv[tau]["M"]
        one = np.ones(St.shape[0])
        assert np.abs(St @ one).max() < 1e-13 * abs(St).max()
        assert math.isclose(one @ Mt @ one, area, rel_tol=1e-13)
        assert abs(St - St.T).max() < 1e-15 * abs(St).max()
        # Galerkin: the level-tau Rayleigh quotient of x equals the fine one of
        # the prolonged vector
        x = np.random.default_rng(tau).standard_normal(St.shape[0])
        y = x
        for k in range(tau - 1, -1, -1):
            y = lv[k]["U"] @ y
        assert math.isclose(x @ St @ x, y @ S @ y, rel_tol=1e-11)
        assert math.isclose(x @ Mt @ x, y @ (m * y), rel_tol=1e-11)


def test_prolongation_preserves_ritz_pairs(small_hierarchy):
    """(U Phi)^T M^tau (U Phi) = Phi^T M^{tau+1} Phi = I and likewise for S."""
    V, F, S, m, lv = small_hierarchy
    S2 = lv[2]["S"].toarray()
    M2 = lv[2]["M"].toarray()
    lam, X = jacobi.jacobi_gep(S2, M2)
    Phi = lv[1]["U"] @ X[:, :20]
    M1 = lv[1]["M"]
    assert np.allclose(Phi.T @ (M1 @ Phi), np.eye(20), atol=1e-11)
    assert np.allclose(Phi.T @ (lv[1]["S"] @ Phi), np.diag(lam[:20]), atol=1e-10 * lam[19])
    # Ritz values on nested spaces bound the fine eigenvalues from above
    ref = sl.eigh(S.toarray(), np.diag(m), eigvals_only=True)
    assert (lam[1:20] >= ref[1:20] * (1 - 1e-12)).all()


def test_hsim_oracle_reaches_dense_solution():
    V, F, _ = synth.config_mesh("sphere2k", seed=0)
    S, m = assembly.assemble(V, F)
    ref, Y = sl.eigh(S.toarray(), np.diag(m))
    lam, X, info = hsim.hsim(V, F, S, m, p=20, eps=1e-8, levels=3, n_coarsest=150)
    assert info["iters"][0] == "F" and len(info["iters"]) == 3
    assert np.abs(lam - ref[:20])[1:].max() < 1e-9 * ref[19]
    assert info["resid"].max() < 1e-8
    assert metrics.eigenvector_err(X, Y[:, :40], m, ref[:40]).max() < 1e-5
    assert metrics.m_orthonormality(X, m) < 1e-10


# ------------------------------------------------------------ error metrics
@pytest.fixture(scope="module")
def sphere162_pairs():
    """All eigenpairs of the 162-vertex icosphere (LAPACK): exact clusters of
    the sphere spectrum, 1, 3, 5, 7, ... (slightly split by the mesh)."""
    V, F = synth.icosphere(2)
    S, m = assembly.assemble(V, F)
    lam, Y = sl.eigh(S.toarray(), np.diag(m))
    return S, m, lam, Y


def test_eigenvector_err_wrong_cluster_is_one(sphere162_pairs):
    """A vector from another cluster is M-orthogonal to the reference cluster:
    error exactly 1 (a projection onto the whole reference block instead of
    the cluster would give 0)."""
    S, m, lam, Y = sphere162_pairs
    cl = metrics.clusters(lam[:16])
    assert [b - a for a, b in cl][:3] == [1, 3, 5]
    X = Y[:, :9].copy()
    X[:, 1], X[:, 5] = Y[:, 5], Y[:, 1]          # swap a l=1 vector with a l=2 vector
    err = metrics.eigenvector_err(X, Y[:, :16], m, lam[:16])
    assert abs(err[1] - 1.0) < 1e-12 and abs(err[5] - 1.0) < 1e-12
    others = np.delete(err, [1, 5])
    assert others.max() < 1e-12


def test_eigenvector_err_value_of_a_mixed_vector(sphere162_pairs):
    """x = cos t y_i + sin t y_j with y_j outside the cluster of y_i has error |sin t|."""
    S, m, lam, Y = sphere162_pairs
    X = Y[:, :9].copy()
    for t in (1e-6, 1e-3, 0.3):
        X[:, 2] = np.cos(t) * Y[:, 2] + np.sin(t) * Y[:, 12]
        err = metrics.eigenvector_err(X, Y[:, :16], m, lam[:16])
        assert abs(err[2] - np.sin(t)) <= 1e-9 * max(np.sin(t), 1e-3), t
        # a rotation inside the cluster costs nothing
    X[:, 1:4] = Y[:, 1:4] @ sl.qr(np.random.default_rng(1).standard_normal((3, 3)))[0]
    assert metrics.eigenvector_err(X[:, :4], Y[:, :16], m, lam[:16]).max() < 1e-12


def test_m_orthonormality_flags_a_bad_block(sphere162_pairs):
    S, m, lam, Y = sphere162_pairs
    X = Y[:, :10].copy()
    assert metrics.m_orthonormality(X, m) < 1e-12
    X[:, 3] *= 1.1                                   # ||x_3||_M^2 = 1.21
    assert abs(metrics.m_orthonormality(X, m) - 0.21) < 1e-12
    X = Y[:, :10].copy()
    X[:, 4] += 0.05 * Y[:, 7]                        # x_7^T M x_4 = 0.05
    assert abs(metrics.m_orthonormality(X, m) - 0.05) < 1e-12
    # Euclidean-orthonormal but not M-orthonormal
    Q = sl.qr(Y[:, :10], mode="economic")[0]
    assert metrics.m_orthonormality(Q, m) > 0.1


def test_sketch_estimates_cluster_error(sphere162_pairs):
    """The sketch estimate of the cluster-aware error agrees with the exact
    error (chi-square spread with r - |C| degrees of freedom), is about 1 for
    a vector of another cluster and exactly 0 for an in-cluster rotation."""
    S, m, lam, Y = sphere162_pairs
    r = 400
    G = synth.gaussian_matrix(len(m), r, seed=5)
    cl = metrics.clusters(lam[:16])
    a, b = cl[2]                                       # the l = 2 cluster
    Zc = metrics.sketch(Y[:, a:b], m, G)
    for t in (1e-7, 1e-4, 0.2, np.pi / 2):
        x = np.cos(t) * Y[:, a + 1] + np.sin(t) * Y[:, 20]
        est = metrics.sketch_vector_err(metrics.sketch(x, m, G)[:, 0], Zc)
        exact = metrics.eigenvector_err(np.column_stack([Y[:, :a + 1], x]), Y[:, :16], m, lam[:16])[a + 1]
        assert abs(est / exact - 1.0) < 0.25, (t, est, exact)
    # a rotation inside the cluster: out-of-span part 0 up to rounding
    Q = sl.qr(np.random.default_rng(2).standard_normal((b - a, b - a)))[0]
    W = metrics.sketch(Y[:, a:b] @ Q, m, G)
    assert max(metrics.sketch_vector_err(W[:, i], Zc) for i in range(b - a)) < 1e-12
    assert metrics.sketch_projector_diff(W, Zc) < 1e-12
    # the projector sketch sees a vector swapped in from another cluster
    X = Y[:, a:b].copy()
    X[:, 0] = Y[:, 20]
    assert metrics.sketch_projector_diff(metrics.sketch(X, m, G), Zc) > 0.1
