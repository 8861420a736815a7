"""Parity of every step of the GPU hot path with the FP64 oracle.

Each test calls the HIP library through the C ABI (the Python binding only
marshals arguments) and compares, element by element, with the oracle on the
same seeded inputs."""
import math

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import assembly, hierarchy, jacobi, metrics, sim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small(cuda):
    import paper_2111_09039_amd as hs
    rng = np.random.default_rng(5)
    V, F = synth.icosphere(3)
    V = synth.radial_jitter(V, 1e-2, rng)
    S, m = assembly.assemble(V, F)
    lv = hierarchy.build_hierarchy(V, F, S, m, p=24, levels=3, n_coarsest=120, seed=17)
    H = hs.Hierarchy(V, F, 24, levels=3, n_coarsest=120, seed=17)
    print(f"[small hierarchy] sizes {[len(l['verts']) for l in lv]}", flush=True)
    return V, F, S, m, lv, H


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _mass(lv, tau):
    M = lv[tau]["M"]
    return sp.diags(M).tocsr() if tau == 0 else M


def test_prolongation(small):
    V, F, S, m, lv, H = small
    rng = np.random.default_rng(0)
    for tau in range(2):
        nc = len(lv[tau + 1]["verts"])
        for k in (1, 7, 15):
            Xc = rng.standard_normal((nc, k))
            Y = H.prolong(tau, _t(Xc)).cpu().numpy()
            ref = lv[tau]["U"] @ Xc
            assert np.abs(Y - ref).max() <= 1e-14 * np.abs(ref).max(), (tau, k)


def test_prolongation_ignores_stale_workspace_rows(small):
    # the coarse block occupies only the first n_coarse rows of the shared
    # workspace; rows past it hold whatever an earlier call left there
    # (here +inf from a level-0 product), and the prolongation must not touch
    # them (a zero weight times inf would be NaN)
    V, F, S, m, lv, H = small
    rng = np.random.default_rng(3)
    for tau in range(2):
        n, nc = len(lv[tau]["verts"]), len(lv[tau + 1]["verts"])
        k = 13
        H.apply(0, 1, _t(np.full((len(lv[0]["verts"]), k), np.inf)))
        Xc = rng.standard_normal((nc, k))
        Y = H.prolong(tau, _t(Xc)).cpu().numpy()
        assert np.isfinite(Y).all(), tau
        ref = lv[tau]["U"] @ Xc
        assert np.abs(Y - ref).max() <= 1e-14 * np.abs(ref).max(), tau


def test_operator_products(small):
    V, F, S, m, lv, H = small
    rng = np.random.default_rng(1)
    for tau in range(3):
        n = len(lv[tau]["verts"])
        X = rng.standard_normal((n, 15))
        for op, A in ((0, lv[tau]["S"]), (1, _mass(lv, tau))):
            Y = H.apply(tau, op, _t(X)).cpu().numpy()
            ref = A @ X
            assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max(), (tau, op)


@pytest.mark.parametrize("tau", [0, 1])
def test_factor_inertia_and_solve(small, tau):
    V, F, S, m, lv, H = small
    St, Mt = lv[tau]["S"], _mass(lv, tau)
    ref = np.linalg.eigvalsh(np.linalg.solve(np.linalg.cholesky(Mt.toarray()),
                                             np.linalg.solve(np.linalg.cholesky(Mt.toarray()), St.toarray()).T))
    rng = np.random.default_rng(2)
    n = St.shape[0]
    for j in (-1, 4, 9):
        mu = -0.1 * ref[1] if j < 0 else 0.5 * (ref[j] + ref[j + 1])
        neg = H.factor(tau, mu)
        assert neg == int(np.sum(ref < mu)), (tau, mu, neg)
        B = rng.standard_normal((n, 13))
        X = H.solve_shifted(tau, _t(B)).cpu().numpy()
        A = (St - mu * Mt).tocsc()
        Xr = spla.splu(A).solve(B)
        assert np.abs(X - Xr).max() <= 1e-10 * np.abs(Xr).max(), (tau, mu)
        # normwise backward error per column (infinity norms)
        Ainf = np.abs(A).sum(axis=1).max()
        bw = (np.abs(A @ X - B).max(axis=0) / (Ainf * np.abs(X).max(axis=0) + np.abs(B).max(axis=0))).max()
        # bound c n u of a backward-stable solve (n = 642: n u = 1.4e-13; a
        # constant c of order one, the measured values are printed)
        print(f"[factor/solve tau={tau} mu={mu:.3g}] normwise backward error {bw:.2e}", flush=True)
        assert bw < 1e-13, bw


def test_gram(small):
    V, F, S, m, lv, H = small
    rng = np.random.default_rng(3)
    for tau in range(3):
        n = len(lv[tau]["verts"])
        for k in (5, 30, 36):
            Psi = rng.standard_normal((n, k))
            Sb, Mb = H.gram(tau, _t(Psi))
            Sr = Psi.T @ (lv[tau]["S"] @ Psi)
            Mr = Psi.T @ (_mass(lv, tau) @ Psi)
            assert np.abs(Sb.cpu().numpy() - Sr).max() <= 1e-13 * np.abs(Sr).max()
            assert np.abs(Mb.cpu().numpy() - Mr).max() <= 1e-13 * np.abs(Mr).max()


def _check_reduced_eigenproblem(k):
    import paper_2111_09039_amd as hs
    rng = np.random.default_rng(k)
    B = rng.standard_normal((k, k))
    Mb = B @ B.T / k + np.diag(rng.uniform(0.5, 2.0, k))
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    Sb = Q @ np.diag(np.sort(rng.uniform(0, 100, k))) @ Q.T
    lam, Pb, sweeps = hs.rayleigh_ritz_dense(_t(Sb), _t(Mb))
    lam, Pb = lam.cpu().numpy(), Pb.cpu().numpy()
    lr, Xr = jacobi.jacobi_gep(Sb, Mb)
    assert np.abs(lam - lr).max() <= 1e-12 * np.abs(lr).max()
    assert np.abs(Pb.T @ Mb @ Pb - np.eye(k)).max() < 1e-12
    assert np.abs(Sb @ Pb - Mb @ Pb * lam[None, :]).max() < 1e-11 * np.abs(lr).max()
    # distinct eigenvalues: vectors equal up to sign
    s = np.sign(np.sum(Pb * Xr, axis=0))
    assert np.abs(Pb - Xr * s[None, :]).max() < 1e-9


@pytest.mark.parametrize("k", [2, 17, 30, 64])
def test_reduced_eigenproblem(cuda, k):
    _check_reduced_eigenproblem(k)


@pytest.mark.parametrize("k", [96, 130, 200])
def test_reduced_eigenproblem_wide(cuda, k):
    """Several 32-row tiles of the dense factor and its inverse panel, the last
    one ragged (130, 200), and several 16-column groups of the products."""
    _check_reduced_eigenproblem(k)


def test_coarsest_dense_solve(small):
    V, F, S, m, lv, H = small
    k = H.q
    lam, X, sweeps = H.coarse(k)
    lam, X = lam.cpu().numpy(), X.cpu().numpy()
    lr, Xr = jacobi.jacobi_gep(lv[2]["S"].toarray(), lv[2]["M"].toarray())
    assert np.abs(lam - lr[:k]).max() <= 1e-12 * lr[k - 1]
    Mc = lv[2]["M"].toarray()
    assert np.abs(X.T @ Mc @ X - np.eye(k)).max() < 1e-11
    err = metrics.eigenvector_err(X, Xr, Mc, lr)
    assert err[1:].max() < 1e-8


@pytest.mark.parametrize("p", [20, 100])
def test_coarsest_spectral_projection(cuda, monkeypatch, capfd, p):
    """The library's default coarsest level (1000 unknowns) wants q of its
    eigenpairs: the spectral projection (Newton-Schulz sign of sigma I - C,
    Rayleigh-Ritz on the projector's range) against LAPACK's dense generalized
    eigensolver, and the Jacobi sweeps over the whole level against both."""
    import paper_2111_09039_amd as hs
    V, F, d = synth.config_mesh("sphere2k", seed=0)
    H = hs.Hierarchy(V, F, p, levels=3)
    e = H.export(H.levels - 1)
    n = len(e["verts"])
    assert n == 1000
    Sc = sp.csr_matrix((e["S_data"], e["S_indices"], e["S_indptr"]), shape=(n, n)).toarray()
    Mc = sp.csr_matrix((e["M_data"], e["S_indices"], e["S_indptr"]), shape=(n, n)).toarray()
    lr, Xr = sl.eigh(Sc, Mc)
    k = H.q
    results = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("HSIM_COARSE_JACOBI", mode)
        monkeypatch.setenv("HSIM_VERBOSE", "1")
        lam, X, sweeps = H.coarse(k)
        lam, X = lam.cpu().numpy(), X.cpu().numpy()
        out = capfd.readouterr().err
        assert ("spectral projection" in out) == (mode == "0"), out
        print(f"[coarsest p={p} q={k} jacobi={mode}] {out.strip()}", flush=True)
        assert np.abs(lam - lr[:k]).max() <= 1e-12 * lr[k - 1]
        assert np.abs(X.T @ Mc @ X - np.eye(k)).max() < 1e-11
        err = metrics.eigenvector_err(X, Xr, Mc, lr)
        assert err[1:].max() < 1e-8, err.max()
        results[mode] = lam
    assert np.abs(results["0"] - results["1"]).max() <= 2e-12 * lr[k - 1]


def test_ritz_update_and_residual(small):
    V, F, S, m, lv, H = small
    rng = np.random.default_rng(4)
    for tau in range(3):
        n = len(lv[tau]["verts"])
        k = 15
        Psi = rng.standard_normal((n, k))
        Pb = rng.standard_normal((k, k))
        lam = np.sort(rng.uniform(0.5, 20, k))
        Phi, r = H.ritz(tau, _t(Psi), _t(Pb), _t(lam), 0.5)
        Phi, r = Phi.cpu().numpy(), r.cpu().numpy()
        ref = Psi @ Pb
        assert np.abs(Phi - ref).max() <= 1e-13 * np.abs(ref).max()
        rr = sim.residual(lv[tau]["S"], lv[tau]["M"] if tau == 0 else _mass(lv, tau), ref, lam, lam_c=0.5,
                          norm="minv" if tau == 0 else "l2")
        assert np.abs(r - rr).max() <= 1e-12 * np.abs(rr).max()


@pytest.mark.parametrize("case", ["sphere2k", "sphere2k-default-coarsest", "torus"])
def test_hsim_end_to_end(cuda, case):
    import paper_2111_09039_amd as hs
    if case == "sphere2k":
        V, F, d = synth.config_mesh("sphere2k", seed=0)
        p, T, nc = 20, 3, 300
    elif case == "sphere2k-default-coarsest":
        # the small configuration exactly as the library sizes it: levels 2562, 1601, 1000
        V, F, d = synth.config_mesh("sphere2k", seed=0)
        p, T, nc = 20, 3, 0
    else:
        rng = np.random.default_rng(11)
        V, F = synth.torus(60, 30)
        V = synth.isotropic_noise(V, F, 0.2 * synth.mean_edge_length(V, F), rng)
        d = synth.random_density(len(V), rng)
        p, T, nc = 24, 3, 200
    print(f"[end-to-end {case}] n={len(V)} p={p}", flush=True)
    S, m = assembly.assemble(V, F, density=d)
    H = hs.Hierarchy(V, F, p, density=d, levels=T, n_coarsest=nc)
    if nc == 0:
        assert [H.level_info(t)["n"] for t in range(H.levels)] == [2562, 1601, 1000]
    ev, X, r, st = H.solve(tol=1e-10)
    ev, X, r = ev.cpu().numpy(), X.cpu().numpy(), r.cpu().numpy()
    lr, Xr, _, _ = sim.sim_lowest(S, m, p + 10, eps=1e-12)
    rel = np.abs(ev - lr[:p])[1:] / lr[1:p]
    assert rel.max() <= 1e-9, rel.max()
    assert abs(ev[0]) <= 1e-10 * lr[1]
    assert metrics.m_orthonormality(X, m) < 1e-10
    assert r.max() < 1e-10
    err = metrics.eigenvector_err(X, Xr, m, lr)
    assert err.max() < 1e-6, err.max()
    # host-side residual with the oracle's own assembly
    rh = sim.residual(S, m, X, ev)
    assert rh.max() < 2e-10
    # sign convention: largest-magnitude entry positive
    idx = np.argmax(np.abs(X), axis=0)
    assert (X[idx, np.arange(p)] > 0).all()


def test_hsim_dirichlet_end_to_end(cuda):
    # surface with boundary, Dirichlet condition: HSIM on the interior unknowns
    # against the dense generalized eigenproblem of the oracle's restriction
    import paper_2111_09039_amd as hs
    rng = np.random.default_rng(8)
    V, F = synth.rectangle_grid(60, 40, 0.05)
    V = synth.isotropic_noise(V, F, 0.2 * synth.mean_edge_length(V, F), rng)
    S, m = assembly.assemble(V, F)
    Si, mi, interior = assembly.dirichlet(S, m, F)
    p = 20
    H = hs.Hierarchy(V, F, p, levels=3, n_coarsest=200, boundary="dirichlet")
    print(f"[dirichlet] n={len(V)} interior={len(interior)} levels {[H.level_info(t)['n'] for t in range(3)]}",
          flush=True)
    ev, X, r, st = H.solve(tol=1e-10)
    ev, X, r = ev.cpu().numpy(), X.cpu().numpy(), r.cpu().numpy()
    lr, Xr = sl.eigh(Si.toarray(), np.diag(mi), subset_by_index=[0, p + 9])
    assert np.abs(ev - lr[:p]).max() <= 1e-9 * lr[p - 1], np.abs(ev - lr[:p]).max()
    boundary = np.setdiff1d(np.arange(len(V)), interior)
    assert (X[boundary] == 0).all()
    Xi = X[interior]
    assert r.max() < 1e-10
    assert metrics.m_orthonormality(Xi, mi) < 1e-10
    assert sim.residual(Si, mi, Xi, ev).max() < 2e-10
    assert metrics.eigenvector_err(Xi, Xr, mi, lr).max() < 1e-6
    # mixed precision (FP32 solves with FP64 refinement) reaches the same pairs
    evm, Xm, rm, stm = H.solve(tol=1e-10, precision=hs.MIXED)
    evm, Xm = evm.cpu().numpy(), Xm.cpu().numpy()
    assert np.abs(evm - lr[:p]).max() <= 1e-9 * lr[p - 1], np.abs(evm - lr[:p]).max()
    assert (Xm[boundary] == 0).all() and rm.max().item() < 1e-10


def test_adjoint_dirichlet_vs_dense_reference(cuda):
    # Dirichlet condition: eigenvalue + cluster-invariant eigenvector loss on a
    # bumped open sheet with density, against the oracle's dense gradient of the
    # interior problem (boundary vertices included: they move the interior's
    # cotangent weights and masses)
    import torch
    import paper_2111_09039_amd as hs
    from oracle import gradient
    rng = np.random.default_rng(12)
    V, F = synth.rectangle_grid(40, 30, 0.05)
    V = synth.isotropic_noise(V, F, 0.15 * synth.mean_edge_length(V, F), rng)
    V[:, 2] += 0.3 * np.exp(-((V[:, 0] - 1.0) ** 2 + (V[:, 1] - 0.7) ** 2) / 0.2)
    d = synth.random_density(len(V), rng)
    p = 12
    H = hs.Hierarchy(V, F, p, levels=2, n_coarsest=200, boundary="dirichlet", density=d)
    print(f"[adjoint dirichlet] n={len(V)} p={p}", flush=True)
    ev, X, r, st = H.solve(tol=1e-11, save_forward=True)
    lam = ev.cpu().numpy()
    cl = gradient.clusters_of(lam, 1e-2)
    wl = np.random.default_rng(1).uniform(0.5, 2.0, p)
    T = np.random.default_rng(4).standard_normal((len(V), p))

    def grad_X(Xn):
        G = np.zeros_like(Xn)
        for c in np.unique(cl[:p]):
            idx = np.nonzero(cl[:p] == c)[0]
            G[:, idx] = 2 * T[:, idx] @ (Xn[:, idx].T @ T[:, idx]).T
        return G

    gl = torch.from_numpy(2 * wl * lam).cuda()
    gX = torch.from_numpy(grad_X(X.cpu().numpy())).cuda()
    gV = H.backward(grad_evals=gl, grad_evecs=gX).cpu().numpy()
    gr, lr, _ = gradient.reference_gradient(V, F, p, grad_lam=lambda l: 2 * wl * l, grad_X=grad_X, density=d,
                                            boundary="dirichlet")
    assert np.abs(lam - lr).max() <= 1e-9 * lr[-1]
    err = np.linalg.norm(gV - gr) / np.linalg.norm(gr)
    print(f"[adjoint dirichlet] rel err vs dense reference {err:.2e}", flush=True)
    assert err < 1e-6
    # eigenvalue part alone, the tighter bar of the Neumann test
    gV1 = H.backward(grad_evals=gl).cpu().numpy()
    gr1, _, _ = gradient.reference_gradient(V, F, p, grad_lam=lambda l: 2 * wl * l, density=d, boundary="dirichlet")
    assert np.linalg.norm(gV1 - gr1) / np.linalg.norm(gr1) < 1e-7


def test_adjoint_circumcentric_vs_dense_reference(cuda):
    # circumcentric lumping: eigenvalue + cluster-invariant eigenvector loss on a
    # noisy torus with density, against the oracle's dense gradient of that lumping
    import torch
    import paper_2111_09039_amd as hs
    from oracle import gradient
    rng = np.random.default_rng(13)
    V, F = synth.torus(36, 24)
    V = synth.isotropic_noise(V, F, 0.1 * synth.mean_edge_length(V, F), rng)
    d = synth.random_density(len(V), rng)
    assert assembly.lumped_mass(V, F, lumping="voronoi").min() > 0
    p = 12
    H = hs.Hierarchy(V, F, p, levels=2, n_coarsest=200, lumping=1, density=d)
    print(f"[adjoint circumcentric] n={len(V)} p={p}", flush=True)
    ev, X, r, st = H.solve(tol=1e-11, save_forward=True)
    lam = ev.cpu().numpy()
    cl = gradient.clusters_of(lam, 1e-2)
    wl = np.random.default_rng(1).uniform(0.5, 2.0, p)
    T = np.random.default_rng(4).standard_normal((len(V), p))

    def grad_X(Xn):
        G = np.zeros_like(Xn)
        for c in np.unique(cl[:p]):
            idx = np.nonzero(cl[:p] == c)[0]
            G[:, idx] = 2 * T[:, idx] @ (Xn[:, idx].T @ T[:, idx]).T
        return G

    gl = torch.from_numpy(2 * wl * lam).cuda()
    gX = torch.from_numpy(grad_X(X.cpu().numpy())).cuda()
    gV = H.backward(grad_evals=gl, grad_evecs=gX).cpu().numpy()
    gr, lr, _ = gradient.reference_gradient(V, F, p, grad_lam=lambda l: 2 * wl * l, grad_X=grad_X, density=d,
                                            lumping="voronoi")
    assert np.abs(lam - lr)[1:].max() <= 1e-9 * lr[-1]
    err = np.linalg.norm(gV - gr) / np.linalg.norm(gr)
    print(f"[adjoint circumcentric] rel err vs dense reference {err:.2e}", flush=True)
    assert err < 1e-6
    gV1 = H.backward(grad_evals=gl).cpu().numpy()
    gr1, _, _ = gradient.reference_gradient(V, F, p, grad_lam=lambda l: 2 * wl * l, density=d, lumping="voronoi")
    assert np.linalg.norm(gV1 - gr1) / np.linalg.norm(gr1) < 1e-7




# ---------------------------------------------------------------- mixed precision
def test_mixed_solve_refinement(small):
    import paper_2111_09039_amd as hs
    V, F, S, m, lv, H = small
    rng = np.random.default_rng(7)
    for tau in (0, 1):
        St, Mt = lv[tau]["S"], _mass(lv, tau)
        n = St.shape[0]
        mu = 3.0
        H.factor(tau, mu, precision=hs.MIXED)
        B = rng.standard_normal((n, 9))
        X = H.solve_shifted(tau, _t(B), precision=hs.MIXED, refine_tol=1e-13).cpu().numpy()
        A = (St - mu * Mt).tocsc()
        Xr = spla.splu(A).solve(B)
        assert np.abs(X - Xr).max() <= 1e-10 * np.abs(Xr).max(), tau
        rel = np.linalg.norm(A @ X - B, axis=0) / np.linalg.norm(B, axis=0)
        assert rel.max() <= 1e-13


def test_mixed_gram(small):
    import paper_2111_09039_amd as hs
    V, F, S, m, lv, H = small
    rng = np.random.default_rng(8)
    for tau in range(3):
        n = len(lv[tau]["verts"])
        Psi = rng.standard_normal((n, 30))
        Sb, Mb = H.gram(tau, _t(Psi), precision=hs.MIXED)
        Sr = Psi.T @ (lv[tau]["S"] @ Psi)
        Mr = Psi.T @ (_mass(lv, tau) @ Psi)
        # FP32 rounding of the operands and FP32 accumulation over 256 rows
        assert np.abs(Sb.cpu().numpy() - Sr).max() <= 2e-5 * np.abs(Sr).max()
        assert np.abs(Mb.cpu().numpy() - Mr).max() <= 2e-5 * np.abs(Mr).max()
        assert np.abs(Sb.cpu().numpy() - Sr).max() > 0      # really the low-precision path


def test_compensated_gram(small):
    """Compensated Gram (hi/lo FP32 split of the FP64 operands, three FP32
    matrix-core products, FP64 sums of 32-row stages): more accurate than the
    FP32 Gram, bounded by the FP32 rounding of the matrix cores' accumulation
    (a 4-term sum per instruction), far above FP64 rounding."""
    import paper_2111_09039_amd as hs
    V, F, S, m, lv, H = small
    rng = np.random.default_rng(8)
    for tau in range(3):
        n = len(lv[tau]["verts"])
        Psi = rng.standard_normal((n, 30))
        Sr = Psi.T @ (lv[tau]["S"] @ Psi)
        Mr = Psi.T @ (_mass(lv, tau) @ Psi)
        Sc, Mc = (x.cpu().numpy() for x in H.gram(tau, _t(Psi), precision=hs.GRAM_COMPENSATED))
        S32, M32 = (x.cpu().numpy() for x in H.gram(tau, _t(Psi), precision=hs.MIXED))
        ec = max(np.abs(Sc - Sr).max() / np.abs(Sr).max(), np.abs(Mc - Mr).max() / np.abs(Mr).max())
        e32 = max(np.abs(S32 - Sr).max() / np.abs(Sr).max(), np.abs(M32 - Mr).max() / np.abs(Mr).max())
        print(f"[compensated gram] level {tau}: rel err {ec:.2e} (FP32 {e32:.2e})")
        assert ec <= 2e-7 and ec < 0.5 * e32 and ec > 0


def test_hsim_mixed_end_to_end(cuda):
    import paper_2111_09039_amd as hs
    V, F, d = synth.config_mesh("sphere2k", seed=0)
    p = 20
    S, m = assembly.assemble(V, F)
    H = hs.Hierarchy(V, F, p, levels=3, n_coarsest=300)
    ev, X, r, st = H.solve(tol=1e-6, precision=hs.MIXED)
    ev, X, r = ev.cpu().numpy(), X.cpu().numpy(), r.cpu().numpy()
    lr, Xr, _, _ = sim.sim_lowest(S, m, p + 10, eps=1e-12)
    rel = np.abs(ev - lr[:p])[1:] / lr[1:p]
    print(f"[mixed] max rel eig err {rel.max():.2e}, refine {st['refine_steps']}, escalated {st['escalated']}")
    assert rel.max() <= 1e-6
    assert r.max() < 1e-6
    assert sim.residual(S, m, X, ev).max() < 1.5e-6
    assert metrics.m_orthonormality(X, m) < 1e-8


# ---------------------------------------------------------------- adjoint
def _adjoint_mesh(nu=40, nv_=24, seed=0):
    rng = np.random.default_rng(seed)
    V, F = synth.torus(nu, nv_)
    V = synth.isotropic_noise(V, F, 0.2 * synth.mean_edge_length(V, F), rng)
    return V, F


def test_adjoint_eigenvalues_vs_dense_reference(cuda):
    import torch
    import paper_2111_09039_amd as hs
    from oracle import gradient
    V, F = _adjoint_mesh()
    p = 16
    wl = np.random.default_rng(1).uniform(0.5, 2.0, p)
    H = hs.Hierarchy(V, F, p, levels=2, n_coarsest=200)
    ev, X, r, st = H.solve(tol=1e-11, save_forward=True)
    gl = torch.from_numpy(2 * wl * ev.cpu().numpy()).cuda()
    gV = H.backward(grad_evals=gl).cpu().numpy()
    gr, lam, _ = gradient.reference_gradient(V, F, p, grad_lam=lambda l: 2 * wl * l)
    assert np.abs(ev.cpu().numpy() - lam)[1:].max() < 1e-9 * lam[-1]
    err = np.linalg.norm(gV - gr) / np.linalg.norm(gr)
    print(f"[adjoint eigenvalues] rel err vs dense reference {err:.2e}")
    assert err < 1e-7


def test_adjoint_eigenvectors_vs_dense_reference(cuda):
    import torch
    import paper_2111_09039_amd as hs
    from oracle import gradient
    V, F = _adjoint_mesh(seed=2)
    p = 12
    H = hs.Hierarchy(V, F, p, levels=2, n_coarsest=200)
    ev, X, r, st = H.solve(tol=1e-11, save_forward=True)
    lam = ev.cpu().numpy()
    cl = gradient.clusters_of(lam, 1e-2)
    T = np.random.default_rng(4).standard_normal((len(V), p))

    def grad_X(Xn):
        G = np.zeros_like(Xn)
        for c in np.unique(cl[:p]):
            idx = np.nonzero(cl[:p] == c)[0]
            G[:, idx] = 2 * T[:, idx] @ (Xn[:, idx].T @ T[:, idx]).T
        return G

    gX = torch.from_numpy(grad_X(X.cpu().numpy())).cuda()
    gV = H.backward(grad_evecs=gX).cpu().numpy()
    gr, _, _ = gradient.reference_gradient(V, F, p, grad_X=grad_X)
    err = np.linalg.norm(gV - gr) / np.linalg.norm(gr)
    print(f"[adjoint eigenvectors] rel err vs dense reference {err:.2e}")
    assert err < 1e-6


def test_autograd_function_fd(cuda):
    import torch
    import paper_2111_09039_amd as hs
    from paper_2111_09039_amd.autograd import eigs
    from oracle import gradient
    V, F = _adjoint_mesh(30, 20, seed=7)
    p = 10
    Vt = torch.tensor(V, requires_grad=True)
    Ft = torch.tensor(F)
    ev, X = eigs(Vt, Ft, p, levels=2, n_coarsest=150, tol=1e-12)
    cl = gradient.clusters_of(ev.detach().cpu().numpy(), 1e-2)
    T = torch.from_numpy(np.random.default_rng(3).standard_normal((len(V), p))).cuda()
    wl = torch.linspace(0.5, 1.5, p, dtype=torch.float64, device=ev.device)

    def loss_fn(ev, X):
        tot = (wl * ev ** 2).sum()
        for c in np.unique(cl[:p]):
            idx = torch.from_numpy(np.nonzero(cl[:p] == c)[0]).cuda()
            tot = tot + ((X[:, idx].T @ T[:, idx]) ** 2).sum()
        return tot

    loss_fn(ev, X).backward()
    g = Vt.grad.numpy()
    rng = np.random.default_rng(9)
    for _ in range(3):
        D = rng.standard_normal(V.shape)
        h = 1e-6
        with torch.no_grad():
            lp = loss_fn(*eigs(torch.tensor(V + h * D), Ft, p, levels=2, n_coarsest=150, tol=1e-12)).item()
            lm = loss_fn(*eigs(torch.tensor(V - h * D), Ft, p, levels=2, n_coarsest=150, tol=1e-12)).item()
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(g * D))
        print(f"[autograd fd] fd {fd:.10e} adjoint {an:.10e}")
        assert abs(fd - an) <= 1e-5 * abs(fd)


# ------------------------------------------------------- q above 160 columns
@pytest.fixture(scope="module")
def wide(cuda):
    """p = 120 (q = 180): the Gram and Ritz kernels take their general
    column tilings (more than 160 columns), the solves more column groups."""
    import paper_2111_09039_amd as hs
    rng = np.random.default_rng(21)
    V, F = synth.icosphere(5)
    V = synth.radial_jitter(V, 1e-2, rng)
    S, m = assembly.assemble(V, F)
    lv = hierarchy.build_hierarchy(V, F, S, m, p=120, levels=3, n_coarsest=400, seed=3)
    H = hs.Hierarchy(V, F, 120, levels=3, n_coarsest=400, seed=3)
    print(f"[wide hierarchy] sizes {[len(l['verts']) for l in lv]} q {H.q}", flush=True)
    assert H.q == 180
    return V, F, S, m, lv, H


def test_wide_gram_and_ritz(wide):
    V, F, S, m, lv, H = wide
    rng = np.random.default_rng(8)
    k = H.q
    for tau in range(3):
        n = len(lv[tau]["verts"])
        Psi = rng.standard_normal((n, k))
        Sb, Mb = H.gram(tau, _t(Psi))
        Sr = Psi.T @ (lv[tau]["S"] @ Psi)
        Mr = Psi.T @ (_mass(lv, tau) @ Psi)
        assert np.abs(Sb.cpu().numpy() - Sr).max() <= 1e-13 * np.abs(Sr).max(), tau
        assert np.abs(Mb.cpu().numpy() - Mr).max() <= 1e-13 * np.abs(Mr).max(), tau
        Pb = rng.standard_normal((k, k))
        lam = np.sort(rng.uniform(0.5, 20, k))
        Phi, r = H.ritz(tau, _t(Psi), _t(Pb), _t(lam), 0.5)
        Phi, r = Phi.cpu().numpy(), r.cpu().numpy()
        ref = Psi @ Pb
        assert np.abs(Phi - ref).max() <= 1e-13 * np.abs(ref).max(), tau
        rr = sim.residual(lv[tau]["S"], lv[tau]["M"] if tau == 0 else _mass(lv, tau), ref, lam, lam_c=0.5,
                          norm="minv" if tau == 0 else "l2")
        assert np.abs(r - rr).max() <= 1e-12 * np.abs(rr).max(), tau


def test_wide_hsim(wide):
    V, F, S, m, lv, H = wide
    p = 120
    ev, X, r, st = H.solve(tol=1e-9)
    ev, X, r = ev.cpu().numpy(), X.cpu().numpy(), r.cpu().numpy()
    print(f"[wide hsim] iters {st['iters']} total {st['ms_total']:.1f} ms", flush=True)
    lr, Xr, _, _ = sim.sim_lowest(S, m, p + 10, eps=1e-11)
    rel = np.abs(ev - lr[:p])[1:] / lr[1:p]
    assert rel.max() <= 1e-9, rel.max()
    assert r.max() < 1e-9
    assert metrics.m_orthonormality(X, m) < 1e-10
    assert sim.residual(S, m, X, ev).max() < 2e-9
    err = metrics.eigenvector_err(X, Xr, m, lr)
    assert err.max() < 1e-5, err.max()


def test_device_assembly_equals_host(cuda, monkeypatch):
    """The finest level's cotangent stiffness and lumped mass assembled on the
    device (the default build) equal the host assembly bit for bit (same
    terms, same order, no contraction), and the oracle's to rounding."""
    import paper_2111_09039_amd as hs
    rng = np.random.default_rng(5)
    V, F = synth.torus(60, 40)
    V = synth.isotropic_noise(V, F, 0.2 * synth.mean_edge_length(V, F), rng)
    d = synth.random_density(len(V), rng)
    Hd = hs.Hierarchy(V, F, 10, density=d, levels=2, n_coarsest=200)
    monkeypatch.setenv("HSIM_HOST_ASSEMBLY", "1")
    Hh = hs.Hierarchy(V, F, 10, density=d, levels=2, n_coarsest=200)
    ed, eh = Hd.export(0), Hh.export(0)
    for k in ("S_indptr", "S_indices", "S_data", "M_data", "U_data", "perm"):
        assert np.array_equal(ed[k], eh[k]), k
    S, m = assembly.assemble(V, F, density=d)
    Sd = sp.csr_matrix((ed["S_data"], ed["S_indices"], ed["S_indptr"]), shape=S.shape)
    assert abs(Sd - S).max() <= 1e-13 * abs(S).max()
    diag = np.zeros(len(V))
    rows = np.repeat(np.arange(len(V)), np.diff(ed["S_indptr"]))
    on = ed["S_indices"] == rows
    diag[rows[on]] = ed["M_data"][on]
    assert np.abs(diag - m).max() <= 1e-14 * m.max()
