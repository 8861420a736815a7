"""The adjoint at the differentiation workload's size: perturbed 200k-vertex
torus (500 x 400), p = 64, FP64 forward.

Loss (clusters: relative eigenvalue gaps < 1e-2 at the unperturbed mesh;
weights and targets constant within a cluster, so the loss is invariant to
rotations inside near-degenerate clusters such as the torus's +-m pairs):

    L(V) = sum_k w_k (lambda_k - lhat_k)^2 + sum_C || X_C^T M(V) T_C ||_F^2

over the clusters that lie wholly inside the first p pairs, with seeded
target fields T.  Its gradient with respect to the 200k x 3 vertex positions
comes from the library's adjoint (through torch.autograd for the direct
M(V) term of the alignment) and is checked

* against central finite differences (h = 1e-6) of L along 32 seeded random
  directions with N(0, 0.1^2) entries, each within a relative error of 1e-5.
  The scale balances the two errors of the difference: with N(0, 1) entries
  some vertices of the noisy mesh move by a percent of their shortest edge
  and the O(h^2) truncation error reaches 1e-5 (measured 1.3e-3 / 1.4e-5 /
  1.3e-7 at h = 1e-5 / 1e-6 / 1e-7); with unit-norm directions the change of
  L is so small that the rounding of the eigenvalues (about eps * lambda_max
  each) reaches 1e-5 of it; at 0.1 both stay near 1e-7.  The loss is evaluated
  with a fixed number of lock-free subspace iterations, beyond the converged
  solve's count, so that both sides of a difference take the same steps;
* on the 2,000-vertex copy (50 x 40 torus), against the oracle's dense FP64
  reference gradient (all eigenpairs, explicit derivative formulas) for the
  same cotangents of the eigenvalues and eigenvectors.
"""
import numpy as np
import pytest

import synth
from oracle import gradient

pytestmark = pytest.mark.gpu

P = 64
TOL = 1e-10
# The floored residual of the constant mode (eq. conv2 with lambda_c = lambda_1)
# cannot fall below about u lambda_max / lambda_1 in FP64: a rounding-level
# error of the constant vector is multiplied by S.  On the 200k torus that is
# 2.2e-16 * 2.52e6 / 0.968 = 5.7e-10, so its forward solve asks for 2e-9
# (the 2k copy's floor is far below 1e-10).
TOL_200K = 2e-9


def _loss_parts(lam0, n, seed=11):
    """Per-pair weights and targets, constant within clusters, and the
    clusters (index arrays) that lie wholly inside the first P pairs.  lam0
    must hold eigenvalues beyond index P - 1, so that a cluster cut by P (whose
    part inside P is not invariant to rotations in the cluster) is seen."""
    assert len(lam0) > P
    cl = gradient.clusters_of(lam0, 1e-2)
    rng = np.random.default_rng(seed)
    ncl = int(cl.max()) + 1
    wc, oc = rng.uniform(0.5, 2.0, ncl), rng.uniform(-0.05, 0.05, ncl)
    full = [np.nonzero(cl[:P] == c)[0] for c in range(ncl)
            if np.all(np.nonzero(cl == c)[0] < P) and np.any(cl[:P] == c)]
    w = np.zeros(P)
    lhat = np.zeros(P)
    for idx in full:
        w[idx] = wc[cl[idx[0]]]
        lhat[idx] = lam0[idx].mean() * (1.0 + oc[cl[idx[0]]])
    T = synth.gaussian_matrix(n, P, seed + 1)
    return w, lhat, full, T


def _loss(ev, X, m, w, lhat, full, T):
    """torch: (eigenvalue term, alignment sum_C ||X_C^T M T_C||_F^2)."""
    import torch
    val = (torch.as_tensor(w) * (ev - torch.as_tensor(lhat)) ** 2).sum()
    MT = m[:, None] * torch.as_tensor(T)
    align = 0.0
    for idx in full:
        ii = torch.as_tensor(idx)
        align = align + ((X[:, ii].T @ MT[:, ii]) ** 2).sum()
    return val, align


def test_adjoint_vs_dense_reference_2k(cuda):
    import torch
    import paper_2111_09039_amd as hs
    V, F, _ = synth.config_mesh("torus2k", seed=0)
    n = len(V)
    Hx = hs.Hierarchy(V, F, P + 8, levels=2, n_coarsest=400)
    lam_ext = Hx.solve(tol=1e-10)[0].cpu().numpy()
    Hx.close()
    H = hs.Hierarchy(V, F, P, levels=2, n_coarsest=400)
    ev, X, r, st = H.solve(tol=1e-12, save_forward=True)
    lam = ev.cpu().numpy()
    w, lhat, full, T = _loss_parts(lam_ext, n)
    from oracle import assembly
    _, m = assembly.assemble(V, F)
    MT = m[:, None] * T

    def grad_lam(l):
        return 2.0 * w * (l - lhat)

    def grad_X(Xn):
        G = np.zeros_like(Xn)
        for idx in full:
            G[:, idx] = 2.0 * MT[:, idx] @ (Xn[:, idx].T @ MT[:, idx]).T
        return G

    gl = torch.from_numpy(grad_lam(lam)).cuda()
    gx = torch.from_numpy(grad_X(X.cpu().numpy())).cuda()
    gV = H.backward(grad_evals=gl, grad_evecs=gx).cpu().numpy()
    gr, lr, _ = gradient.reference_gradient(V, F, P, grad_lam=grad_lam, grad_X=grad_X)
    assert np.abs(lam - lr)[1:].max() <= 1e-9 * lr[-1]
    err = np.linalg.norm(gV - gr) / np.linalg.norm(gr)
    # the two parts separately
    gV1 = H.backward(grad_evals=gl).cpu().numpy()
    gr1, _, _ = gradient.reference_gradient(V, F, P, grad_lam=grad_lam)
    gV2 = H.backward(grad_evecs=gx).cpu().numpy()
    gr2, _, _ = gradient.reference_gradient(V, F, P, grad_X=grad_X)
    e1 = np.linalg.norm(gV1 - gr1) / np.linalg.norm(gr1)
    e2 = np.linalg.norm(gV2 - gr2) / np.linalg.norm(gr2)
    print(f"[adjoint 2k] relative error against the dense reference gradient {err:.2e} "
          f"(eigenvalue cotangent {e1:.2e}, eigenvector cotangent {e2:.2e})", flush=True)
    assert err < 1e-6 and e1 < 1e-6 and e2 < 1e-6


@pytest.mark.slow
def test_adjoint_fd_200k(cuda):
    import torch
    import paper_2111_09039_amd as hs
    from paper_2111_09039_amd.autograd import eigs
    V, F, _ = synth.config_mesh("torus200k", seed=0)
    n = len(V)
    Ft = torch.tensor(F, dtype=torch.int64)
    Vt = torch.tensor(V, requires_grad=True)
    ev, X = eigs(Vt, torch.tensor(F), P, levels=2, tol=TOL_200K)
    Hx = hs.Hierarchy(V, F, P + 8, levels=2)
    lam_ext = Hx.solve(tol=TOL_200K)[0].cpu().numpy()
    Hx.close()
    w, lhat, full, T = _loss_parts(lam_ext, n)
    assert sum(len(i) for i in full) >= P - 4
    Lv, La = _loss(ev.cpu(), X.cpu(), gradient.lumped_mass_torch(Vt, Ft), w, lhat, full, T)
    Lv.backward(retain_graph=True)
    gv = Vt.grad.numpy().copy()
    Vt.grad = None
    La.backward()
    ga = Vt.grad.numpy().copy()
    g = gv + ga
    print(f"[adjoint 200k] n {n}, clusters {len(full)}, loss {Lv.item():.6e} + {La.item():.6e}", flush=True)

    # The finite differences evaluate the loss through a forward pass with a
    # fixed number of subspace iterations and no locking, so that both sides
    # of a difference take the same steps (the computed eigenpairs are then a
    # smooth function of V); the count exceeds the converged solve's, so the
    # iterate is at least as accurate (residual at the FP64 floor).
    H0 = hs.Hierarchy(V, F, P, levels=2)
    it0 = H0.solve(tol=TOL_200K)[3]["iters"][-1]
    H0.close()
    n_it = it0 + 6

    def L_at(Vn):
        H = hs.Hierarchy(Vn, F, P, levels=2)
        e, Xn, _, st = H.solve(tol=1e-15, max_iters=n_it, lock=False, raise_noconv=False)
        H.close()
        with torch.no_grad():
            a, b = _loss(e.cpu(), Xn.cpu(), gradient.lumped_mass_torch(torch.tensor(Vn), Ft), w, lhat, full, T)
            return np.array([a.item(), b.item()])

    h = 1e-6
    D = synth.gaussian_matrix(n, 3 * 32, seed=31)
    worst = 0.0
    for k in range(32):
        d = 0.1 * D[:, 3 * k:3 * k + 3]
        fdp = (L_at(V + h * d) - L_at(V - h * d)) / (2 * h)
        anp = np.array([np.sum(gv * d), np.sum(ga * d)])
        fd, an = float(fdp.sum()), float(anp.sum())
        rel = abs(fd - an) / abs(fd)
        worst = max(worst, rel)
        print(f"[adjoint 200k] direction {k}: fd {fd:.10e} adjoint {an:.10e} rel {rel:.2e} "
              f"(eigenvalue term {abs(fdp[0] - anp[0]) / abs(fdp[0]):.1e}, alignment "
              f"{abs(fdp[1] - anp[1]) / abs(fdp[1]):.1e})", flush=True)
        assert rel <= 1e-5, (k, fd, an)
    print(f"[adjoint 200k] worst relative FD error over 32 directions {worst:.2e}", flush=True)
