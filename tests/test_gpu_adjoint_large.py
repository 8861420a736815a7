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
  directions, each within a relative error of 1e-5;
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


def _loss_parts(lam0, n, seed=11):
    """Per-pair weights and targets, constant within clusters, and the
    clusters (index arrays) that lie wholly inside the first P pairs."""
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
    """torch: eigenvalue term + alignment sum_C ||X_C^T M T_C||_F^2."""
    import torch
    tot = (torch.as_tensor(w) * (ev - torch.as_tensor(lhat)) ** 2).sum()
    MT = m[:, None] * torch.as_tensor(T)
    for idx in full:
        ii = torch.as_tensor(idx)
        tot = tot + ((X[:, ii].T @ MT[:, ii]) ** 2).sum()
    return tot


@pytest.mark.slow
def test_adjoint_fd_200k(cuda):
    import torch
    from paper_2111_09039_amd.autograd import eigs
    V, F, _ = synth.config_mesh("torus200k", seed=0)
    n = len(V)
    Ft = torch.tensor(F, dtype=torch.int64)
    Vt = torch.tensor(V, requires_grad=True)
    ev, X = eigs(Vt, torch.tensor(F), P, levels=2, tol=TOL)
    lam0 = ev.detach().cpu().numpy()
    w, lhat, full, T = _loss_parts(lam0, n)
    assert sum(len(i) for i in full) >= P - 4
    L0 = _loss(ev.cpu(), X.cpu(), gradient.lumped_mass_torch(Vt, Ft), w, lhat, full, T)
    L0.backward()
    g = Vt.grad.numpy()
    print(f"[adjoint 200k] n {n}, clusters {len(full)}, loss {L0.item():.6e}", flush=True)

    def L_at(Vn):
        with torch.no_grad():
            Vn_t = torch.tensor(Vn)
            e, Xn = eigs(Vn_t, torch.tensor(F), P, levels=2, tol=TOL)
            return _loss(e.cpu(), Xn.cpu(), gradient.lumped_mass_torch(Vn_t, Ft), w, lhat, full, T).item()

    h = 1e-6
    D = synth.gaussian_matrix(n, 3 * 32, seed=31)
    worst = 0.0
    for k in range(32):
        d = D[:, 3 * k:3 * k + 3]
        fd = (L_at(V + h * d) - L_at(V - h * d)) / (2 * h)
        an = float(np.sum(g * d))
        rel = abs(fd - an) / abs(fd)
        worst = max(worst, rel)
        print(f"[adjoint 200k] direction {k}: fd {fd:.10e} adjoint {an:.10e} rel {rel:.2e}", flush=True)
        assert rel <= 1e-5, (k, fd, an)
    print(f"[adjoint 200k] worst relative FD error over 32 directions {worst:.2e}", flush=True)


def test_adjoint_vs_dense_reference_2k(cuda):
    import torch
    import paper_2111_09039_amd as hs
    V, F, _ = synth.config_mesh("torus2k", seed=0)
    n = len(V)
    H = hs.Hierarchy(V, F, P, levels=2, n_coarsest=400)
    ev, X, r, st = H.solve(tol=1e-12, save_forward=True)
    lam = ev.cpu().numpy()
    w, lhat, full, T = _loss_parts(lam, n)
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

    gV = H.backward(grad_evals=torch.from_numpy(grad_lam(lam)).cuda(),
                    grad_evecs=torch.from_numpy(grad_X(X.cpu().numpy())).cuda()).cpu().numpy()
    gr, lr, _ = gradient.reference_gradient(V, F, P, grad_lam=grad_lam, grad_X=grad_X)
    assert np.abs(lam - lr)[1:].max() <= 1e-9 * lr[-1]
    err = np.linalg.norm(gV - gr) / np.linalg.norm(gr)
    print(f"[adjoint 2k] relative error against the dense reference gradient {err:.2e}", flush=True)
    assert err < 1e-6
