"""torch.autograd.Function around hsim_solve / hsim_solve_backward.

eigs(V, F, p) returns (evals [p], evecs [nv, p]); the backward pass is the
library's hand-written adjoint (gradients with respect to the vertex
positions V through the cotangent and lumped-mass assembly).
"""
from __future__ import annotations

import torch

from . import FP64, Hierarchy


class _Eigs(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, F, p, density, options):
        H = Hierarchy(V.detach().cpu().double().numpy(), F.detach().cpu().numpy(), p,
                      density=None if density is None else density.detach().cpu().double().numpy(),
                      **options.get("build", {}))
        ev, X, r, st = H.solve(save_forward=True, **options.get("solve", {}))
        ctx.H = H
        ctx.V_device, ctx.V_dtype = V.device, V.dtype
        ctx.stats = st
        ctx.mark_non_differentiable(r)
        return ev, X, r

    @staticmethod
    def backward(ctx, g_ev, g_X, g_r):
        H = ctx.H
        gV = H.backward(g_ev if g_ev is not None else None, g_X if g_X is not None else None)
        return gV.to(ctx.V_device, ctx.V_dtype), None, None, None, None


def eigs(V, F, p, density=None, levels=0, n_coarsest=0, seed=0, tol=1e-10, precision=FP64, max_iters=200):
    """Lowest p eigenpairs (differentiable in V)."""
    opts = {"build": dict(levels=levels, n_coarsest=n_coarsest, seed=seed),
            "solve": dict(tol=tol, precision=precision, max_iters=max_iters)}
    ev, X, r = _Eigs.apply(V, F, p, density, opts)
    return ev, X
