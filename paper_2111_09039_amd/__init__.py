"""MI355X-native Hierarchical Subspace Iteration Method (HSIM) for the lowest
Laplace-Beltrami eigenpairs of triangle meshes.

Python binding of the C ABI (include/hsim.h).  It only marshals arguments:
PyTorch provides device memory and the current stream, every step of the
solver runs in the HIP library ``libhsim.so``.  Importing works without the
library; the first call that needs it raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import HsimError

__all__ = ["Hierarchy", "HsimError", "FP64", "MIXED", "GRAM_COMPENSATED", "build_library", "solve_batch",
           "rayleigh_ritz_dense"]

FP64, MIXED, GRAM_COMPENSATED = 0, 1, 2
FLAG_NOLOCK, FLAG_SAVE_FORWARD, FLAG_PROFILE, FLAG_DETERMINISTIC = 1, 2, 4, 8
FLAG_COMPENSATED_GRAM, FLAG_NO_FP32_GRAM, FLAG_FP32_GRAM, FLAG_GRAPH = 16, 32, 64, 128


def build_library(verbose=False):
    from .build import build
    return build(verbose=verbose)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != _torch().float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


class Hierarchy:
    """Handle of ``hsim_build_hierarchy``: levels, prolongations, Galerkin
    operators and the symbolic factor of every level, resident on the
    current device."""

    def __init__(self, V, F, p, density=None, levels=0, n_coarsest=0, growth_mode=0, lumping=0,
                 support_sigma=7.0, seed=0, host_only=False, boundary="neumann"):
        lib = _lib.load()
        V = np.ascontiguousarray(V, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.int32)
        if V.ndim != 2 or V.shape[1] != 3 or F.ndim != 2 or F.shape[1] != 3:
            raise ValueError("V must be (nv, 3) and F (nf, 3)")
        d = None if density is None else np.ascontiguousarray(density, dtype=np.float64)
        if d is not None and d.shape != (len(V),):
            raise ValueError("density must have one entry per vertex")
        o = _lib.BuildOpts()
        lib.hsim_default_build_opts(C.byref(o))
        o.p, o.levels, o.n_coarsest, o.growth_mode = int(p), int(levels), int(n_coarsest), int(growth_mode)
        o.lumping, o.support_sigma, o.seed = int(lumping), float(support_sigma), int(seed)
        o.flags = 1 if host_only else 0
        bc = {"neumann": 0, "natural": 0, "dirichlet": 1}
        if boundary not in bc:
            raise ValueError("boundary must be 'neumann' or 'dirichlet'")
        o.boundary = bc[boundary]
        h = C.c_void_p()
        _lib.check(lib.hsim_build_hierarchy(V.ctypes.data_as(C.c_void_p), len(V), F.ctypes.data_as(C.c_void_p),
                                            len(F), None if d is None else d.ctypes.data_as(C.c_void_p),
                                            C.byref(o), C.byref(h)))
        self._h = h
        self.nv = len(V)
        T, q, pp = C.c_int32(), C.c_int32(), C.c_int32()
        _lib.check(lib.hsim_hierarchy_shape(h, C.byref(T), C.byref(q), C.byref(pp)))
        self.levels, self.q, self.p = T.value, q.value, pp.value

    # ------------------------------------------------------------------ life
    def close(self):
        if getattr(self, "_h", None):
            _lib.load().hsim_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("hierarchy is closed")
        return self._h

    # ----------------------------------------------------------- solve
    def solve(self, tol=1e-2, shift_alpha=0.1, precision=FP64, max_iters=100, lock=True, save_forward=False,
              stream=None, raise_noconv=True, profile=False, compensated_gram=False, fp32_gram=None, graph=False):
        """Returns (evals [p], evecs [nv, p], resid [p], stats dict) with CUDA
        float64 tensors; evecs is the transpose view of a (p, nv) buffer.
        fp32_gram (mixed precision): None = the library's rule (FP32 interim
        Gram above q = 160), True = at any q, False = never; compensated_gram:
        the compensated FP32 Gram instead of the FP64 one near convergence."""
        torch = _torch()
        lib = _lib.load()
        o = _lib.SolveOpts()
        lib.hsim_default_solve_opts(C.byref(o))
        o.tol, o.shift_alpha, o.precision, o.max_iters = float(tol), float(shift_alpha), int(precision), int(max_iters)
        o.flags = ((0 if lock else FLAG_NOLOCK) | (FLAG_SAVE_FORWARD if save_forward else 0)
                   | (FLAG_PROFILE if profile else 0) | (FLAG_COMPENSATED_GRAM if compensated_gram else 0)
                   | {None: 0, True: FLAG_FP32_GRAM, False: FLAG_NO_FP32_GRAM}[fp32_gram]
                   | (FLAG_GRAPH if graph else 0))
        o.stream = _stream_ptr(stream)
        dev = torch.device("cuda", torch.cuda.current_device())
        ev = torch.empty(self.p, dtype=torch.float64, device=dev)
        X = torch.empty(self.p, self.nv, dtype=torch.float64, device=dev)
        r = torch.empty(self.p, dtype=torch.float64, device=dev)
        st = _lib.Stats()
        code = lib.hsim_solve(self.handle, C.byref(o), _dptr(ev), _dptr(X), _dptr(r), C.byref(st))
        if code != 0 and (raise_noconv or code != -4):
            _lib.check(code)
        stats = st.as_dict()
        stats["status"] = _lib.STATUS.get(code, code)
        return ev, X.t(), r, stats

    def backward(self, grad_evals=None, grad_evecs=None, stream=None):
        """dL/dV (nv x 3) for the last solve (run with save_forward=True);
        grad_evecs is (nv, p)."""
        torch = _torch()
        lib = _lib.load()
        dev = torch.device("cuda", torch.cuda.current_device())
        gV = torch.empty(self.nv, 3, dtype=torch.float64, device=dev)
        ge = None if grad_evals is None else grad_evals.detach().to(dev, torch.float64).contiguous()
        gx = None if grad_evecs is None else grad_evecs.detach().to(dev, torch.float64).t().contiguous()
        _lib.check(lib.hsim_solve_backward(self.handle, _dptr(ge), _dptr(gx), _dptr(gV), _stream_ptr(stream)))
        return gV

    def autotune(self, level=0, stream=None):
        """hsim_autotune: pick and keep the fastest block-solve launch plan of a
        level; returns dict(big_ns, big_ns_bwd, ms, from_cache)."""
        r = _lib.TuneResult()
        _lib.check(_lib.load().hsim_autotune(self.handle, int(level), _stream_ptr(stream), C.byref(r)))
        return {k: getattr(r, k) for k, _ in _lib.TuneResult._fields_}

    # ---------------------------------------------------------- inspection
    def level_info(self, level):
        d = _lib.LevelDesc()
        _lib.check(_lib.load().hsim_level_info(self.handle, int(level), C.byref(d)))
        return {k: getattr(d, k) for k, _ in _lib.LevelDesc._fields_}

    def export(self, level):
        """Host copies of one level: verts, S (CSR), M values on S's pattern,
        U (CSR, rows = this level, cols = next coarser), perm."""
        info = self.level_info(level)
        n, nnz, nu = info["n"], info["nnz"], info["nnz_u"]
        # zero-filled: the coarsest level has no U and no elimination order
        out = dict(verts=np.zeros(n, np.int64), S_indptr=np.zeros(n + 1, np.int64), S_indices=np.zeros(nnz, np.int32),
                   S_data=np.zeros(nnz), M_data=np.zeros(nnz), U_indptr=np.zeros(n + 1, np.int64),
                   U_indices=np.zeros(max(nu, 1), np.int32), U_data=np.zeros(max(nu, 1)),
                   perm=np.zeros(n, np.int32))
        ptr = {k: v.ctypes.data_as(C.c_void_p) for k, v in out.items()}
        _lib.check(_lib.load().hsim_level_export(self.handle, int(level), ptr["verts"], ptr["S_indptr"],
                                                 ptr["S_indices"], ptr["S_data"], ptr["M_data"], ptr["U_indptr"],
                                                 ptr["U_indices"], ptr["U_data"], ptr["perm"]))
        out["U_indices"], out["U_data"] = out["U_indices"][:nu], out["U_data"][:nu]
        return out

    # ------------------------------------------------------------- steps
    def prolong(self, level, Xc):
        torch = _torch()
        n = self.level_info(level)["n"]
        Y = torch.empty(n, Xc.shape[1], dtype=torch.float64, device=Xc.device)
        _lib.check(_lib.load().hsim_step_prolong(self.handle, level, Xc.shape[1], _dptr(Xc), _dptr(Y), _stream_ptr()))
        return Y

    def apply(self, level, op, X):
        torch = _torch()
        Y = torch.empty_like(X)
        _lib.check(_lib.load().hsim_step_apply(self.handle, level, int(op), X.shape[1], _dptr(X), _dptr(Y),
                                               _stream_ptr()))
        return Y

    def factor(self, level, mu, precision=FP64):
        neg = C.c_int32()
        _lib.check(_lib.load().hsim_step_factor(self.handle, level, float(mu), int(precision), C.byref(neg),
                                                _stream_ptr()))
        return neg.value

    def solve_shifted(self, level, B, precision=FP64, refine_tol=1e-12):
        torch = _torch()
        X = torch.empty_like(B)
        _lib.check(_lib.load().hsim_step_solve(self.handle, level, B.shape[1], _dptr(B), _dptr(X), int(precision),
                                               float(refine_tol), _stream_ptr()))
        return X

    def gram(self, level, Psi, precision=FP64):
        torch = _torch()
        k = Psi.shape[1]
        Sb = torch.empty(k, k, dtype=torch.float64, device=Psi.device)
        Mb = torch.empty(k, k, dtype=torch.float64, device=Psi.device)
        _lib.check(_lib.load().hsim_step_gram(self.handle, level, k, _dptr(Psi), _dptr(Sb), _dptr(Mb), int(precision),
                                              _stream_ptr()))
        return Sb, Mb

    def ritz(self, level, Psi, Phibar, lam, lam_floor):
        torch = _torch()
        k = Psi.shape[1]
        Phi = torch.empty_like(Psi)
        r = torch.empty(k, dtype=torch.float64, device=Psi.device)
        _lib.check(_lib.load().hsim_step_ritz(self.handle, level, k, _dptr(Psi), _dptr(Phibar), _dptr(lam),
                                              float(lam_floor), _dptr(Phi), _dptr(r), _stream_ptr()))
        return Phi, r

    def coarse(self, k):
        torch = _torch()
        n = self.level_info(self.levels - 1)["n"]
        dev = torch.device("cuda", torch.cuda.current_device())
        lam = torch.empty(k, dtype=torch.float64, device=dev)
        X = torch.empty(n, k, dtype=torch.float64, device=dev)
        sw = C.c_int32()
        _lib.check(_lib.load().hsim_step_coarse(self.handle, int(k), _dptr(lam), _dptr(X), C.byref(sw), _stream_ptr()))
        return lam, X, sw.value


def solve_batch(hierarchies, tol=1e-2, shift_alpha=0.1, precision=FP64, max_iters=100, lock=True, streams=0,
                graph=False, stream=None):
    """hsim_solve_batch: solve many hierarchies at once over `streams` worker
    streams.  Returns a list of (evals [p], evecs [nv, p], resid [p], stats)
    per hierarchy and the list of per-mesh status names."""
    torch = _torch()
    lib = _lib.load()
    o = _lib.SolveOpts()
    lib.hsim_default_solve_opts(C.byref(o))
    o.tol, o.shift_alpha, o.precision, o.max_iters = float(tol), float(shift_alpha), int(precision), int(max_iters)
    o.flags = (0 if lock else FLAG_NOLOCK) | (FLAG_GRAPH if graph else 0)
    o.stream = _stream_ptr(stream)
    dev = torch.device("cuda", torch.cuda.current_device())
    n = len(hierarchies)
    evs = [torch.empty(H.p, dtype=torch.float64, device=dev) for H in hierarchies]
    Xs = [torch.empty(H.p, H.nv, dtype=torch.float64, device=dev) for H in hierarchies]
    rs = [torch.empty(H.p, dtype=torch.float64, device=dev) for H in hierarchies]
    P = C.c_void_p * n
    hs = P(*[H.handle for H in hierarchies])
    pe, px, pr = P(*[t.data_ptr() for t in evs]), P(*[t.data_ptr() for t in Xs]), P(*[t.data_ptr() for t in rs])
    stats = (_lib.Stats * n)()
    status = (C.c_int32 * n)()
    code = lib.hsim_solve_batch(hs, n, C.byref(o), pe, px, pr, stats, status, int(streams))
    if code not in (0, -4):
        _lib.check(code)
    out = [(evs[i], Xs[i].t(), rs[i], stats[i].as_dict()) for i in range(n)]
    return out, [_lib.STATUS.get(c, c) for c in status]


def rayleigh_ritz_dense(Sbar, Mbar):
    """Reduced dense eigenproblem on the device: (lam [k], Phibar [k, k], sweeps)."""
    torch = _torch()
    k = Sbar.shape[0]
    lam = torch.empty(k, dtype=torch.float64, device=Sbar.device)
    Pb = torch.empty(k, k, dtype=torch.float64, device=Sbar.device)
    sw = C.c_int32()
    _lib.check(_lib.load().hsim_step_rr(k, _dptr(Sbar.contiguous()), _dptr(Mbar.contiguous()), _dptr(lam), _dptr(Pb),
                                        C.byref(sw), _stream_ptr()))
    return lam, Pb, sw.value
