"""ctypes declarations of the C ABI in include/hsim.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsim.so")


class BuildOpts(C.Structure):
    _fields_ = [("p", C.c_int32), ("levels", C.c_int32), ("n_coarsest", C.c_int32), ("growth_mode", C.c_int32),
                ("lumping", C.c_int32), ("support_sigma", C.c_double), ("seed", C.c_uint64),
                ("flags", C.c_int32), ("boundary", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("shift_alpha", C.c_double), ("precision", C.c_int32),
                ("max_iters", C.c_int32), ("flags", C.c_int32), ("reserved", C.c_int32), ("stream", C.c_void_p)]


MAX_LEVELS = 8
KCLASSES = ["solve_fwd", "solve_bwd", "factor", "gram", "ritz", "spmm", "dense_eig", "other"]


class Stats(C.Structure):
    _fields_ = [("levels", C.c_int32), ("q", C.c_int32), ("iters", C.c_int32 * MAX_LEVELS),
                ("n", C.c_int64 * MAX_LEVELS), ("nnz_factor", C.c_int64 * MAX_LEVELS),
                ("neg_pivots", C.c_int32 * MAX_LEVELS), ("mu", C.c_double * MAX_LEVELS),
                ("refine_steps", C.c_int32), ("escalated", C.c_int32), ("ms_build", C.c_double),
                ("ms_coarse", C.c_double), ("ms_factor", C.c_double), ("ms_solve", C.c_double),
                ("ms_gram", C.c_double), ("ms_rr", C.c_double), ("ms_ritz", C.c_double),
                ("ms_prolong", C.c_double), ("ms_total", C.c_double),
                ("k_ms", C.c_double * 8), ("k_launches", C.c_int64 * 8), ("k_bytes", C.c_double * 8),
                ("k_flops", C.c_double * 8), ("block_solves", C.c_int64), ("block_solve_cols", C.c_int64),
                ("gram_steps", C.c_int32 * 3), ("block_solves_fp32", C.c_int64)]

    def as_dict(self):
        T = self.levels
        return dict(levels=T, q=self.q, iters=list(self.iters[:T]), n=list(self.n[:T]),
                    nnz_factor=list(self.nnz_factor[:T]), neg_pivots=list(self.neg_pivots[:T]),
                    mu=list(self.mu[:T]), refine_steps=self.refine_steps, escalated=self.escalated,
                    ms_build=self.ms_build, ms_coarse=self.ms_coarse, ms_factor=self.ms_factor,
                    ms_solve=self.ms_solve, ms_gram=self.ms_gram, ms_rr=self.ms_rr, ms_ritz=self.ms_ritz,
                    ms_prolong=self.ms_prolong, ms_total=self.ms_total, block_solves=self.block_solves,
                    block_solve_cols=self.block_solve_cols, gram_steps=list(self.gram_steps),
                    block_solves_fp32=self.block_solves_fp32,
                    kernels={name: dict(ms=self.k_ms[i], launches=self.k_launches[i], bytes=self.k_bytes[i],
                                        flops=self.k_flops[i]) for i, name in enumerate(KCLASSES)})


class TuneResult(C.Structure):
    _fields_ = [("big_ns", C.c_int32), ("big_ns_bwd", C.c_int32), ("ms", C.c_double), ("from_cache", C.c_int32)]


class LevelDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("nnz_u", C.c_int64), ("fronts", C.c_int64),
                ("tree_levels", C.c_int64), ("factor_entries", C.c_int64), ("rho", C.c_double),
                ("factor_flops", C.c_double), ("factor_nnz", C.c_int64), ("qpanel_tree_levels", C.c_int64),
                ("qpanel_entries", C.c_int64)]


STATUS = {0: "HSIM_OK", -1: "HSIM_E_INVALID", -2: "HSIM_E_MESH", -3: "HSIM_E_FACTOR", -4: "HSIM_E_NOCONV",
          -5: "HSIM_E_NOMEM", -6: "HSIM_E_DEVICE", -7: "HSIM_E_STATE", -8: "HSIM_E_UNIMPLEMENTED"}

# symbol -> (restype, argtypes)
_P = C.c_void_p
_I32, _I64, _D = C.c_int32, C.c_int64, C.c_double
SIGNATURES = {
    "hsim_default_build_opts": (None, [C.POINTER(BuildOpts)]),
    "hsim_default_solve_opts": (None, [C.POINTER(SolveOpts)]),
    "hsim_build_hierarchy": (C.c_int, [_P, _I64, _P, _I64, _P, C.POINTER(BuildOpts), C.POINTER(_P)]),
    "hsim_solve": (C.c_int, [_P, C.POINTER(SolveOpts), _P, _P, _P, C.POINTER(Stats)]),
    "hsim_solve_backward": (C.c_int, [_P, _P, _P, _P, _P]),
    "hsim_free": (None, [_P]),
    "hsim_last_error": (C.c_char_p, []),
    "hsim_hierarchy_shape": (C.c_int, [_P, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32)]),
    "hsim_level_info": (C.c_int, [_P, _I32, C.POINTER(LevelDesc)]),
    "hsim_level_export": (C.c_int, [_P, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "hsim_step_prolong": (C.c_int, [_P, _I32, _I32, _P, _P, _P]),
    "hsim_step_apply": (C.c_int, [_P, _I32, _I32, _I32, _P, _P, _P]),
    "hsim_step_factor": (C.c_int, [_P, _I32, _D, _I32, C.POINTER(_I32), _P]),
    "hsim_step_solve": (C.c_int, [_P, _I32, _I32, _P, _P, _I32, _D, _P]),
    "hsim_step_gram": (C.c_int, [_P, _I32, _I32, _P, _P, _P, _I32, _P]),
    "hsim_step_rr": (C.c_int, [_I32, _P, _P, _P, _P, C.POINTER(_I32), _P]),
    "hsim_step_rr_noalloc": (C.c_int, [_I32, _P, _P, _P, _P, C.POINTER(_I32), _P]),
    "hsim_autotune": (C.c_int, [_P, _I32, _P, C.POINTER(TuneResult)]),
    "hsim_solve_batch": (C.c_int, [_P, _I32, C.POINTER(SolveOpts), _P, _P, _P, C.POINTER(Stats), _P, _I32]),
    "hsim_step_ritz": (C.c_int, [_P, _I32, _I32, _P, _P, _P, _D, _P, _P, _P]),
    "hsim_step_coarse": (C.c_int, [_P, _I32, _P, _P, C.POINTER(_I32), _P]),
}

_lib = None


def load():
    """Load libhsim.so (built in-tree by paper_2111_09039_amd.build); raises
    if it is missing -- there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2111_09039_amd.build.build() "
                          "(or __graft_entry__.build()) first")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HsimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def check(code):
    if code != 0:
        raise HsimError(code, load().hsim_last_error().decode(errors="replace"))
