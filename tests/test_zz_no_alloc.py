"""hsim_step_rr_noalloc (the allocation-free form of the reduced dense
eigenproblem, for callers that cannot allocate device memory) against
hsim_step_rr through the C ABI: two calls in a row, the second smaller, on
seeded symmetric / symmetric positive definite pencils; sizes beyond the
fixed work region are rejected."""
import ctypes as C

import numpy as np
import pytest
import scipy.linalg as sl

pytestmark = pytest.mark.gpu


def _pencil(k, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((k, k))
    M = B @ B.T / k + np.eye(k)
    A = rng.standard_normal((k, k))
    S = A + A.T
    return S, M


def _call(fn, k, S, M):
    import torch
    from paper_2111_09039_amd import _lib
    dS = torch.from_numpy(np.ascontiguousarray(S)).cuda()
    dM = torch.from_numpy(np.ascontiguousarray(M)).cuda()
    lam = torch.empty(k, dtype=torch.float64, device="cuda")
    Pb = torch.empty(k, k, dtype=torch.float64, device="cuda")
    sw = C.c_int32()
    code = getattr(_lib.load(), fn)(k, C.c_void_p(dS.data_ptr()), C.c_void_p(dM.data_ptr()),
                                    C.c_void_p(lam.data_ptr()), C.c_void_p(Pb.data_ptr()), C.byref(sw),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(code)
    return lam.cpu().numpy(), Pb.cpu().numpy(), sw.value


def test_noalloc_rr_matches_allocating_entry_point(cuda):
    for k, seed in ((200, 1), (120, 2), (256, 3), (7, 4)):
        S, M = _pencil(k, seed)
        l1, P1, s1 = _call("hsim_step_rr_noalloc", k, S, M)
        l0, P0, s0 = _call("hsim_step_rr", k, S, M)
        # the same kernels in the same order: equal results
        assert s1 == s0
        assert np.array_equal(l1, l0) and np.array_equal(P1, P0), k
        ref = sl.eigh(S, M, eigvals_only=True)
        assert np.abs(l1 - ref).max() <= 1e-10 * np.abs(ref).max(), k
        assert np.abs(P1.T @ M @ P1 - np.eye(k)).max() < 1e-10


def test_noalloc_rr_rejects_sizes_beyond_its_region(cuda):
    import torch
    from paper_2111_09039_amd import _lib
    lib = _lib.load()
    k = 257
    buf = torch.zeros(k * k, dtype=torch.float64, device="cuda")
    code = lib.hsim_step_rr_noalloc(k, C.c_void_p(buf.data_ptr()), C.c_void_p(buf.data_ptr()),
                                    C.c_void_p(buf.data_ptr()), C.c_void_p(buf.data_ptr()), None, None)
    assert _lib.STATUS[code] == "HSIM_E_INVALID"
    assert b"256" in lib.hsim_last_error()
