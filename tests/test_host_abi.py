"""The C ABI on the host (no GPU): the library loads and exports every
function that include/hsim.h declares, and the host part of the hierarchy
build (HSIM_BUILD_HOST_ONLY: mesh checks, assembly, level rules, the
Dirichlet restriction, prolongation, symbolic analysis; no device work)
agrees with the oracle's definitions."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import assembly, hierarchy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2111_09039_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib


def _declared():
    txt = open(os.path.join(ROOT, "include", "hsim.h")).read()
    return re.findall(r"^(?:hsim_status|void|const char\s*\*)\s*(hsim_\w+)\s*\(", txt, re.M)


def test_library_exports_every_declared_function(lib):
    names = _declared()
    assert len(names) >= 18, names
    so = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing
    # the Python binding marshals exactly the declared entry points
    assert set(names) == set(lib.SIGNATURES), set(names) ^ set(lib.SIGNATURES)


def test_host_build_rules_and_errors(lib):
    import paper_2111_09039_amd as hs
    V, F = synth.icosphere(3)
    H = hs.Hierarchy(V, F, 24, levels=3, n_coarsest=120, host_only=True)
    assert (H.levels, H.q) == (3, 36)
    sizes = [H.level_info(t)["n"] for t in range(3)]
    assert sizes == list(hierarchy.level_sizes(len(V), 3, 120)), sizes
    assert np.array_equal(H.export(0)["verts"], np.arange(len(V)))
    with pytest.raises(lib.HsimError) as e:
        hs.Hierarchy(V, F, 0, host_only=True)
    assert e.value.code == -1
    with pytest.raises(lib.HsimError):
        hs.Hierarchy(V, F, 24, levels=3, n_coarsest=20, host_only=True)   # coarsest below q
    with pytest.raises(ValueError):
        hs.Hierarchy(V, F, 24, host_only=True, boundary="robin")
    Fbad = F.copy()
    Fbad[0, 1] = Fbad[0, 0]
    with pytest.raises(lib.HsimError) as e:
        hs.Hierarchy(V, Fbad, 24, host_only=True)
    assert e.value.code == -2


def test_host_build_dirichlet_restriction(lib):
    import paper_2111_09039_amd as hs
    rng = np.random.default_rng(4)
    V, F = synth.rectangle_grid(30, 20, 0.1)
    V = synth.isotropic_noise(V, F, 0.2 * synth.mean_edge_length(V, F), rng)
    S, m = assembly.assemble(V, F)
    Si, mi, interior = assembly.dirichlet(S, m, F)
    H = hs.Hierarchy(V, F, 10, levels=3, n_coarsest=120, host_only=True, boundary="dirichlet")
    n0 = len(interior)
    assert H.level_info(0)["n"] == n0 == 28 * 18
    e = H.export(0)
    assert np.array_equal(e["verts"], interior)
    S0 = sp.csr_matrix((e["S_data"], e["S_indices"], e["S_indptr"]), shape=(n0, n0))
    assert abs(S0 - Si).max() <= 1e-12 * abs(Si).max()
    M0 = sp.csr_matrix((e["M_data"], e["S_indices"], e["S_indptr"]), shape=(n0, n0))
    assert np.abs(M0.diagonal() - mi).max() <= 1e-14 * mi.max()
    n1 = H.level_info(1)["n"]
    U = sp.csr_matrix((e["U_data"], e["U_indices"], e["U_indptr"]), shape=(n0, n1))
    assert np.all(np.diff(U.indptr) > 0) and np.all(U.getnnz(axis=0) > 0)
    # without the option the boundary stays in (natural condition)
    Hn = hs.Hierarchy(V, F, 10, levels=3, n_coarsest=120, host_only=True)
    assert Hn.level_info(0)["n"] == len(V)
