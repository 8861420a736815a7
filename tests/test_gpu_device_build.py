"""The device part of the hierarchy build (mesh checks, edge graph, farthest
point sampling; Algorithm 3) against the host build, through the C ABI.

The default build runs these steps on the GPU; HSIM_HOST_HIERARCHY=1 runs
them on the host (the code the host-only tests pin to the oracle).  Both must
give the same hierarchy bit for bit -- the same sample order, hence the same
levels, prolongations, Galerkin operators and elimination orders -- and the
same error for every invalid mesh.  The sampling's distances are the least
fixpoint of d(u) = min(d(u), d(v) + w(v, u)) in floating point, which the
device's parallel relaxation and the host's Dijkstra both reach, so equality
is exact, not approximate."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FIELDS = ("verts", "S_indptr", "S_indices", "S_data", "M_data", "U_indptr", "U_indices", "U_data", "perm")


def _build(monkeypatch, host, *args, **kw):
    import paper_2111_09039_amd as hs
    if host:
        monkeypatch.setenv("HSIM_HOST_HIERARCHY", "1")
    else:
        monkeypatch.delenv("HSIM_HOST_HIERARCHY", raising=False)
    return hs.Hierarchy(*args, **kw)


def _meshes():
    rng = np.random.default_rng(21)
    V, F = synth.icosphere(3)
    yield "sphere642", synth.radial_jitter(V, 1e-2, rng), F, None, {}, dict(p=24, levels=3, n_coarsest=120)
    V, F = synth.torus(60, 40)
    V = synth.isotropic_noise(V, F, 0.2 * synth.mean_edge_length(V, F), rng)
    yield "torus2400", V, F, synth.random_density(len(V), rng), {}, dict(p=20, levels=3, n_coarsest=200)
    V, F = synth.rectangle_grid(40, 30, 0.05)
    V = synth.isotropic_noise(V, F, 0.2 * synth.mean_edge_length(V, F), rng)
    yield "sheet1200", V, F, None, dict(boundary="dirichlet"), dict(p=10, levels=2, n_coarsest=150)
    V, F, d = synth.config_mesh("torus100k", seed=0)
    yield "torus100k", V, F, d, {}, dict(p=100, levels=5)


@pytest.mark.parametrize("case", list(_meshes()), ids=lambda c: c[0])
def test_device_build_equals_host(cuda, monkeypatch, case):
    name, V, F, d, extra, shape = case
    p = shape.pop("p")
    Hd = _build(monkeypatch, False, V, F, p, density=d, **shape, **extra)
    Hh = _build(monkeypatch, True, V, F, p, density=d, **shape, **extra)
    assert Hd.levels == Hh.levels
    for t in range(Hd.levels):
        ed, eh = Hd.export(t), Hh.export(t)
        for k in FIELDS:
            if k in ed and ed[k] is not None:
                assert np.array_equal(ed[k], eh[k]), (name, t, k)
    print(f"[{name}] {Hd.levels} levels equal bit for bit, sizes {[Hd.level_info(t)['n'] for t in range(Hd.levels)]}",
          flush=True)


def _bad_meshes():
    V, F = synth.icosphere(2)
    V = V.copy()
    F = F.copy()
    a = V.copy()
    a[7, 1] = np.nan
    yield "nonfinite", a, F
    f = F.copy()
    f[5, 2] = len(V) + 3
    yield "index-range", V, f
    f = F.copy()
    f[9, 1] = f[9, 0]
    yield "repeated", V, f
    yield "unused", np.vstack([V, [[2.0, 0.0, 0.0]]]), F
    a = V.copy()
    a[F[11, 2]] = 0.5 * (a[F[11, 0]] + a[F[11, 1]])   # collinear corners
    yield "degenerate", a, F
    x = next(int(v) for v in F[20] if v not in F[3])   # a third triangle on the edge (F[3, 0], F[3, 1])
    yield "non-manifold", V, np.vstack([F, [[F[3, 0], F[3, 1], x]]]).astype(np.int32)
    V2, F2 = synth.icosphere(1)
    yield "disconnected", np.vstack([V, V2 + 5.0]), np.vstack([F, F2 + len(V)])


@pytest.mark.parametrize("case", list(_bad_meshes()), ids=lambda c: c[0])
def test_device_build_errors_match_host(cuda, monkeypatch, case):
    from paper_2111_09039_amd import _lib
    name, V, F = case
    msgs = []
    for host in (False, True):
        with pytest.raises(_lib.HsimError) as e:
            _build(monkeypatch, host, V, F, 8, levels=2, n_coarsest=40)
        msgs.append((e.value.code, str(e.value)))
    print(f"[{name}] {msgs[0]}", flush=True)
    assert msgs[0] == msgs[1], msgs
    assert msgs[0][0] == -2
