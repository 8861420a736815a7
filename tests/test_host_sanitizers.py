"""The library's host hierarchy code (mesh.cpp, hierarchy.cpp, order.cpp)
built with AddressSanitizer and UndefinedBehaviorSanitizer (g++, no HIP) and
run on closed meshes, a mesh with boundary and a noisy mesh; any invalid
memory access or undefined behaviour aborts the driver.  Its printed
invariants are checked against the oracle's independent assembly."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import synth
from oracle import assembly

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2111_09039_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "hsim_host_asan")
    srcs = [os.path.join(HERE, "host_asan_driver.cpp")] + [os.path.join(CSRC, s) for s in
                                                          ("mesh.cpp", "hierarchy.cpp", "order.cpp")]
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"),
           *srcs, "-o", out]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    assert r.returncode == 0, r.stdout
    return out


def run(driver, tmp_path, V, F, p, T, nc, boundary=0):
    path = str(tmp_path / "mesh.bin")
    with open(path, "wb") as f:
        f.write(struct.pack("<qqiiqi", len(V), len(F), p, T, nc, boundary))
        f.write(np.ascontiguousarray(V, dtype="<f8").tobytes())
        f.write(np.ascontiguousarray(F, dtype="<i4").tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run([driver, path], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=600,
                       env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    out = {}
    for line in r.stdout.splitlines():
        k, *v = line.split()
        out.setdefault(k, []).append(v)
    return out


@pytest.mark.parametrize("name", ["sphere", "torus", "sheet"])
def test_host_build_under_sanitizers(driver, tmp_path, name):
    rng = np.random.default_rng(3)
    if name == "sphere":
        V, F, _ = synth.config_mesh("sphere2k", seed=0)
        T, nc = 3, 300
    elif name == "torus":
        V, F = synth.torus(60, 30)
        V = synth.isotropic_noise(V, F, 0.2 * synth.mean_edge_length(V, F), rng)
        T, nc = 3, 200
    else:
        V, F = synth.rectangle_grid(40, 30, 1.0 / 40)
        V = synth.isotropic_noise(V, F, 0.2 * synth.mean_edge_length(V, F), rng)
        T, nc = 2, 150
    out = run(driver, tmp_path, V, F, 10, T, nc)
    assert out["ok"] == [[]]
    # the device assembly's index structures reproduce the host assembly term for term
    assert out["assembly_maps_match"] == [["1"]]
    S, m = assembly.assemble(V, F)
    assert int(out["S_nnz"][0][0]) == S.nnz
    assert float(out["S_max_abs_rowsum"][0][0]) < 1e-12
    assert abs(float(out["mass_sum"][0][0]) - m.sum()) < 1e-12 * m.sum()
    nb = int(out["boundary_vertices"][0][0])
    assert nb == int(assembly.boundary_vertices(F, len(V)).sum())
    for lv in out["level"]:
        assert float(lv[lv.index("partition_of_unity") + 1]) < 1e-12
    for gl in out["galerkin"]:
        # 1^T U^T M U 1 = 1^T M 1 (partition of unity): the coarse mass keeps the area
        assert abs(float(gl[gl.index("mass_total") + 1]) - m.sum()) < 1e-10 * m.sum()


def test_invalid_mesh_is_an_error_under_sanitizers(driver, tmp_path):
    V, F = synth.icosphere(2)
    F = F.copy()
    F[5] = F[5][[0, 0, 1]]          # degenerate triangle (repeated vertex)
    path = str(tmp_path / "bad.bin")
    with open(path, "wb") as f:
        f.write(struct.pack("<qqiiqi", len(V), len(F), 10, 2, 60, 0))
        f.write(np.ascontiguousarray(V, dtype="<f8").tobytes())
        f.write(np.ascontiguousarray(F, dtype="<i4").tobytes())
    r = subprocess.run([driver, path], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 3 and r.stdout.startswith("error -2"), r.stdout + r.stderr
