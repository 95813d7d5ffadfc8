"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two programs are built in a temporary directory and must run without a sanitizer report:
* the library's host-side mesh build (host_mesh.cpp: canonical topology, geometry,
  assembly, the auxiliary space's node order, the point-location grid) on a distorted
  Kuhn mesh, a prism cylinder and three invalid meshes that must be rejected;
* the oracle's C particle loop (particles.c: gather, Boris, walk, deposit) pushing
  particles through a distorted mesh with paths aimed at vertices and edges, and through
  the wall.
Mesh arrays are written by Python to raw files that the programs read.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.mesh import Mesh
from paper_2102_06248_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_06248_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

HOST_DRIVER = r"""
#include "host_mesh.h"
#include <cstdio>
#include <vector>
template <typename T> static std::vector<T> slurp(const char* path) {
    std::vector<T> v;
    FILE* f = std::fopen(path, "rb");
    if (!f) return v;
    std::fseek(f, 0, SEEK_END);
    long n = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    v.resize(n / sizeof(T));
    if (std::fread(v.data(), sizeof(T), v.size(), f) != v.size()) v.clear();
    std::fclose(f);
    return v;
}
int main(int argc, char** argv) {
    // argv: pairs of (xyz file, tets file); prints rc and entity counts per mesh
    for (int i = 1; i + 1 < argc; i += 2) {
        std::vector<double> xyz = slurp<double>(argv[i]);
        std::vector<int32_t> tets = slurp<int32_t>(argv[i + 1]);
        fepic::HostMesh m;
        std::string err;
        int rc = fepic::build_host_mesh(m, (int64_t)xyz.size() / 3, xyz.data(), (int64_t)tets.size() / 4,
                                        tets.data(), err);
        std::printf("%d %lld %lld %lld %lld\n", rc, (long long)m.n_edges, (long long)m.n_faces,
                    (long long)m.n_int_edges, (long long)m.n_aux);
    }
    return 0;
}
"""

ORACLE_DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
typedef struct { int64_t n_tets; const double *xyz; const int64_t *tets, *tet_edges, *tet_faces, *nbr;
                 const double *grad; } orc_mesh;
typedef struct { int64_t n_crossings, max_crossings, n_absorbed, n_cap_exceeded; } orc_push_stats;
int orc_push(const orc_mesh*, int64_t, double*, double*, int64_t*, int8_t*, double, double, double, double,
             const double*, const double*, double*, int, orc_push_stats*);
static void* slurp(const char* path, long* n) {
    FILE* f = fopen(path, "rb");
    if (!f) exit(3);
    fseek(f, 0, SEEK_END);
    *n = ftell(f);
    fseek(f, 0, SEEK_SET);
    void* p = malloc(*n);
    if (fread(p, 1, *n, f) != (size_t)*n) exit(4);
    fclose(f);
    return p;
}
int main(int argc, char** argv) {
    long n[12];
    void* a[12];
    if (argc < 13) return 2;
    for (int i = 0; i < 12; i++) a[i] = slurp(argv[1 + i], &n[i]);
    orc_mesh m = {n[1] / 32, a[0], a[1], a[2], a[3], a[4], a[5]};
    int64_t np = n[7] / 8;
    orc_push_stats st;
    memset(&st, 0, sizeof(st));
    int rc = orc_push(&m, np, a[6], a[8], a[7], a[9], -1.602176634e-19, 9.1093837015e-31, 1.0, 1e-9,
                      a[10], a[11], calloc(n[10] / 8, 8), 64, &st);
    printf("%d %lld %lld\n", rc, (long long)st.n_crossings, (long long)st.n_absorbed);
    return 0;
}
"""


def _have(path):
    return os.path.exists(path) or shutil.which(path) is not None


@pytest.mark.skipif(not _have(CLANG), reason="clang++ not found")
def test_host_mesh_build_is_clean_under_asan_ubsan(tmp_path):
    drv = tmp_path / "drv.cpp"
    drv.write_text(HOST_DRIVER)
    exe = tmp_path / "host_mesh_san"
    subprocess.check_call([CLANG, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC] + SAN
                          + [os.path.join(CSRC, "host_mesh.cpp"), str(drv), "-o", str(exe)])
    meshes = []
    xyz, tets = inputs.kuhn_cube(4)
    meshes.append((inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(4), 0.25, 0.15, seed=2), tets))
    meshes.append(inputs.prism_cylinder(0.05, 0.2, 3, 4))
    bad_deg = (np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]], float), np.array([[0, 1, 2, 3]], np.int32))
    bad_id = (np.eye(4)[:, :3].copy(), np.array([[0, 1, 2, 7]], np.int32))
    x3 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 1]], float)
    bad_3 = (x3, np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]], np.int32))
    meshes += [bad_deg, bad_id, bad_3]
    args = []
    for k, (x, t) in enumerate(meshes):
        px, pt = tmp_path / f"x{k}.bin", tmp_path / f"t{k}.bin"
        np.ascontiguousarray(x, dtype=np.float64).tofile(px)
        np.ascontiguousarray(t, dtype=np.int32).tofile(pt)
        args += [str(px), str(pt)]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)] + args, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    rows = [list(map(int, ln.split())) for ln in r.stdout.strip().splitlines()]
    ref = Mesh(*meshes[0])
    assert rows[0][:3] == [0, ref.n_edges, ref.n_faces]
    assert rows[1][0] == 0
    assert all(row[0] != 0 for row in rows[2:])


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_particle_loop_is_clean_under_asan_ubsan(tmp_path):
    drv = tmp_path / "drv.c"
    drv.write_text(ORACLE_DRIVER)
    exe = tmp_path / "oracle_san"
    subprocess.check_call(["gcc", "-std=c99"] + SAN + [os.path.join(ROOT, "oracle", "particles.c"), str(drv),
                                                       "-lm", "-o", str(exe)])
    xyz, tets = inputs.kuhn_cube(3)
    m = Mesh(inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(3), 1 / 3, 0.15, seed=5), tets)
    rng = np.random.default_rng(3)
    n = 600
    t = rng.integers(m.n_tets, size=n)
    lam = rng.dirichlet(np.ones(4), size=n)
    x = np.einsum("pk,pkd->pd", lam, m.xyz[m.tets[t]])
    # a third of the particles head for a vertex or an edge midpoint of their tet
    aim = np.where(rng.random(n)[:, None] < 0.5, m.xyz[m.tets[t, 0]], 0.5 * (m.xyz[m.tets[t, 1]] + m.xyz[m.tets[t, 2]]))
    u = rng.normal(size=(n, 3)) * 2e8
    u[: n // 3] = (aim - x)[: n // 3] * 3e9
    e, b = rng.normal(size=m.n_edges) * 10, rng.normal(size=m.n_faces) * 1e-4
    arrs = [m.xyz, m.tets, m.tet_edges, m.tet_faces, m.nbr, m.grad_lambda, x, t.astype(np.int64), u,
            np.ones(n, np.int8), e, b]
    paths = []
    for k, a in enumerate(arrs):
        p = tmp_path / f"a{k}.bin"
        np.ascontiguousarray(a).tofile(p)
        paths.append(str(p))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)] + paths, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    rc, n_cross, n_abs = map(int, r.stdout.split())
    assert rc in (0, 1) and n_cross > 100 and n_abs > 0
