"""Host-side logic without a GPU: the synthetic workloads have the sizes and distributions
they stand for, and the benchmark's byte model and profile bookkeeping behave as stated.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

from paper_2102_06248_amd import inputs, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    from paper_2102_06248_amd import fepic
    if not os.path.exists(fepic.LIB_PATH):
        from paper_2102_06248_amd import build
        build.build()
    return fepic


def _sizes(F, xyz, tets):
    ctx = F.fepic_create(device=-1)
    try:
        F.fepic_upload_mesh(ctx, xyz, tets)
        return F.fepic_get_topology_sizes(ctx)
    finally:
        F.fepic_destroy(ctx)


def test_beam_mesh_sizes(F):
    wl = workloads.c2_beam(n_particles=10)
    assert len(wl["tets"]) == 202_176
    s = _sizes(F, wl["xyz"], wl["tets"])
    assert (s["n_edges"], s["n_int_edges"], s["n_faces"]) == (245_706, 226_266, 410_832)
    assert len(wl["xyz"]) == 37_051


def test_kuhn_mesh_sizes_closed_form(F):
    # n^3 cubes x 6 tets; nodes (n+1)^3; edges 3n(n+1)^2 axis + 3n^2(n+1) face + n^3 body diagonals
    for n in (6, 13):
        xyz, tets = inputs.kuhn_cube(n)
        s = _sizes(F, xyz, tets)
        assert len(tets) == 6 * n ** 3 and len(xyz) == (n + 1) ** 3
        assert s["n_edges"] == 3 * n * (n + 1) ** 2 + 3 * n ** 2 * (n + 1) + n ** 3
        assert s["n_faces"] == 12 * n ** 3 + 6 * n ** 2   # 4T = 2 F_int + F_bnd, F_bnd = 12 n^2
        assert len(xyz) - s["n_edges"] + s["n_faces"] - len(tets) == 1


def test_beam_particles_distribution():
    from oracle.constants import C_LIGHT, M_E, Q_E
    x, u = inputs.beam_particles(200_000, 0.01, 0.0, 0.5, 1000.0, 1.0, M_E, seed=3)
    r = np.hypot(x[:, 0], x[:, 1])
    assert r.max() <= 0.01 and 0.0 <= x[:, 2].min() and x[:, 2].max() < 0.5
    # uniform on the disk: P(r <= R/2) = 1/4
    assert abs(np.mean(r <= 0.005) - 0.25) < 0.01
    gam = np.sqrt(1 + np.sum(u * u, axis=1) / C_LIGHT ** 2)
    v = u / gam[:, None]
    ke = np.mean((gam - 1) * M_E * C_LIGHT ** 2) / Q_E
    assert ke == pytest.approx(1000.0, rel=0.01)
    sig = math.sqrt(Q_E / M_E)   # 1 eV
    assert np.std(v[:, 0]) == pytest.approx(sig, rel=0.01)


def test_plasma_pairs_distribution():
    from oracle.constants import M_E
    m_p = inputs.PROTON_ELECTRON_MASS_RATIO * M_E
    x, ue, ui = inputs.gaussian_ball_pairs(100_000, 0.01, 3.9, 1.0, 0.1, M_E, m_p, seed=4)
    rr = np.linalg.norm(x, axis=1)
    assert rr.max() <= 0.039
    assert np.std(x[:, 1]) == pytest.approx(0.01, rel=0.02)
    assert np.std(ue[:, 2]) == pytest.approx(inputs.thermal_sigma_v(1.0, M_E), rel=0.02)
    assert np.std(ui[:, 0]) == pytest.approx(inputs.thermal_sigma_v(0.1, m_p), rel=0.02)


def test_plasma_weight_and_step():
    wl = workloads.c3_plasma(n_pairs=1000, n_cells=4)
    eps0, q, me = 8.8541878128e-12, inputs.ELEMENTARY_CHARGE, inputs.ELECTRON_MASS
    wpe = math.sqrt(2.5e13 * q * q / (eps0 * me))
    assert wl["dt"] == pytest.approx(0.05 / wpe, rel=1e-12)
    total = 2.5e13 * (2 * math.pi) ** 1.5 * 0.01 ** 3
    assert wl["species"][0]["w"] * 1000 == pytest.approx(total, rel=1e-12)


def test_bench_byte_model_and_profile_bookkeeping(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    geo = {"n_rows": 100, "nnz": 1500, "n_edges": 100, "n_faces": 180, "n_tets": 60, "n_int_edges": 70,
           "n_aux": 12}
    st = {"particles": 1000, "occupied_tets": 40, "crossings": 300}
    assert bench.algorithmic_bytes("cg_iter", geo, st, "jacobi") == 12 * 1500 + 80 * 100
    assert bench.algorithmic_bytes("cg_iter", geo, st, "aux") == 12 * 1500 + 144 * 100 + 8 * 70 + 96 * 12
    # FP32 inner iterations of the mixed-precision solve: 4 B values and vectors, the same
    # column ids, incidences, FP16 edge vectors and ends
    assert bench.algorithmic_bytes("cg_iter", geo, st, "aux", "mixed") == 8 * 1500 + 84 * 100 + 8 * 70 + 48 * 12
    # with far levels, their fold reads and writes each node's Y once more
    far = dict(geo, far_levels=2)
    assert bench.algorithmic_bytes("cg_iter", far, st, "aux") == 12 * 1500 + 144 * 100 + 8 * 70 + 160 * 12
    assert bench.algorithmic_bytes("cg_iter", far, st, "aux", "mixed") == 8 * 1500 + 84 * 100 + 8 * 70 + 80 * 12
    assert bench.profile_key("cg_iter", "aux", "mixed") == "cg_iter_mixed"
    assert bench.profile_key("cg_iter", "jacobi") == "cg_iter_jacobi"
    assert bench.profile_key("push", "aux", "mixed") == "push"
    # the particle step's per-unit bytes: 56 per particle (104 all-FP64), 284 per occupied
    # tet, 164 per crossing
    assert bench.algorithmic_bytes("push", geo, st) == 56 * 1000 + 284 * 40 + 164 * 300
    assert bench.algorithmic_bytes("push", geo, st, precision=1) == 104 * 1000 + 284 * 40 + 164 * 300
    # counter summaries are used only while the kernel source is unchanged
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    src_dir = tmp_path / "paper_2102_06248_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (src_dir / "kernels_fields.hip").write_text("kernel v1")
    rec = {"source_sha1": bench.source_hash("cg_iter"), "hbm_bytes_per_launch": 123456}
    (tmp_path / "profiles" / "cg_iter_c2_beam_counters.json").write_text(json.dumps(rec))
    assert bench.traffic_from_profile("cg_iter", "c2_beam") == 123456
    assert bench.traffic_from_profile("cg_iter", "c2_beam", "jacobi") is None   # its own summary
    assert bench.traffic_from_profile("cg_iter", "c2_beam", "aux", "mixed") is None
    (src_dir / "kernels_fields.hip").write_text("kernel v2")
    assert bench.traffic_from_profile("cg_iter", "c2_beam") is None
    assert bench.traffic_from_profile("cg_iter", "c3_plasma") is None


def test_solve_precision_options(F):
    """The mixed-precision solve is an option of the auxiliary-space preconditioner only;
    its inner tolerance lies in (0, 1); the setters keep the pair consistent."""
    o = F.fepic_default_options()
    assert o.solve_precision == F.FEPIC_SOLVE_FP64 and o.mixed_inner_tol == 1e-4
    for bad in ({"solve_precision": F.FEPIC_SOLVE_MIXED, "preconditioner": F.FEPIC_PC_JACOBI},
                {"solve_precision": 2}, {"solve_precision": F.FEPIC_SOLVE_MIXED, "mixed_inner_tol": 1.0},
                {"solve_precision": F.FEPIC_SOLVE_MIXED, "mixed_inner_tol": 0.0}):
        with pytest.raises(F.FepicError) as ei:
            F.fepic_create(device=-1, **bad)
        assert F.ERROR_NAMES[ei.value.code] == "FEPIC_E_ARG"
    ctx = F.fepic_create(device=-1, solve_precision=F.FEPIC_SOLVE_MIXED)
    try:
        with pytest.raises(F.FepicError):
            F.fepic_set_preconditioner(ctx, F.FEPIC_PC_JACOBI)
        F.fepic_set_solve_precision(ctx, F.FEPIC_SOLVE_FP64)
        F.fepic_set_preconditioner(ctx, F.FEPIC_PC_JACOBI)
        with pytest.raises(F.FepicError):
            F.fepic_set_solve_precision(ctx, F.FEPIC_SOLVE_MIXED)
    finally:
        F.fepic_destroy(ctx)


def test_ab_byte_model():
    """Adams-Bashforth-k bytes per particle-step: the particle state both ways (tet, three
    barycentric coordinates, velocity: 52 B each), the k positions, k - 1 velocities and
    k - 1 accelerations the step reads, and the three new levels it writes."""
    import bench
    for k in range(1, 6):
        reads = 8 * 3 * (k + (k - 1) + (k - 1))
        assert bench.ab_bytes_per_particle_step(k) == 2 * 52 + reads + 8 * 9
    assert bench.ab_bytes_per_particle_step(4) == 416
    assert bench.ab_bytes_per_particle_step(2) == 272
    # the committed counter summary names the kernel source it was taken on
    d = json.load(open(os.path.join(os.path.dirname(__file__), "..", "profiles", "push_ab4_c3_plasma_counters.json")))
    assert d["source"] == "kernels_ab.hip" and len(d["source_sha1"]) == 12 and d["hbm_bytes_per_launch"] > 0


def test_deterministic_option_checks(F):
    """The deterministic mode takes the Jacobi preconditioner, the FP64 solve and a warm
    start other than the learned one; the setters refuse to leave them."""
    assert F.fepic_default_options().deterministic == 0
    for bad in ({"deterministic": 1}, {"deterministic": 2, "preconditioner": F.FEPIC_PC_JACOBI},
                {"deterministic": 1, "preconditioner": F.FEPIC_PC_JACOBI, "warm_start": F.FEPIC_WS_MLP}):
        with pytest.raises(F.FepicError) as ei:
            F.fepic_create(device=-1, **bad)
        assert F.ERROR_NAMES[ei.value.code] == "FEPIC_E_ARG"
    ctx = F.fepic_create(device=-1, deterministic=1, preconditioner=F.FEPIC_PC_JACOBI)
    try:
        for call in (lambda: F.fepic_set_preconditioner(ctx, F.FEPIC_PC_AUX),
                     lambda: F.fepic_set_warm_start(ctx, F.FEPIC_WS_MLP),
                     lambda: F.fepic_set_solve_precision(ctx, F.FEPIC_SOLVE_MIXED)):
            with pytest.raises(F.FepicError):
                call()
        F.fepic_set_warm_start(ctx, F.FEPIC_WS_EXTRAP1)
    finally:
        F.fepic_destroy(ctx)


def test_sort_period_option_checks(F):
    """sort_period: a period >= 0, or FEPIC_SORT_AUTO (each species by its own need);
    other negative values are refused."""
    for bad in (-2, -64):
        with pytest.raises(F.FepicError):
            F.fepic_create(device=-1, sort_period=bad)
    for ok in (F.FEPIC_SORT_AUTO, 0, 1, 7):
        F.fepic_destroy(F.fepic_create(device=-1, sort_period=ok))
