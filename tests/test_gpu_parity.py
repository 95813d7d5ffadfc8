"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on the same
seeded inputs.  Tolerances (from the precision each mode computes in):

* ALL_FP64: positions and momenta to 1e-10 relative; deposits to 1e-10 of their max.
* FP32 push / FP64 deposit: positions within 1e-5 of the element size (FP32 barycentric
  storage is ~6e-8 h); momenta 1e-5 relative; deposits within 1e-5 of their max (FP32
  displacement, ~1e-7, accumulated over a step's crossings).
* Fields after a Newmark step: 1e-6 relative (both solves stop at ||r|| <= 1e-10 ||b||;
  the FP32 push perturbs the source at ~1e-7).
* Charge continuity from the library's own diagnostics: 1e-12 relative, every step.
"""
import math

import numpy as np
import pytest

from gpu_common import (announce, compare_particles, divfree_fields, have_gpu, jittered_kuhn, require_lib)
from oracle.constants import C_LIGHT, M_E, Q_E
from oracle.pic import OracleSim
from paper_2102_06248_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    if not have_gpu():
        pytest.fail("GPU tests need an MI355X")
    return require_lib()


def _lib_sim(F, xyz, tets, **opts):
    return F.Simulation(xyz, tets, **opts)


# ----------------------------------------------------------------------------- one push
@pytest.mark.parametrize("precision,n,walk", [(1, 4099, "queue"), (1, 4099, "fused"), (0, 4099, "queue"),
                                              (0, 4099, "fused"), (0, 70001, "queue"), (0, 70001, "fused")])
def test_particle_step_vs_oracle(F, precision, n, walk):
    """One particle step against the oracle, with the crossing paths finished from the
    queue by a second kernel or in place by the first."""
    announce(f"particle step precision={precision} n={n} walk={walk}")
    xyz, tets, h = jittered_kuhn(6)
    osim = OracleSim(xyz, tets)
    e, b = divfree_fields(osim, 50.0, 1e-4, [0.0, 0.0, 0.002], seed=1)
    x, u = inputs.uniform_box_particles(n, [0.02] * 3, [0.98] * 3, 3e6, seed=2)
    qw = -Q_E * 1e3
    s = osim.add_species(-Q_E, M_E, 1e3)
    assert osim.upload_particles(s, x, u, ids=np.arange(n)) == 0
    osim.e, osim.b = e.copy(), b.copy()
    dt = 2e-8
    mode = F.FEPIC_WALK_QUEUE if walk == "queue" else F.FEPIC_WALK_FUSED
    with _lib_sim(F, xyz, tets, precision=precision, walk=mode) as L:
        F.fepic_set_fields(L.ctx, e=e, e_prev=e, b=b)
        sp = F.fepic_add_species(L.ctx, -Q_E, M_E, 1e3)
        assert F.fepic_upload_particles(L.ctx, sp, x, u, ids=np.arange(n)) == 0
        g0 = F.fepic_get_particles(L.ctx, sp)
        # upload locates every particle in the same tet as the oracle
        o0 = osim.particles(s)
        oi = np.argsort(o0["id"])
        gi = np.argsort(g0["id"])
        assert np.array_equal(g0["tet"][gi], o0["tet"][oi])
        st = F.fepic_push_particles(L.ctx, dt)
        gp = F.fepic_get_particles(L.ctx, sp)
        dg_gpu, _ = F.fepic_get_current(L.ctx)
        # the live count (absorbed particles stay in the arrays until the next sort)
        n_live = F.fepic_num_particles(L.ctx, sp)
    assert n_live == len(gp["id"]) == n - st.n_absorbed
    ost = osim.step(dt, solve=False)
    op = osim.particles(s)
    tol = (1e-10, 1e-10) if precision == 1 else (1e-5, 1e-5)
    ncommon, nodd = compare_particles(gp, op, h, *tol)
    assert nodd <= max(1, n // 2000)
    assert ncommon > 0.9 * n
    assert st.n_crossings == pytest.approx(ost["n_crossings"], rel=0.01, abs=3)
    assert st.n_absorbed == pytest.approx(ost["n_absorbed"], abs=max(1, n // 2000))
    dg_orc = osim.dG
    dtol = 1e-10 if precision == 1 else 1e-5
    if nodd:
        # a few particles were absorbed on one side only (FP32 rounding at a wall): push the
        # particles both sides agree on again, on both sides, and compare their current
        alive_g = set(gp["id"].tolist())
        alive_o = set(op["id"].tolist())
        keep = np.array(sorted(set(range(n)) - (alive_g ^ alive_o)))
        osim = OracleSim(xyz, tets)
        s = osim.add_species(-Q_E, M_E, 1e3)
        osim.upload_particles(s, x[keep], u[keep], ids=keep)
        osim.e, osim.b = e.copy(), b.copy()
        osim.step(dt, solve=False)
        dg_orc = osim.dG
        with _lib_sim(F, xyz, tets, precision=precision, walk=mode) as L:
            F.fepic_set_fields(L.ctx, e=e, e_prev=e, b=b)
            sp = F.fepic_add_species(L.ctx, -Q_E, M_E, 1e3)
            F.fepic_upload_particles(L.ctx, sp, x[keep], u[keep], ids=keep)
            F.fepic_push_particles(L.ctx, dt)
            dg_gpu, _ = F.fepic_get_current(L.ctx)
            gp2 = F.fepic_get_particles(L.ctx, sp)
        _, nodd2 = compare_particles(gp2, osim.particles(s), h, *tol)
        assert nodd2 == 0
    scale = np.abs(dg_orc).max()
    assert np.max(np.abs(dg_gpu - dg_orc)) <= dtol * scale
    # particles come back sorted by tet (the sort runs at upload)
    assert np.all(np.diff(g0["tet"]) >= 0)


@pytest.mark.parametrize("precision", [1, 0])
def test_rarely_crossing_species_vs_oracle(F, precision):
    """Slow particles (a few crossings per thousand particle-steps): after the first step
    the species' own crossing share is below 1/64, so its crossing paths are walked by the
    sparse form (resident one-wave workgroups visiting the non-empty queue regions).  Three
    steps, particles and current against the oracle after each."""
    announce(f"rarely crossing species precision={precision}")
    xyz, tets, h = jittered_kuhn(6)
    osim = OracleSim(xyz, tets)
    e, b = divfree_fields(osim, 50.0, 1e-4, [0.0, 0.0, 0.002], seed=3)
    n = 20000
    x, u = inputs.uniform_box_particles(n, [0.02] * 3, [0.98] * 3, 2.5e4, seed=4)
    s = osim.add_species(-Q_E, M_E, 1e3)
    assert osim.upload_particles(s, x, u, ids=np.arange(n)) == 0
    osim.e, osim.b = e.copy(), b.copy()
    dt = 2e-9          # the field's kick dominates: a few tens of crossings per step
    tol = (1e-10, 1e-10) if precision == 1 else (1e-5, 1e-5)
    dtol = 1e-10 if precision == 1 else 1e-5
    with _lib_sim(F, xyz, tets, precision=precision, walk=F.FEPIC_WALK_QUEUE) as L:
        F.fepic_set_fields(L.ctx, e=e, e_prev=e, b=b)
        sp = F.fepic_add_species(L.ctx, -Q_E, M_E, 1e3)
        assert F.fepic_upload_particles(L.ctx, sp, x, u, ids=np.arange(n)) == 0
        for k in range(3):
            st = F.fepic_push_particles(L.ctx, dt)
            # the library's particle-only push keeps the fields; the oracle's step without a
            # solve would still advance b by Faraday's law, so its fields are put back
            osim.e, osim.e_prev, osim.b = e.copy(), e.copy(), b.copy()
            ost = osim.step(dt, solve=False)
            assert 0 < st.n_crossings < n / 64, st.n_crossings
            assert st.n_crossings == pytest.approx(ost["n_crossings"], rel=0.01, abs=3), k
            gp = F.fepic_get_particles(L.ctx, sp)
            ncommon, nodd = compare_particles(gp, osim.particles(s), h, *tol)
            assert nodd == 0 and ncommon == n - st.n_absorbed, k
            dg_gpu, _ = F.fepic_get_current(L.ctx)
            scale = np.abs(osim.dG).max()
            assert np.max(np.abs(dg_gpu - osim.dG)) <= dtol * scale, k
    print(f"\n[rarely crossing p{precision}] {st.n_crossings} crossings of {n} particles in the last step")


@pytest.mark.parametrize("pusher", ["boris", "ab"])
def test_automatic_sort_schedule(F, pusher):
    """FEPIC_SORT_AUTO re-bins a species only when a 64th of its particles left their tet
    since its last re-binning: over six pushes of a fast and a slow species the slow one is
    re-binned less often than every step, and particles and current equal those of
    re-binning every step (to rounding order).  With the Boris pusher and with the
    Adams-Bashforth one, whose histories move with the particles when they are re-binned."""
    announce(f"automatic sort schedule, {pusher}")
    xyz, tets, h = jittered_kuhn(6)
    osim = OracleSim(xyz, tets)
    e, b = divfree_fields(osim, 50.0, 1e-4, [0.0, 0.0, 0.002], seed=3)
    n = 20000
    xf, uf = inputs.uniform_box_particles(n, [0.02] * 3, [0.98] * 3, 3e6, seed=5)
    xs, us = inputs.uniform_box_particles(n, [0.02] * 3, [0.98] * 3, 2.5e4, seed=6)
    dt = 2e-9
    out = {}
    for period in (F.FEPIC_SORT_AUTO, 1):
        extra = dict(pusher=F.FEPIC_PUSHER_AB, ab_order=3) if pusher == "ab" else {}
        with _lib_sim(F, xyz, tets, precision=1, sort_period=period, timing=1, **extra) as L:
            F.fepic_set_fields(L.ctx, e=e, e_prev=e, b=b)
            sf = F.fepic_add_species(L.ctx, -Q_E, M_E, 1e3)
            ss = F.fepic_add_species(L.ctx, -Q_E, M_E, 1e3)
            F.fepic_upload_particles(L.ctx, sf, xf, uf, ids=np.arange(n))
            F.fepic_upload_particles(L.ctx, ss, xs, us, ids=np.arange(n))
            F.fepic_kernel_timing(L.ctx, "sort", 100)
            for _ in range(6):
                F.fepic_push_particles(L.ctx, dt)
            _, n_sorts = F.fepic_kernel_time(L.ctx, "sort")
            dG, G = F.fepic_get_current(L.ctx)
            out[period] = (n_sorts, G, F.fepic_get_particles(L.ctx, sf), F.fepic_get_particles(L.ctx, ss))
    n_auto, G_auto, pf_a, ps_a = out[F.FEPIC_SORT_AUTO]
    n_every, G_every, pf_e, ps_e = out[1]
    assert n_every == 12 and 1 <= n_auto < 12, (n_auto, n_every)
    assert np.abs(G_auto - G_every).max() <= 1e-12 * np.abs(G_every).max()
    for pa, pe in ((pf_a, pf_e), (ps_a, ps_e)):
        ncommon, nodd = compare_particles(pa, pe, h, 1e-12, 1e-12)
        assert nodd == 0 and ncommon == len(pe["id"])
    print(f"\n[automatic sort, {pusher}] {n_auto} re-binnings in 6 steps of two species (12 when every step)")


def test_gather_uniform_fields_exact(F):
    """A uniform E0 is reproduced exactly by the Whitney-1 interpolant, so one push from
    rest with B = 0 gives the closed-form Boris update u = (q dt / m) E0."""
    announce("uniform-field gather")
    xyz, tets, h = jittered_kuhn(4)
    osim = OracleSim(xyz, tets)
    E0 = np.array([3e3, -1e3, 2e3])
    e = osim.mesh.edge_dofs_of_uniform_field(E0)
    e[osim.mesh.boundary_edge] = 0.0
    x, _ = inputs.uniform_box_particles(500, [0.2] * 3, [0.8] * 3, 0.0, seed=5)
    u = np.zeros_like(x)
    dt = 1e-12
    with _lib_sim(F, xyz, tets, precision=1) as L:
        # interior tets only see interior edges; boundary edges are zeroed by the library,
        # so keep particles in tets with no wall edge
        F.fepic_set_fields(L.ctx, e=e, e_prev=e)
        sp = F.fepic_add_species(L.ctx, -Q_E, M_E, 1.0)
        F.fepic_upload_particles(L.ctx, sp, x, u)
        F.fepic_push_particles(L.ctx, dt)
        gp = F.fepic_get_particles(L.ctx, sp)
    m = osim.mesh
    wall_tet = np.any(m.boundary_edge[m.tet_edges], axis=1)
    inner = ~wall_tet[m.locate(x)]
    ids = np.arange(len(x))[inner]
    sel = np.isin(gp["id"], ids)
    expect = -Q_E * dt / M_E * E0
    assert np.allclose(gp["u"][sel], expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())


# ----------------------------------------------------------------------------- C1
def test_c1_single_electron_2000_steps_fp64(F):
    announce("C1: single electron, Kuhn 6x6x6, 2000 steps, all FP64")
    xyz, tets = inputs.kuhn_cube(6)
    B0, v0 = 0.1, 1e5
    gam = 1 / math.sqrt(1 - (v0 / C_LIGHT) ** 2)
    om = Q_E * B0 / (gam * M_E)
    dt = 2 * math.pi / om / 50
    rL = gam * M_E * v0 / (Q_E * B0)
    c = np.full(3, 5 / 12)
    x0, u0 = [c + [rL, 0, 0]], [[0, gam * v0, 0]]
    # Like for like with the oracle: Jacobi-PCG to ||r|| <= 1e-10 ||b|| on both sides.
    osim = OracleSim(xyz, tets, cg_tol=1e-10)
    osim.set_uniform_B([0, 0, B0])
    s = osim.add_species(-Q_E, M_E, 1.0)
    osim.upload_particles(s, x0, u0)
    osim.init_electrostatic()
    with _lib_sim(F, xyz, tets, precision=1, diagnostics=1, cg_tol=1e-10, preconditioner=F.FEPIC_PC_JACOBI) as L:
        F.fepic_set_uniform_B(L.ctx, [0, 0, B0])
        sp = F.fepic_add_species(L.ctx, -Q_E, M_E, 1.0)
        F.fepic_upload_particles(L.ctx, sp, x0, u0)
        F.fepic_init_electrostatic(L.ctx, 1e-14)
        e0, _, _ = F.fepic_get_fields(L.ctx)
        assert np.allclose(e0, osim.e, rtol=0, atol=1e-9 * np.abs(osim.e).max())
        worst = 0.0
        cont, drift, ncross, it_diff = 0.0, 0.0, 0, 0
        for n in range(2000):
            st = F.fepic_step(L.ctx, dt, 0.25, 0.5)
            ost = osim.step(dt, 0.25, 0.5)
            ncross += st.n_crossings
            it_diff = max(it_diff, abs(st.cg_iters - ost["cg_iters"]))
            cont = max(cont, st.cont_resid_rel)
            if st.gauss_drift_check_rel >= 0:
                drift = max(drift, st.gauss_drift_check_rel)
            if n % 50 == 0 or n == 1999:
                gp = F.fepic_get_particles(L.ctx, sp)
                worst = max(worst, np.max(np.abs(gp["x"][0] - osim.species[0].x[0])) / rL)
        e, _, b = F.fepic_get_fields(L.ctx)
    assert worst < 1e-7
    assert ncross > 200
    assert it_diff <= 1        # the same Jacobi-PCG on both sides: the same iteration counts
    assert cont < 1e-12
    assert drift < 1e-12
    assert np.linalg.norm(e - osim.e) <= 1e-6 * np.linalg.norm(osim.e)
    assert np.max(np.abs(b - osim.b)) <= 1e-12 * np.abs(osim.b).max()


# ----------------------------------------------------------------------------- full steps
@pytest.mark.parametrize("precision", [1, 0])
def test_beam_steps_fields_and_conservation(F, precision):
    announce(f"tiny beam, 12 full steps, precision={precision}")
    xyz, tets, h = jittered_kuhn(4, lo=(-0.02, -0.02, 0.0), hi=(0.02, 0.02, 0.04), seed=5)
    x, u = inputs.beam_particles(700, 0.008, 0.004, 0.03, 1000.0, 1.0, M_E, 5)
    osim = OracleSim(xyz, tets)
    s = osim.add_species(-Q_E, M_E, 5e4)
    osim.upload_particles(s, x, u, ids=np.arange(len(x)))
    osim.init_electrostatic()
    dt = 1e-10
    with _lib_sim(F, xyz, tets, precision=precision, diagnostics=1) as L:
        sp = F.fepic_add_species(L.ctx, -Q_E, M_E, 5e4)
        F.fepic_upload_particles(L.ctx, sp, x, u, ids=np.arange(len(x)))
        F.fepic_init_electrostatic(L.ctx, 1e-14)
        for n in range(12):
            st = F.fepic_step(L.ctx, dt, 0.25, 0.5)
            osim.step(dt, 0.25, 0.5)
            assert st.cont_resid_rel < 1e-12
            if st.gauss_drift_check_rel >= 0:
                assert st.gauss_drift_check_rel < 1e-12
            assert st.cg_rel_resid <= 1e-10 * 1.01
        e, ep, b = F.fepic_get_fields(L.ctx)
        dg, G = F.fepic_get_current(L.ctx)
        gp = F.fepic_get_particles(L.ctx, sp)
    # energies of the last step's diagnostics against the oracle's state (quadratic in the
    # fields, which agree to 1e-6)
    from oracle import diagnostics as odiag, fem
    o = osim.particles(s)
    w_e = 0.5 * float(osim.e @ (osim.M @ osim.e))
    w_b = odiag.magnetic_energy(fem.face_mass_matrix(osim.mesh), osim.b)
    w_k = odiag.kinetic_energy(o["u"], 5e4, M_E, C_LIGHT)
    assert st.field_energy == pytest.approx(w_e, rel=5e-6)
    assert st.magnetic_energy == pytest.approx(w_b, rel=5e-6, abs=1e-12 * w_e)
    assert st.kinetic_energy == pytest.approx(w_k, rel=5e-6)
    assert np.linalg.norm(e - osim.e) <= 1e-6 * np.linalg.norm(osim.e)
    assert np.linalg.norm(b - osim.b) <= 1e-6 * np.linalg.norm(osim.b) + 1e-30
    assert np.linalg.norm(G - osim.G) <= 1e-6 * np.linalg.norm(osim.G)
    tol = (1e-9, 1e-9) if precision == 1 else (1e-5, 1e-5)
    compare_particles(gp, osim.particles(s), h, *tol)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_newmark_solve_vs_oracle(F, mode):
    """No particles: the step is the Newmark update alone, from random e^n, e^{n-1}."""
    announce(f"Newmark solve, warm start {mode}")
    xyz, tets, h = jittered_kuhn(7, seed=9)
    osim = OracleSim(xyz, tets)
    rng = np.random.default_rng(4)
    e = rng.normal(size=osim.mesh.n_edges)
    ep = e + 0.01 * rng.normal(size=osim.mesh.n_edges)
    e[osim.mesh.boundary_edge] = ep[osim.mesh.boundary_edge] = 0.0
    b = osim.mesh.face_dofs_of_uniform_field([0.1, 0.0, 0.0])
    osim.e, osim.e_prev, osim.b = e.copy(), ep.copy(), b.copy()
    dt = 3e-10
    with _lib_sim(F, xyz, tets, precision=0, warm_start=mode) as L:
        F.fepic_set_fields(L.ctx, e=e, e_prev=ep, b=b)
        for _ in range(3):
            st = F.fepic_step(L.ctx, dt, 0.25, 0.5)
            osim.step(dt, 0.25, 0.5)
        eg, epg, bg = F.fepic_get_fields(L.ctx)
    assert st.cg_iters > 0
    assert np.linalg.norm(eg - osim.e) <= 1e-6 * np.linalg.norm(osim.e)
    assert np.linalg.norm(bg - osim.b) <= 1e-6 * np.linalg.norm(osim.b)


@pytest.mark.parametrize("pc,n,cfl_ratio,far", [("jacobi", 7, 4.0, -1), ("jacobi", 16, 20.0, -1), ("aux", 7, 4.0, -1),
                                                ("aux", 16, 8.0, -1), ("aux", 22, 20.0, -1), ("aux", 16, 20.0, 1),
                                                ("aux", 16, 40.0, 3)])
def test_preconditioned_cg_vs_oracle_pcg(F, pc, n, cfl_ratio, far):
    """One field-only step with each preconditioner: the library's iteration count matches
    the oracle's PCG with the same preconditioner (for the auxiliary space: the same
    aggregate levels, 8 and 64 nodes and as many of 512, 4096 as the library used) on the
    same right-hand side and start, within the spread that summation order gives, and the
    fields match the direct solve.  An auxiliary-space preconditioner with a wrong sign,
    scale, aggregate or asymmetry still converges, but not in the oracle's number of
    iterations.  far = -1 lets the library choose the far levels from dt; the choice is
    checked against the rule computed from the oracle's matrices."""
    from oracle import auxspace, newmark
    import scipy.sparse.linalg as spla
    announce(f"PCG {pc} on a {n}^3 Kuhn mesh, dt = {cfl_ratio} x the explicit limit, far levels {far}")
    xyz, tets, h = jittered_kuhn(n, seed=11)
    osim = OracleSim(xyz, tets)
    m = osim.mesh
    rng = np.random.default_rng(8)
    e = rng.normal(size=m.n_edges)
    ep = e + 0.05 * rng.normal(size=m.n_edges)
    e[m.boundary_edge] = ep[m.boundary_edge] = 0.0
    hmin = np.linalg.norm(m.xyz[m.edges[:, 1]] - m.xyz[m.edges[:, 0]], axis=1).min()
    dt = cfl_ratio * hmin / C_LIGHT
    ie = osim.ie
    A, B1, B2 = osim.operators(dt, 0.25, 0.5)
    rhs = newmark.newmark_rhs(B1, B2, e[ie], ep[ie], np.zeros(len(ie)))
    code = F.FEPIC_PC_AUX if pc == "aux" else F.FEPIC_PC_JACOBI
    with _lib_sim(F, xyz, tets, precision=0, preconditioner=code, cg_check_every=4, aux_far_levels=far) as L:
        F.fepic_set_fields(L.ctx, e=e, e_prev=ep)
        st = F.fepic_step(L.ctx, dt, 0.25, 0.5)
        eg, _, _ = F.fepic_get_fields(L.ctx)
    if pc == "aux":
        tau2 = np.mean(0.25 * dt * dt * osim.Si.diagonal() / osim.Mi.diagonal())
        n_aux = len(m.interior_nodes)
        rule = 0
        while rule < 3 and tau2 >= 4 * 2.0 ** (2 * (9 + 3 * rule) / 3) and n_aux >= 16 * 2 ** (9 + 3 * rule):
            rule += 1
        assert st.pc_far_levels == (rule if far < 0 else far)
        levels = (8, 64, 512, 4096, 32768)[:2 + st.pc_far_levels]
        x_o, it_o, _ = auxspace.pcg(A, rhs, e[ie], auxspace.aux_space_preconditioner(A, m, levels=levels)[0], tol=1e-10)
    else:
        assert st.pc_far_levels == -1
        levels = None
        x_o, it_o, _ = newmark.pcg_jacobi(A, rhs, e[ie], 1e-10)
    x_direct = spla.spsolve(A.tocsc(), rhs)
    # a residual of 1e-10 leaves an error of up to cond(A) 1e-10: the oracle's own PCG sets
    # the scale
    err_o = np.linalg.norm(x_o - x_direct)
    print(f"\n[pcg] {pc} n={n} levels {levels}: library {st.cg_iters} iterations, oracle {it_o}")
    assert abs(st.cg_iters - it_o) <= max(2, 0.03 * it_o)
    assert st.cg_rel_resid <= 1e-10
    assert np.linalg.norm(eg[ie] - x_direct) <= 10 * err_o + 1e-12 * np.linalg.norm(x_direct)
    assert np.abs(eg[m.boundary_edge]).max() == 0.0


@pytest.mark.parametrize("n,cfl_ratio,far", [(7, 4.0, -1), (16, 8.0, -1), (22, 20.0, -1), (16, 40.0, 3)])
def test_mixed_precision_solve_vs_oracle(F, n, cfl_ratio, far):
    """The mixed-precision solve (FP64 residuals, FP32 inner PCG from zero): the true FP64
    residual meets 1e-10, the fields are as close to the direct solve as the FP64 PCG's,
    and the passes and the total of inner iterations agree with the oracle's refinement
    with the same levels and inner tolerance (FP32 sums in another order move a few
    iterations)."""
    from oracle import auxspace, newmark
    import scipy.sparse.linalg as spla
    announce(f"mixed-precision PCG on a {n}^3 Kuhn mesh, dt = {cfl_ratio} x the explicit limit, far levels {far}")
    xyz, tets, h = jittered_kuhn(n, seed=11)
    osim = OracleSim(xyz, tets)
    m = osim.mesh
    rng = np.random.default_rng(8)
    e = rng.normal(size=m.n_edges)
    ep = e + 0.05 * rng.normal(size=m.n_edges)
    e[m.boundary_edge] = ep[m.boundary_edge] = 0.0
    hmin = np.linalg.norm(m.xyz[m.edges[:, 1]] - m.xyz[m.edges[:, 0]], axis=1).min()
    dt = cfl_ratio * hmin / C_LIGHT
    ie = osim.ie
    A, B1, B2 = osim.operators(dt, 0.25, 0.5)
    rhs = newmark.newmark_rhs(B1, B2, e[ie], ep[ie], np.zeros(len(ie)))
    with _lib_sim(F, xyz, tets, precision=0, preconditioner=F.FEPIC_PC_AUX, cg_check_every=4, aux_far_levels=far,
                  solve_precision=F.FEPIC_SOLVE_MIXED) as L:
        F.fepic_set_fields(L.ctx, e=e, e_prev=ep)
        st = F.fepic_step(L.ctx, dt, 0.25, 0.5)
        eg, _, _ = F.fepic_get_fields(L.ctx)
    levels = (8, 64, 512, 4096, 32768)[:2 + st.pc_far_levels]
    apply32 = auxspace.aux_space_preconditioner(A, m, levels=levels, dtype=np.float32)[0]
    _, it_m, passes_m, res_m = auxspace.pcg_refined(A, rhs, e[ie], apply32, tol=1e-10, inner_tol=1e-4)
    apply64 = auxspace.aux_space_preconditioner(A, m, levels=levels)[0]
    x_o, it_o, _ = auxspace.pcg(A, rhs, e[ie], apply64, tol=1e-10)
    x_direct = spla.spsolve(A.tocsc(), rhs)
    err_o = np.linalg.norm(x_o - x_direct)
    print(f"\n[mixed] n={n} levels {levels}: library {st.cg_iters} iterations in {st.cg_passes} passes, "
          f"oracle refinement {it_m} in {passes_m}, oracle FP64 PCG {it_o}")
    assert res_m <= 1e-10
    assert st.cg_rel_resid <= 1e-10
    assert abs(st.cg_passes - passes_m) <= 1 and st.cg_passes >= 1
    assert abs(st.cg_iters - it_m) <= max(4, 0.1 * it_m)
    assert np.linalg.norm(eg[ie] - x_direct) <= 10 * err_o + 1e-12 * np.linalg.norm(x_direct)
    assert np.abs(eg[m.boundary_edge]).max() == 0.0


def test_general_beta_gamma(F):
    announce("Newmark beta=0.3 gamma=0.6")
    xyz, tets, h = jittered_kuhn(5, seed=10)
    osim = OracleSim(xyz, tets)
    rng = np.random.default_rng(6)
    e = rng.normal(size=osim.mesh.n_edges)
    e[osim.mesh.boundary_edge] = 0.0
    osim.e, osim.e_prev = e.copy(), 0.9 * e
    with _lib_sim(F, xyz, tets) as L:
        F.fepic_set_fields(L.ctx, e=e, e_prev=0.9 * e)
        for _ in range(2):
            F.fepic_step(L.ctx, 5e-10, 0.3, 0.6)
            osim.step(5e-10, 0.3, 0.6)
        eg, _, bg = F.fepic_get_fields(L.ctx)
    assert np.linalg.norm(eg - osim.e) <= 1e-7 * np.linalg.norm(osim.e)
    assert np.linalg.norm(bg - osim.b) <= 1e-7 * np.linalg.norm(osim.b)


# ----------------------------------------------------------------------------- edge cases
def test_empty_and_degenerate_inputs(F):
    announce("edge cases: no particles, single tet, rejected uploads")
    # a single tet: every edge is on the wall, the system is empty
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    tets = np.array([[0, 1, 2, 3]], np.int32)
    with _lib_sim(F, xyz, tets) as L:
        st = F.fepic_step(L.ctx, 1e-9)
        assert st.cg_iters == 0
        sp = F.fepic_add_species(L.ctx, -Q_E, M_E, 1.0)
        x = np.array([[0.1, 0.1, 0.1], [2.0, 0, 0], [np.nan, 0, 0]])
        assert F.fepic_upload_particles(L.ctx, sp, x, np.zeros((3, 3))) == 2
        assert F.fepic_num_particles(L.ctx, sp) == 1
        # at rest it stays; one pushed out through the wall x = 0 is absorbed
        st = F.fepic_push_particles(L.ctx, 1e-9)
        assert st.n_absorbed == 0
        F.fepic_upload_particles(L.ctx, sp, np.array([[0.2, 0.2, 0.2]]), np.array([[-5e8, 0, 0]]))
        st = F.fepic_push_particles(L.ctx, 1e-9)
        assert st.n_absorbed == 1
        assert F.fepic_num_particles(L.ctx, sp) == 1
    # bad meshes are refused
    with pytest.raises(F.FepicError):
        F.Simulation(xyz, np.array([[0, 1, 2, 2]], np.int32))
    with pytest.raises(F.FepicError):
        F.Simulation(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float), tets)


def test_failed_step_commits_nothing(F):
    announce("atomic step: crossing cap and CG failure")
    xyz, tets, h = jittered_kuhn(4, seed=2)
    x, u = inputs.uniform_box_particles(200, [0.1] * 3, [0.9] * 3, 4e7, seed=3)
    with _lib_sim(F, xyz, tets, precision=1, crossing_cap=1) as L:
        sp = F.fepic_add_species(L.ctx, -Q_E, M_E, 1e3)
        F.fepic_upload_particles(L.ctx, sp, x, u, ids=np.arange(200))
        before = F.fepic_get_particles(L.ctx, sp)
        rc, st = F.fepic_step(L.ctx, 1e-8, check=False)
        assert rc == F.FEPIC_E_CROSSING_CAP
        after = F.fepic_get_particles(L.ctx, sp)
        assert np.array_equal(np.sort(before["id"]), np.sort(after["id"]))
        o1, o2 = np.argsort(before["id"]), np.argsort(after["id"])
        assert np.array_equal(before["x"][o1], after["x"][o2])
    with _lib_sim(F, xyz, tets, precision=1, cg_max_iters=1) as L:
        rng = np.random.default_rng(0)
        e = rng.normal(size=L.sizes["n_edges"])
        F.fepic_set_fields(L.ctx, e=e, e_prev=0.5 * e)
        e_before = F.fepic_get_fields(L.ctx)[0]
        rc, st = F.fepic_step(L.ctx, 1e-9, check=False)
        assert rc == F.FEPIC_E_CG_NOT_CONVERGED
        assert np.array_equal(F.fepic_get_fields(L.ctx)[0], e_before)


def test_sort_period_and_many_waves(F):
    """Ragged counts over many waves, sorting every 3rd step: conservation still exact."""
    announce("sort period 3, 64*300+37 particles")
    xyz, tets, h = jittered_kuhn(6, seed=12)
    n = 64 * 300 + 37
    x, u = inputs.uniform_box_particles(n, [0.05] * 3, [0.95] * 3, 2e6, seed=8)
    with _lib_sim(F, xyz, tets, sort_period=3, diagnostics=1) as L:
        sp = F.fepic_add_species(L.ctx, -Q_E, M_E, 1e2)
        sp2 = F.fepic_add_species(L.ctx, Q_E, 1836 * M_E, 1e2)
        F.fepic_upload_particles(L.ctx, sp, x, u)
        F.fepic_upload_particles(L.ctx, sp2, x, u / 40)
        F.fepic_init_electrostatic(L.ctx, 1e-14)
        for k in range(7):
            st = F.fepic_step(L.ctx, 3e-9, 0.25, 0.5)
            assert st.cont_resid_rel < 1e-12
            if st.gauss_drift_check_rel >= 0:
                assert st.gauss_drift_check_rel < 1e-12
        assert st.n_crossings > 0


def test_sort_groups_of_equal_tets(F):
    """The counting sort groups the lanes of a wave by tet: every particle in one tet, two
    tets alternating lane by lane (groups that are not runs), and 200 tets in turn (64
    distinct tets in every wave).  The result is sorted by tet, keeps every particle in the
    tet it was placed in, and a step at rest in zero fields re-sorts it unchanged."""
    announce("sort: one tet, alternating tets, 64 distinct tets per wave")
    xyz, tets, h = jittered_kuhn(5, seed=13)
    m = OracleSim(xyz, tets).mesh
    cent = xyz[tets].mean(axis=1)
    n = 64 * 20 + 11
    k = np.arange(n)
    patterns = {"one tet": np.full(n, 17), "alternating": np.where(k % 2 == 0, 3, 140),
                "200 in turn": (k % 200) * 3 % len(tets)}
    for name, sel in patterns.items():
        x = cent[sel]
        want = m.locate(x)
        assert np.all(want >= 0)
        with _lib_sim(F, xyz, tets, sort_period=1) as L:
            sp = F.fepic_add_species(L.ctx, -Q_E, M_E, 1.0)
            assert F.fepic_upload_particles(L.ctx, sp, x, np.zeros((n, 3)), ids=k) == 0
            for step in range(2):
                g = F.fepic_get_particles(L.ctx, sp)
                assert len(g["id"]) == n, name
                assert np.all(np.diff(g["tet"]) >= 0), name
                assert np.array_equal(np.sort(g["id"]), k), name
                assert np.array_equal(g["tet"], want[g["id"]]), name
                F.fepic_push_particles(L.ctx, 1e-15)


def test_caller_allocator_matches_default(F):
    """Device memory from torch's caching allocator through fepic_set_allocator gives the
    same results as hipMalloc, and every allocation is returned when the context closes."""
    announce("caller allocator (torch caching allocator)")
    import torch
    xyz, tets, h = jittered_kuhn(4, lo=(-0.02, -0.02, 0.0), hi=(0.02, 0.02, 0.04), seed=5)
    x, u = inputs.beam_particles(700, 0.008, 0.004, 0.03, 1000.0, 1.0, M_E, 5)
    out = []
    counts = {"alloc": 0, "free": 0}
    a_fn, f_fn = F.torch_allocator(0)

    def a_count(n):
        counts["alloc"] += 1
        return a_fn(n)

    def f_count(p):
        counts["free"] += 1
        f_fn(p)

    before = torch.cuda.memory_allocated(0)
    for mode in ("default", "torch"):
        L = F.Simulation(xyz, tets, device=0, precision=1) if mode == "default" else None
        if mode == "torch":
            ctx = F.fepic_create(device=0, precision=1)
            cbs = F.fepic_set_allocator(ctx, a_count, f_count)
            F.fepic_upload_mesh(ctx, xyz, tets)
        else:
            ctx = L.ctx
        sp = F.fepic_add_species(ctx, -Q_E, M_E, 5e4)
        F.fepic_upload_particles(ctx, sp, x, u, ids=np.arange(len(x)))
        F.fepic_init_electrostatic(ctx, 1e-14)
        for _ in range(3):
            F.fepic_step(ctx, 1e-10)
        if mode == "torch":
            assert torch.cuda.memory_allocated(0) > before
        e, _, b = F.fepic_get_fields(ctx)
        out.append((e, F.fepic_get_particles(ctx, sp)))
        if mode == "torch":
            F.fepic_destroy(ctx)
            del cbs
        else:
            L.close()
    assert counts["alloc"] > 0 and counts["alloc"] == counts["free"]
    assert torch.cuda.memory_allocated(0) == before
    (e0, p0), (e1, p1) = out
    # the two runs differ only in the order of FP64 atomic additions (~1e-16 in the
    # current), which the solves carry to the fields at the CG tolerance's level
    assert np.linalg.norm(e0 - e1) <= 1e-9 * np.linalg.norm(e0)
    i0, i1 = np.argsort(p0["id"]), np.argsort(p1["id"])
    assert np.array_equal(p0["id"][i0], p1["id"][i1])
    assert np.max(np.abs(p0["x"][i0] - p1["x"][i1])) <= 1e-12
