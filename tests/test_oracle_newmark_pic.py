"""Pins for the oracle's field update and whole PIC step (Sec. II-B, III-A, IV-A).

* Newmark coefficients: the scalar recurrence reproduces the textbook dispersion
  relations (trapezoid tan(w_d dt/2) = w dt/2 for beta = 1/4; central difference
  cos(w_d dt) = 1 - (w dt)^2/2 for beta = 0; amplitude decay for gamma > 1/2).
* Vacuum energy invariant of the beta = 1/4, gamma = 1/2 scheme; static charge is a fixed
  point; PCG agrees with a sparse direct solve.
* Faraday keeps D2 b fixed and leaves a uniform B untouched when e = 0.
* Whole step: charge continuity and the Gauss-drift identity every step; the cyclotron
  orbit against its closed form; the paper's Table I orbit; the naive-current scheme
  (eqs. (badNmB)/(badwave)) breaks Gauss while the time-integrated current keeps it.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem, newmark
from oracle.constants import C_LIGHT, M_E, Q_E
from oracle.mesh import Mesh
from oracle.pic import OracleSim
from paper_2102_06248_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _scalar_recurrence(m, k, dt, beta, gamma):
    A, B1, B2 = newmark.newmark_operators(sp.csr_matrix([[m]]), sp.csr_matrix([[k]]), dt, beta, gamma)
    return A[0, 0], B1[0, 0], B2[0, 0]


@pytest.mark.parametrize("Om", [0.1, 0.7, 2.0, 30.0])
def test_newmark_dispersion_trapezoid(Om):
    A, B1, B2 = _scalar_recurrence(1.0, Om * Om, 1.0, 0.25, 0.5)
    z = np.roots([A, -B1, -B2])
    assert np.allclose(np.abs(z), 1.0, atol=1e-14)
    th = abs(np.angle(z[0]))
    assert math.tan(th / 2) == pytest.approx(Om / 2, rel=1e-12)


def test_newmark_dispersion_central_difference_and_damping():
    Om = 0.9
    A, B1, B2 = _scalar_recurrence(1.0, Om * Om, 1.0, 0.0, 0.5)
    z = np.roots([A, -B1, -B2])
    assert math.cos(abs(np.angle(z[0]))) == pytest.approx(1 - Om * Om / 2, rel=1e-13)
    A, B1, B2 = _scalar_recurrence(1.0, Om * Om, 1.0, 0.3, 0.6)
    z = np.roots([A, -B1, -B2])
    # product of roots = (1 + (1/2 + beta - gamma) Om^2) / (1 + beta Om^2) < 1
    assert np.prod(np.abs(z)) == pytest.approx((1 + 0.2 * Om * Om) / (1 + 0.3 * Om * Om), rel=1e-13)


@pytest.fixture(scope="module")
def sim_small():
    xyz, tets = inputs.kuhn_cube(3)
    xyz = inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(3), 1 / 3, 0.1, seed=4)
    return xyz, tets


def test_vacuum_energy_invariant(sim_small):
    sim = OracleSim(*sim_small, cg_tol=1e-13)
    rng = np.random.default_rng(0)
    ie = sim.ie
    sim.e[ie] = rng.normal(size=len(ie))
    sim.e_prev[ie] = sim.e[ie] + 0.05 * rng.normal(size=len(ie))
    dt = 2e-9          # many times the explicit stability limit of this mesh
    M, S = sim.M, sim.S
    energies = []
    for _ in range(40):
        e_old = sim.e.copy()
        sim.step(dt, 0.25, 0.5)
        de = sim.e - e_old
        eb = 0.5 * (sim.e + e_old)
        energies.append(de @ (M @ de) / dt ** 2 + eb @ (S @ eb))
    energies = np.array(energies)
    assert np.max(np.abs(energies / energies[0] - 1)) < 1e-9


def test_static_charge_fixed_point(sim_small):
    sim = OracleSim(*sim_small, cg_tol=1e-13)
    rng = np.random.default_rng(1)
    phi = np.zeros(sim.mesh.n_nodes)
    phi[sim.inode] = rng.normal(size=len(sim.inode))
    sim.e = -(sim.D @ phi)
    sim.e_prev = sim.e.copy()
    e0 = sim.e.copy()
    for _ in range(3):
        sim.step(1e-9, 0.25, 0.5)
    assert np.allclose(sim.e, e0, rtol=0, atol=1e-10 * abs(e0).max())


def test_pcg_matches_direct_solve(sim_small):
    sim = OracleSim(*sim_small)
    A, _, _ = sim.operators(5e-10, 0.25, 0.5)
    rng = np.random.default_rng(2)
    b = rng.normal(size=A.shape[0])
    x, it, res = newmark.pcg_jacobi(A, b, np.zeros_like(b), 1e-12)
    xd = spla.spsolve(A.tocsc(), b)
    assert res <= 1e-12 * 1.01
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_faraday_invariants(sim_small):
    sim = OracleSim(*sim_small)
    B0 = np.array([0.1, -0.2, 0.3])
    b0 = sim.mesh.face_dofs_of_uniform_field(B0)
    assert np.allclose(newmark.faraday(sim.C, b0, np.zeros(sim.mesh.n_edges), np.zeros(sim.mesh.n_edges),
                                       1e-9, 0.5), b0)
    rng = np.random.default_rng(3)
    b1 = newmark.faraday(sim.C, b0, rng.normal(size=sim.mesh.n_edges), rng.normal(size=sim.mesh.n_edges), 1e-9, 0.5)
    assert np.allclose(sim.D2 @ b1, sim.D2 @ b0, atol=1e-15)


# ---------------------------------------------------------------- whole steps

def _c1(n_steps, check_every=1):
    xyz, tets = inputs.kuhn_cube(6)
    sim = OracleSim(xyz, tets)
    B0, v0 = 0.1, 1e5
    gam = 1 / math.sqrt(1 - (v0 / C_LIGHT) ** 2)
    om = Q_E * B0 / (gam * M_E)
    dt = 2 * math.pi / om / 50
    rL = gam * M_E * v0 / (Q_E * B0)
    sim.set_uniform_B([0, 0, B0])
    s = sim.add_species(-Q_E, M_E, 1.0)
    c = np.full(3, 5 / 12)
    sim.upload_particles(s, [c + [rL, 0, 0]], [[0, gam * v0, 0]])
    sim.init_electrostatic()
    xs, stats = [], []
    for n in range(n_steps):
        st = sim.step(dt, 0.25, 0.5)
        xs.append(sim.species[0].x[0].copy())
        stats.append(st)
    return np.array(xs), stats, dict(c=c, rL=rL, om=om, dt=dt)


@pytest.mark.slow
def test_c1_single_electron_orbit_and_conservation():
    xs, stats, p = _c1(2000)
    a = 0.5 * p["om"] * p["dt"]
    R = p["rL"] * math.sqrt(1 + a * a)
    P = xs[:, :2] - p["c"][:2]
    A = np.column_stack([2 * P, np.ones(len(P))])
    sol = np.linalg.lstsq(A, (P ** 2).sum(1), rcond=None)[0]
    cc = sol[:2]
    assert abs(math.sqrt(sol[2] + cc @ cc) / R - 1) < 1e-8
    r = np.linalg.norm(P - cc, axis=1)
    assert np.max(np.abs(r / R - 1)) < 1e-8
    ang = np.unwrap(np.arctan2(P[:, 1] - cc[1], P[:, 0] - cc[0]))
    assert np.max(np.abs(np.diff(ang) - 2 * math.atan(a))) < 1e-8
    assert abs(xs[:, 2] - p["c"][2]).max() < 1e-12
    assert sum(s["n_crossings"] for s in stats) > 200
    assert max(s["cont_resid_rel"] for s in stats) < 1e-12
    assert max(s["gauss_drift_check_rel"] for s in stats[2:]) < 1e-12
    assert max(s["cg_rel_resid"] for s in stats) <= 1e-10


def test_table1_cyclotron_closed_form():
    """Table I parameters: r_L = m v0 / (|Q| B) = 0.25 m and omega = |Q| B / m = 1.2e7
    (non-relativistic values the table is built on).  The discrete relativistic orbit's
    radius converges to the relativistic r_L at second order in dt."""
    g = json.load(open(os.path.join(HERE, "golden", "cyclotron_table1.json")))
    B, Q, m, v0 = g["B_z_T"], g["Q_C"], g["m_kg"], g["v0_y_m_per_s"]
    assert m * v0 / (abs(Q) * B) == pytest.approx(0.25, rel=1e-6)
    assert abs(Q) * B / m == pytest.approx(1.2e7, rel=1e-6)
    gam = 1 / math.sqrt(1 - (v0 / C_LIGHT) ** 2)
    rL = gam * m * v0 / (abs(Q) * B)
    om = abs(Q) * B / (gam * m)
    xyz, tets = inputs.kuhn_cube(6)
    errs = []
    for nper in (25, 50, 100):
        sim = OracleSim(xyz, tets)
        sim.set_uniform_B([0, 0, B])
        s = sim.add_species(Q, m, 1e-12)      # negligible self-field
        r0 = np.array([g["r0_m"][0], g["r0_m"][1], 5 / 12])
        sim.upload_particles(s, [r0], [[0, gam * v0, 0]])
        dt = 2 * math.pi / om / nper
        xs = []
        ncross = 0
        for _ in range(nper):
            st = sim.step(dt, 0.25, 0.5, solve=False)
            ncross += st["n_crossings"]
            xs.append(sim.species[0].x[0].copy())
        assert sim.species[0].alive[0] == 1
        assert ncross >= 10
        P = np.array(xs)[:, :2] - 0.5
        A = np.column_stack([2 * P, np.ones(len(P))])
        sol = np.linalg.lstsq(A, (P ** 2).sum(1), rcond=None)[0]
        Rfit = math.sqrt(sol[2] + sol[:2] @ sol[:2])
        a = 0.5 * om * dt
        assert Rfit == pytest.approx(rL * math.sqrt(1 + a * a), rel=1e-10)
        errs.append(abs(Rfit / rL - 1))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2) < 0.05)


def _tiny_beam(n=300, seed=5):
    xyz, tets = inputs.kuhn_cube(4, lo=(-0.02, -0.02, 0.0), hi=(0.02, 0.02, 0.04))
    xyz = inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(4), 0.01, 0.1, seed=seed)
    x, u = inputs.beam_particles(n, 0.008, 0.004, 0.03, 1000.0, 1.0, M_E, seed)
    return xyz, tets, x, u


def test_tiny_beam_continuity_and_gauss_drift_every_step():
    xyz, tets, x, u = _tiny_beam()
    sim = OracleSim(xyz, tets)
    s = sim.add_species(-Q_E, M_E, 5e4)
    assert sim.upload_particles(s, x, u) == 0
    sim.init_electrostatic()
    dt = 1e-10
    for n in range(12):
        st = sim.step(dt, 0.25, 0.5)
        assert st["cont_resid_rel"] < 1e-12
        if st["gauss_drift_check_rel"] is not None:
            assert st["gauss_drift_check_rel"] < 1e-12
        assert st["gauss_resid_rel"] < 1e-6
    assert st["n_crossings"] > 0


def test_naive_current_breaks_gauss():
    """Feeding the point-sampled current J(t_n) through the Newmark source (the scheme of
    eqs. (badNmB)/(badwave)) violates Gauss far above solver tolerance; the time-
    integrated current does not."""
    xyz, tets, x, u = _tiny_beam(200, seed=6)
    dt = 1e-10
    res = {}
    for mode in ("G", "naive"):
        sim = OracleSim(xyz, tets)
        s = sim.add_species(-Q_E, M_E, 5e4)
        sim.upload_particles(s, x, u)
        sim.init_electrostatic()
        j_hist = []

        def point_current():
            sp_ = sim.species[0]
            a = sp_.alive.astype(bool)
            j = np.zeros(sim.mesh.n_edges)
            lam = sim.mesh.barycentric(sp_.tet[a], sp_.x[a])
            W = fem.whitney1(lam, sim.mesh.grad_lambda[sp_.tet[a]])
            v = sp_.u[a] / np.sqrt(1 + np.sum(sp_.u[a] ** 2, 1) / C_LIGHT ** 2)[:, None]
            np.add.at(j, sim.mesh.tet_edges[sp_.tet[a]].ravel(),
                      (sp_.q * sp_.w * np.einsum("pid,pd->pi", W, v)).ravel())
            return j

        j_hist.append(point_current())

        def naive(dG_new, dG_old):
            # -dt^2 d_t J with J sampled at the particle positions and a backward difference
            jn = point_current_after[0]
            return (dt * (jn - j_hist[-1]))[sim.ie]

        worst = 0.0
        for _ in range(10):
            if mode == "naive":
                # the particle step runs inside sim.step; sample J after it via a hook
                point_current_after = [None]
                orig = sim.push_particles

                def hooked(dt_, orig=orig, holder=point_current_after):
                    out = orig(dt_)
                    holder[0] = point_current()
                    return out
                sim.push_particles = hooked
                st = sim.step(dt, 0.25, 0.5, source_override=naive)
                sim.push_particles = orig
                j_hist.append(point_current_after[0])
            else:
                st = sim.step(dt, 0.25, 0.5)
            worst = max(worst, st["gauss_resid_rel"])
            assert st["cont_resid_rel"] < 1e-12
        res[mode] = worst
    assert res["G"] < 1e-7
    assert res["naive"] > 1e3 * res["G"]
