"""Pins of the oracle's first-order absorbing boundary (oracle/fem.py boundary_matrix,
oracle/newmark.py damped recurrence, OracleSim(abc_faces=...)), each against something
the mathematics fixes rather than the oracle's own formulas:

* K's quadratic form on fields the Whitney-1 space represents exactly: a uniform E0 gives
  the sum over absorbing faces of area (|E0|^2 - (n . E0)^2) (unit cube: 4 |E0|^2); a linear
  tangential field a + w n x (r - r_c) on one face gives the integral of |E_t|^2, computed
  with the three-midpoint rule (exact for quadratics);
* symmetry, positive semi-definiteness, and no weight on edges off the absorbing faces;
* the discrete energy balance of the damped Newmark recurrence at beta = 1/4, gamma = 1/2:
  E^{n+1/2} - E^{n-1/2} = -(e^{n+1} - e^{n-1})^T C (e^{n+1} - e^{n-1}) / (4 dt), which a
  wrong sign or weight of any damping term breaks (a planted mistake shows it does);
* physics: a pulse in a box with absorbing walls leaves (energy below 5 % after four
  crossing times) while with PEC walls its energy is conserved;
* the Gauss and continuity identities on interior nodes are untouched with a beam running
  into an absorbing wall.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, newmark
from oracle.constants import C_LIGHT, M_E, MU0, Q_E
from oracle.mesh import Mesh
from oracle.pic import OracleSim
from paper_2102_06248_amd import inputs


def _jittered(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), seed=3):
    xyz, tets = inputs.kuhn_cube(n, lo, hi)
    h = (np.asarray(hi) - np.asarray(lo)).min() / n
    return inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(n), h, 0.1, seed), tets


def test_uniform_field_unit_cube():
    xyz, tets = inputs.kuhn_cube(3)
    m = Mesh(xyz, tets)
    K = fem.boundary_matrix(m, m.boundary_face)
    E0 = np.array([0.3, -1.2, 0.7])
    e = m.edge_dofs_of_uniform_field(E0)
    assert e @ (K @ e) == pytest.approx(4.0 * E0 @ E0, rel=1e-13)


def test_uniform_field_on_selected_faces_of_a_box():
    xyz, tets = _jittered(4, lo=(-0.1, 0.0, 0.2), hi=(0.3, 0.5, 0.45), seed=7)
    m = Mesh(xyz, tets)
    rng = np.random.default_rng(1)
    wall = np.nonzero(m.boundary_face)[0]
    sel = wall[rng.random(len(wall)) < 0.4]
    K = fem.boundary_matrix(m, sel)
    av = m.face_area_vectors()[sel]
    area = np.linalg.norm(av, axis=1)
    n = av / area[:, None]
    for E0 in rng.normal(size=(3, 3)):
        e = m.edge_dofs_of_uniform_field(E0)
        expect = np.sum(area * (E0 @ E0 - (n @ E0) ** 2))
        assert e @ (K @ e) == pytest.approx(expect, rel=1e-12)


def test_linear_tangential_field_on_one_face():
    """One tet, one absorbing face: E = a + w n x (r - r_c) is tangential on the face and
    lies in the Whitney-1 space, so its edge integrals are exact at edge midpoints and
    eT K e = int |E|^2 dS, which the three-midpoint rule gives exactly."""
    xyz = np.array([[0.1, 0.0, 0.0], [1.3, 0.2, 0.1], [0.2, 0.9, -0.1], [0.4, 0.3, 1.1]])
    tets = np.array([[0, 1, 2, 3]], dtype=np.int32)
    m = Mesh(xyz, tets)
    f = int(np.nonzero((m.faces == [0, 1, 2]).all(axis=1))[0][0])
    K = fem.boundary_matrix(m, [f])
    p = xyz[[0, 1, 2]]
    N = np.cross(p[1] - p[0], p[2] - p[0])
    n, area = N / np.linalg.norm(N), 0.5 * np.linalg.norm(N)
    rc = p.mean(axis=0)
    t1 = (p[1] - p[0]) / np.linalg.norm(p[1] - p[0])
    t2 = np.cross(n, t1)
    for a1, a2, w in [(1.0, 0.0, 0.0), (0.3, -0.7, 0.0), (0.0, 0.0, 2.0), (0.5, 0.2, -1.5)]:
        def E(r):
            return a1 * t1 + a2 * t2 + w * np.cross(n, r - rc)
        mid = 0.5 * (xyz[m.edges[:, 0]] + xyz[m.edges[:, 1]])
        e = np.array([E(mid[i]) @ (xyz[m.edges[i, 1]] - xyz[m.edges[i, 0]]) for i in range(m.n_edges)])
        mids = [0.5 * (p[0] + p[1]), 0.5 * (p[1] + p[2]), 0.5 * (p[0] + p[2])]
        expect = area / 3.0 * sum(E(r) @ E(r) for r in mids)
        assert e @ (K @ e) == pytest.approx(expect, rel=1e-13)


def test_structure():
    xyz, tets = _jittered(3, seed=2)
    m = Mesh(xyz, tets)
    sel = np.nonzero(m.boundary_face)[0][::3]
    K = fem.boundary_matrix(m, sel).toarray()
    scale = np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-15 * scale
    assert np.linalg.eigvalsh(K).min() >= -1e-14 * scale
    on = np.zeros(m.n_edges, dtype=bool)
    on[m.face_edges[sel].ravel()] = True
    assert np.abs(K[~on]).max() <= 1e-14 * scale
    assert np.abs(K[np.ix_(on, on)]).max() == pytest.approx(scale)


def _pulse(o, dt):
    """e^0 = 0, e^{-1} = -dt M^-1 C^T Mf b for a localized b: charge-free (C D = 0)."""
    m = o.mesh
    Mf = fem.face_mass_matrix(m)
    c = m.xyz[m.faces].mean(axis=1)
    b = np.exp(-np.sum((c - 0.5) ** 2, axis=1) / (2 * 0.08 ** 2)) * m.face_area_vectors()[:, 2]
    r = o.C.T @ (Mf @ b)
    v = np.zeros(m.n_edges)
    v[o.ie] = spla.spsolve(o.Mi.tocsc(), r[o.ie])
    o.e = np.zeros(m.n_edges)
    o.e_prev = -dt * v


def _energy_run(abc, steps, operators=None):
    xyz, tets = inputs.kuhn_cube(8)
    o = OracleSim(xyz, tets, cg_tol=1e-14, abc_faces=abc)
    if operators is not None:
        o.operators = operators.__get__(o)
    dt = 1e-10
    _pulse(o, dt)
    Cd = o.K / (MU0 * C_LIGHT) if abc else None
    E0 = newmark.damped_energy(o.M, o.S, o.e, o.e_prev, dt)
    E, worst = E0, 0.0
    for _ in range(steps):
        em1 = o.e_prev.copy()
        o.step(dt)
        En = newmark.damped_energy(o.M, o.S, o.e, o.e_prev, dt)
        loss = 0.0
        if Cd is not None:
            d = o.e - em1
            loss = float(d @ (Cd @ d)) / (4.0 * dt)
        worst = max(worst, abs((E - En) - loss) / E0)
        E = En
    return E / E0, worst


def test_energy_balance_and_absorption():
    frac, worst = _energy_run("all", 130)
    assert worst <= 1e-9
    assert frac < 0.05              # c dt = 3 cm, 130 steps = 3.9 m: four box crossings
    frac_pec, worst_pec = _energy_run(None, 40)
    assert worst_pec <= 1e-9 and abs(frac_pec - 1.0) <= 1e-9


def test_planted_sign_mistake_breaks_the_balance():
    def wrong(self, dt, beta, gamma):
        A, B1, B2 = newmark.newmark_operators(self.Mi, self.Si, dt, beta, gamma, self.Kd)
        return A, B1, B2 - (2.0 * (1.0 - gamma) * dt) * self.Kd     # (1 - gamma) dt C with the wrong sign
    _, worst = _energy_run("all", 20, operators=wrong)
    assert worst > 1e-4


def test_beam_into_absorbing_wall_keeps_gauss_on_interior_nodes():
    xyz, tets = _jittered(4, lo=(-0.02, -0.02, 0.0), hi=(0.02, 0.02, 0.04), seed=5)
    x, u = inputs.beam_particles(400, 0.008, 0.004, 0.03, 1000.0, 1.0, M_E, 5)
    o = OracleSim(xyz, tets, abc_faces="all")
    s = o.add_species(-Q_E, M_E, 5e4)
    o.upload_particles(s, x, u, ids=np.arange(len(x)))
    o.init_electrostatic(1e-14)
    absorbed = 0
    for k in range(10):
        st = o.step(1e-10)
        absorbed += st["n_absorbed"]
        assert st["cont_resid_rel"] <= 1e-12, k
        if k >= 2:
            assert st["gauss_drift_check_rel"] <= 1e-12, k
    assert absorbed > 20
    # the edges on the absorbing walls carry field
    wall = o.mesh.boundary_edge
    assert np.abs(o.e[wall]).max() > 1e-3 * np.abs(o.e).max()
