"""GPU parity of the first-order absorbing boundary (fepic_set_absorbing_faces) against the
oracle (OracleSim(abc_faces=...), oracle/newmark.py, oracle/fem.py boundary_matrix).

* Whole steps of a beam running into absorbing walls (all-FP64 particles, Jacobi-PCG, both
  solves to 1e-10): fields to 1e-6 relative every step, particles to 1e-9 m, continuity and
  the Gauss-drift identity on interior nodes to 1e-12.
* Vacuum pulse with absorbing faces on part of the wall, on the library's own states: the
  damped recurrence's energy balance with the oracle's boundary matrix (assembled by
  quadrature, independently of the library's closed form) to 1e-9 of the initial energy
  per step, the fields against the oracle's to 1e-8, and the energy leaving the box.
* The call is refused once the context has stepped.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gpu_common import announce, have_gpu, jittered_kuhn, require_lib
from oracle import fem, newmark
from oracle.constants import C_LIGHT, M_E, MU0, Q_E
from oracle.pic import OracleSim
from paper_2102_06248_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    if not have_gpu():
        pytest.fail("GPU tests need an MI355X")
    return require_lib()


def test_abc_beam_steps_vs_oracle(F):
    announce("absorbing walls: beam whole steps vs oracle")
    xyz, tets, h = jittered_kuhn(4, lo=(-0.02, -0.02, 0.0), hi=(0.02, 0.02, 0.04), seed=5)
    x, u = inputs.beam_particles(600, 0.008, 0.004, 0.03, 1000.0, 1.0, M_E, 5)
    w, dt = 5e4, 1e-10
    osim = OracleSim(xyz, tets, abc_faces="all")
    s = osim.add_species(-Q_E, M_E, w)
    osim.upload_particles(s, x, u, ids=np.arange(len(x)))
    osim.init_electrostatic(1e-14)
    absorbed = 0
    with F.Simulation(xyz, tets, device=0, precision=F.FEPIC_ALL_FP64, diagnostics=1,
                      preconditioner=F.FEPIC_PC_JACOBI) as L:
        F.fepic_set_absorbing_faces(L.ctx)
        sp = F.fepic_add_species(L.ctx, -Q_E, M_E, w)
        F.fepic_upload_particles(L.ctx, sp, x, u, ids=np.arange(len(x)))
        F.fepic_init_electrostatic(L.ctx, 1e-14)
        for k in range(10):
            so = osim.step(dt)
            st = F.fepic_step(L.ctx, dt)
            absorbed += st.n_absorbed
            assert st.n_absorbed == so["n_absorbed"], k
            assert st.cont_resid_rel <= 1e-12, k
            if k >= 2:
                assert 0 <= st.gauss_drift_check_rel <= 1e-12, (k, st.gauss_drift_check_rel)
            e, _, b = F.fepic_get_fields(L.ctx)
            assert np.linalg.norm(e - osim.e) <= 1e-6 * np.linalg.norm(osim.e), k
            assert np.linalg.norm(b - osim.b) <= 1e-6 * np.linalg.norm(osim.b) + 1e-30, k
            gp = F.fepic_get_particles(L.ctx, sp)
            op_ = osim.particles(s)
            gi, oi = np.argsort(gp["id"]), np.argsort(op_["id"])
            assert np.array_equal(gp["id"][gi], op_["id"][oi]), k
            assert np.abs(gp["x"][gi] - op_["x"][oi]).max() <= 1e-9, k
        wall = osim.mesh.boundary_edge
        assert np.abs(e[wall]).max() > 1e-3 * np.abs(e).max()
    assert absorbed > 20
    print(f"\n[abc beam] {absorbed} absorbed, cg {st.cg_iters} iterations, drift {st.gauss_drift_check_rel:.1e}")


def test_abc_vacuum_pulse_energy_on_library_states(F):
    announce("absorbing faces: vacuum pulse energy balance")
    xyz, tets = inputs.kuhn_cube(6)
    m0 = OracleSim(xyz, tets).mesh
    wall = np.nonzero(m0.boundary_face)[0]
    zc = m0.xyz[m0.faces[wall]].mean(axis=1)[:, 2]
    sel = wall[(zc < 1e-9) | (zc > 1 - 1e-9) | (np.arange(len(wall)) % 3 == 0)]
    osim = OracleSim(xyz, tets, cg_tol=1e-13, abc_faces=sel)
    m = osim.mesh
    dt = 1e-10
    Mf = fem.face_mass_matrix(m)
    c = m.xyz[m.faces].mean(axis=1)
    bpulse = np.exp(-np.sum((c - 0.5) ** 2, axis=1) / (2 * 0.1 ** 2)) * m.face_area_vectors()[:, 0]
    r = osim.C.T @ (Mf @ bpulse)
    v = np.zeros(m.n_edges)
    v[osim.ie] = spla.spsolve(osim.Mi.tocsc(), r[osim.ie])
    e0, em = np.zeros(m.n_edges), -dt * v
    osim.e, osim.e_prev = e0.copy(), em.copy()
    Cd = osim.K / (MU0 * C_LIGHT)
    E0 = newmark.damped_energy(osim.M, osim.S, e0, em, dt)
    with F.Simulation(xyz, tets, device=0, cg_tol=1e-13, preconditioner=F.FEPIC_PC_JACOBI) as L:
        F.fepic_set_absorbing_faces(L.ctx, sel)
        F.fepic_set_fields(L.ctx, e=e0, e_prev=em)
        states = [em, e0]
        for k in range(60):
            F.fepic_step(L.ctx, dt)
            osim.step(dt)
            en, _, _ = F.fepic_get_fields(L.ctx)
            assert np.linalg.norm(en - osim.e) <= 1e-8 * np.linalg.norm(osim.e), k
            states.append(en)
        with pytest.raises(F.FepicError) as ei:
            F.fepic_set_absorbing_faces(L.ctx, sel)
        assert F.ERROR_NAMES[ei.value.code] == "FEPIC_E_STATE"
    worst = 0.0
    for k in range(1, len(states) - 1):
        em1, en, ep1 = states[k - 1], states[k], states[k + 1]
        before = newmark.damped_energy(osim.M, osim.S, en, em1, dt)
        after = newmark.damped_energy(osim.M, osim.S, ep1, en, dt)
        d = ep1 - em1
        worst = max(worst, abs((before - after) - float(d @ (Cd @ d)) / (4.0 * dt)) / E0)
    assert worst <= 1e-9
    final = newmark.damped_energy(osim.M, osim.S, states[-1], states[-2], dt)
    assert final < 0.5 * E0
    print(f"\n[abc pulse] energy {final / E0:.3f} of the initial after 60 steps, balance {worst:.1e}")
