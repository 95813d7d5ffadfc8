"""Pins for the oracle's mixed finite element field updates (oracle/mfem.py): NM-MFEM (the
three-level Newmark recurrence, beta = 1/4, gamma = 1/2) and BD-MFEM (backward
differences), both with the time-integrated current G as source.

* Vacuum, NM-MFEM: the recurrence is the trapezoid rule on two-step averages, so the
  energy of (X^{n+1} + X^n) / 2 is conserved (to the solver tolerance).
* Vacuum, BD-MFEM: the energy drops by exactly 1/2 |X^{n+1} - X^n|^2 each step (an
  identity of backward Euler for a skew system).
* The field of a static charge, e = -D phi with b = 0, is a fixed point of both.
* With moving particles, continuity holds to round-off and the Gauss residual follows
  the solver's own recurrence (NM: r^{n+1} - r^{n-1} = D^T r_cg, BD: r^{n+1} - r^n =
  D^T r_cg) to round-off.
* A planted mistake, the NM-MFEM source taken from the current at the three time levels
  with the Newmark weights (the scheme Sec. II-B shows is not charge conserving), makes
  the Gauss residual drift far beyond the solver tolerance.
"""
import numpy as np
import pytest

from oracle import fem, mfem, newmark
from oracle.constants import M_E, Q_E
from oracle.pic import OracleSim
from paper_2102_06248_amd import inputs


def _mesh(n=3, seed=4):
    xyz, tets = inputs.kuhn_cube(n)
    return inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(n), 1 / n, 0.1, seed=seed), tets


def _vacuum_fields(osim, seed):
    m = osim.mesh
    rng = np.random.default_rng(seed)
    e = rng.normal(size=m.n_edges)
    e[m.boundary_edge] = 0.0
    b = osim.C @ rng.normal(size=m.n_edges) * 1e-9          # divergence-free flux
    return e, b


@pytest.mark.parametrize("solver", ["nm_mfem", "bd_mfem"])
def test_vacuum_energy(solver):
    xyz, tets = _mesh()
    osim = OracleSim(xyz, tets, cg_tol=1e-13, field_solver=solver)
    e, b = _vacuum_fields(osim, 3)
    osim.e = e.copy()
    osim.e_prev = e.copy()
    osim.b = b.copy()
    osim.b_prev = b.copy()
    dt = 2e-9                                             # far beyond the explicit limit
    M, Mf = osim.M, osim.Mf
    W = [mfem.energy(M, Mf, osim.e, osim.b)]
    Wavg = [mfem.energy(M, Mf, osim.e, osim.b)]
    drops = []
    for _ in range(40):
        e0, b0 = osim.e.copy(), osim.b.copy()
        osim.step(dt)
        W.append(mfem.energy(M, Mf, osim.e, osim.b))
        Wavg.append(mfem.energy(M, Mf, 0.5 * (osim.e + e0), 0.5 * (osim.b + b0)))
        drops.append(mfem.energy(M, Mf, osim.e - e0, osim.b - b0))
    W, Wavg, drops = np.array(W), np.array(Wavg), np.array(drops)
    if solver == "nm_mfem":
        assert np.abs(Wavg[1:] - Wavg[0]).max() <= 1e-10 * Wavg[0]
        assert np.abs(W - W[0]).max() > 1e-6 * W[0]           # the step energies themselves oscillate
    else:
        assert np.allclose(W[:-1] - W[1:], drops, rtol=1e-9, atol=1e-10 * W[0])
        assert W[-1] < 0.5 * W[0]                             # dissipative at this step


@pytest.mark.parametrize("solver", ["nm_mfem", "bd_mfem"])
def test_electrostatic_field_is_a_fixed_point(solver):
    """e = -D phi (the field of a static charge: S D = 0) with b = 0 and no current stays."""
    xyz, tets = _mesh()
    osim = OracleSim(xyz, tets, cg_tol=1e-13, field_solver=solver)
    rng = np.random.default_rng(1)
    phi = np.zeros(osim.mesh.n_nodes)
    phi[osim.inode] = rng.normal(size=len(osim.inode))
    osim.e = -(osim.D @ phi)
    osim.e_prev = osim.e.copy()
    e0 = osim.e.copy()
    for _ in range(4):
        osim.step(1e-9)
    assert np.abs(osim.e - e0).max() <= 1e-10 * np.abs(e0).max()
    assert np.abs(osim.b).max() <= 1e-10 * 1e-9 * np.abs(e0).max()


def _beam(solver, **kw):
    xyz, tets = inputs.kuhn_cube(4, lo=(-0.02, -0.02, 0.0), hi=(0.02, 0.02, 0.04))
    xyz = inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(4), 0.01, 0.1, seed=2)
    osim = OracleSim(xyz, tets, field_solver=solver, **kw)
    s = osim.add_species(-Q_E, M_E, 5e4)
    x, u = inputs.beam_particles(400, 0.008, 0.004, 0.03, 1000.0, 1.0, M_E, seed=3)
    osim.upload_particles(s, x, u)
    osim.init_electrostatic(1e-14)
    return osim


@pytest.mark.parametrize("solver", ["nm_mfem", "bd_mfem"])
def test_moving_beam_conserves_charge_and_gauss(solver):
    osim = _beam(solver)
    for k in range(10):
        st = osim.step(1e-10)
        assert st["cont_resid_rel"] <= 1e-13
        if st["gauss_drift_check_rel"] is not None:
            assert st["gauss_drift_check_rel"] <= 1e-12
        assert st["gauss_resid_rel"] <= 1e-8
        assert np.abs(osim.D2 @ osim.b).max() <= 1e-20
    assert st["n_particles"] > 200 and np.abs(osim.e).max() > 0


def test_naive_mfem_source_breaks_gauss():
    """NM-MFEM with the current sampled at t_{n+1}, t_n, t_{n-1} with weights 1/4, 1/2, 1/4
    (eq. (badNmB)) instead of -(G^{n+1} - G^{n-1}): the Gauss residual drifts."""
    osim = _beam("nm_mfem")
    m = osim.mesh
    ie, ni = m.interior_edges, m.interior_nodes
    dt = 1e-10
    A = newmark.newmark_operators(osim.Mi, osim.Si, dt, 0.25, 0.5)[0]
    dG_old2 = np.zeros(m.n_edges)
    worst = 0.0
    for k in range(10):
        dG_new, _ = osim.push_particles(dt)
        rhs = mfem.nm_rhs(osim.M, osim.S, osim.CtMf, dt, osim.e, osim.e_prev, osim.b, osim.b_prev, dG_new, osim.dG)
        # replace -(dG_new + dG_old) by -2 (dG_new / 4 + dG_old / 2 + dG_older / 4)
        rhs += (dG_new + osim.dG) - (0.5 * dG_new + osim.dG + 0.5 * dG_old2)
        xi, _, _ = newmark.pcg_jacobi(A, rhs[ie], osim.e[ie], 1e-12, 10000)
        e_new = np.zeros(m.n_edges)
        e_new[ie] = xi
        b_new = mfem.nm_faraday(osim.C, dt, osim.b_prev, e_new, osim.e, osim.e_prev)
        osim.e_prev, osim.e = osim.e, e_new
        osim.b_prev, osim.b = osim.b, b_new
        dG_old2, osim.dG = osim.dG, dG_new
        rho = osim.charge()
        r_g = -(osim.D.T @ (osim.M @ osim.e))[ni] - rho[ni]
        worst = max(worst, np.abs(r_g).max() / max(np.abs(rho[ni]).max(), 5e4 * Q_E))
    assert worst > 1e-6
