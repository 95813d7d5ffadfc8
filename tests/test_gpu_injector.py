"""GPU parity of the seeded disk source (fepic_set_injector) against the oracle's draws
(oracle/injector.py): the library draws every step's particles on the device from the
counter-based generator; the oracle draws the same batch on the CPU and uploads it before
its own step.  Whole steps of a small beam in a PEC cylinder (all FP64, Jacobi-PCG on both
sides), compared every step: the live particle set by id, positions (1e-10 m), momenta,
the fields (1e-6 relative), the count the step reports as injected, and continuity.
A step that fails commits none of its injected particles and does not count the
injection: the next successful step injects batch 0 again.
"""
import numpy as np
import pytest

from gpu_common import announce, have_gpu, require_lib
from oracle import injector as inj
from oracle.constants import M_E, Q_E
from oracle.pic import OracleSim
from paper_2102_06248_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    if not have_gpu():
        pytest.fail("GPU tests need an MI355X")
    return require_lib()


SPEC = dict(center=[0.0, 0.0, 0.0], normal=[0.0, 0.0, 1.0], radius=0.01, kinetic_eV=1000.0, thermal_eV=1.0,
            per_step=400, seed=2024)


def _set(F, ctx, s, spec):
    F.fepic_set_injector(ctx, s, center=spec["center"], normal=spec["normal"], radius=spec["radius"],
                         kinetic_eV=spec["kinetic_eV"], thermal_eV=spec["thermal_eV"], per_step=spec["per_step"],
                         seed=spec["seed"])


def test_injector_steps_vs_oracle(F):
    announce("disk injector: 8 whole steps vs oracle")
    xyz, tets = inputs.prism_cylinder(0.05, 0.1, 4, 12)
    dt, w = 1e-10, 2e5
    osim = OracleSim(xyz, tets)
    so = osim.add_species(-Q_E, M_E, w)
    interior = ~osim.mesh.boundary_node
    with F.Simulation(xyz, tets, device=0, precision=F.FEPIC_ALL_FP64, diagnostics=1,
                      preconditioner=F.FEPIC_PC_JACOBI) as L:
        s = F.fepic_add_species(L.ctx, -Q_E, M_E, w)
        _set(F, L.ctx, s, SPEC)
        for k in range(8):
            x, u = inj.disk_batch(SPEC, k, 0, M_E)
            n = SPEC["per_step"]
            assert osim.upload_particles(so, x, u, ids=np.arange(k * n, (k + 1) * n)) == 0
            ost = osim.step(dt)
            st = F.fepic_step(L.ctx, dt)
            assert st.n_injected == n
            assert st.cont_resid_rel <= 1e-12 and ost["cont_resid_rel"] <= 1e-12
            gp = F.fepic_get_particles(L.ctx, s)
            op_ = osim.particles(so)
            gi, oi = np.argsort(gp["id"]), np.argsort(op_["id"])
            assert np.array_equal(gp["id"][gi], op_["id"][oi]), k
            assert np.abs(gp["x"][gi] - op_["x"][oi]).max() <= 1e-10, k
            assert np.abs(gp["u"][gi] - op_["u"][oi]).max() <= 1e-9 * np.abs(op_["u"]).max(), k
            e, _, _ = F.fepic_get_fields(L.ctx)
            assert np.linalg.norm(e - osim.e) <= 1e-6 * np.linalg.norm(osim.e), k
            rho = F.fepic_get_rho(L.ctx, osim.mesh.n_nodes)
            assert np.abs(rho - osim.rho).max() <= 1e-12 * abs(Q_E * w) * 50
        assert len(gp["id"]) > 6 * SPEC["per_step"]
        print(f"\n[injector] {len(gp['id'])} particles after 8 steps, continuity {st.cont_resid_rel:.1e}")


def test_failed_step_injects_nothing(F):
    announce("disk injector: a failed step commits none of its particles")
    xyz, tets = inputs.prism_cylinder(0.05, 0.1, 4, 12)
    spec = dict(SPEC, kinetic_eV=1e6, thermal_eV=0.0, per_step=50)
    with F.Simulation(xyz, tets, device=0, precision=F.FEPIC_ALL_FP64, crossing_cap=2) as L:
        s = F.fepic_add_species(L.ctx, -Q_E, M_E, 1.0)
        _set(F, L.ctx, s, spec)
        # 1 MeV electrons cross many cells in 0.1 ns: past the cap, the step fails
        with pytest.raises(F.FepicError) as ei:
            F.fepic_push_particles(L.ctx, 1e-10)
        assert F.ERROR_NAMES[ei.value.code] == "FEPIC_E_CROSSING_CAP"
        assert F.fepic_num_particles(L.ctx, s) == 0
        # a short step succeeds and injects batch 0 (not batch 1); with no fields, u is kept
        st = F.fepic_push_particles(L.ctx, 1e-13)
        assert st.n_injected == 50 and st.n_cap_exceeded == 0
        gp = F.fepic_get_particles(L.ctx, s)
        x0, u0 = inj.disk_batch(spec, 0, 0, M_E)
        gi = np.argsort(gp["id"])
        assert np.array_equal(gp["id"][gi], np.arange(50))
        assert np.abs(gp["u"][gi] - u0).max() <= 1e-12 * np.abs(u0).max()
        g = np.sqrt(1 + np.sum(u0 ** 2, axis=1) / 299792458.0 ** 2)
        assert np.abs(gp["x"][gi] - (x0 + 1e-13 * u0 / g[:, None])).max() <= 1e-15
        # switched off: the next step adds nothing
        F.fepic_set_injector(L.ctx, s, off=True)
        st = F.fepic_push_particles(L.ctx, 1e-13)
        assert st.n_injected == 0 and F.fepic_num_particles(L.ctx, s) == 50
        with pytest.raises(F.FepicError):
            F.fepic_set_injector(L.ctx, s, center=[0, 0, 0], normal=[0, 0, 0], radius=0.01, per_step=1)
