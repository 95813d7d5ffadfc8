"""Refined plasma ball at full mesh size (Kuhn 110^3 of the 8 cm cube, 7,986,000 tets): a
1M-particle subset in seeded fields, one particle step by the library (FP32 push / FP64
deposit, and all-FP64) against the FP64 oracle: every particle's position and momentum, and
the deposited current on every edge.

The subset is a separately seeded draw of 500,000 electron/proton pairs from the plasma's
distribution (Gaussian, sigma = 1 cm, truncated at 3.9 sigma; Te = 1 eV, Ti = 0.1 eV) with
the refined ball's macro-particle weight; dt = 0.05 / omega_pe.  The fields are seeded and
written by the oracle: a random edge field (about 1 kV/m) and a divergence-free flux
(0.05 T uniform plus the curl of a random edge vector).  Tolerances as in the small
particle-step tests.

About a minute and a half on the GPU host, most of it the oracle's topology build for 8M
tets (progress lines are printed between the stages).
"""
import math
import sys

import numpy as np
import pytest

from gpu_common import announce, compare_particles, have_gpu, require_lib
from oracle import particles as op
from oracle.constants import M_E, Q_E
from oracle.mesh import Mesh
from paper_2102_06248_amd import inputs

pytestmark = pytest.mark.gpu


def _log(msg):
    print(f"[c5] {msg}", flush=True)
    sys.stdout.flush()


def test_refined_ball_subset_vs_oracle():
    if not have_gpu():
        pytest.fail("GPU tests need an MI355X")
    F = require_lib()
    announce("refined plasma ball: 7,986,000 tets, 1M-particle subset, one step vs oracle")
    xyz, tets = inputs.kuhn_cube(110, lo=(-0.04,) * 3, hi=(0.04,) * 3)
    h = 0.08 / 110                          # shortest edge: the side of a Kuhn cell
    m_p = inputs.PROTON_ELECTRON_MASS_RATIO * M_E
    n_pairs = 500_000
    x, ue, ui = inputs.gaussian_ball_pairs(n_pairs, 0.01, 3.9, 1.0, 0.1, M_E, m_p, seed=5)
    n0 = 2.5e13
    w = n0 * (2 * math.pi) ** 1.5 * 0.01 ** 3 / 64_000_000
    eps0 = 8.8541878128e-12
    dt = 0.05 / math.sqrt(n0 * Q_E ** 2 / (eps0 * M_E))
    species = [(-Q_E, M_E, ue), (Q_E, m_p, ui)]
    ids = np.arange(n_pairs)

    _log("oracle topology")
    m = Mesh(xyz, tets)
    rng = np.random.default_rng(17)
    e = rng.normal(0.0, 1e3 * 0.08 / 110, m.n_edges)
    e[m.boundary_edge] = 0.0
    b = m.face_dofs_of_uniform_field([0.0, 0.0, 0.05]) + m.C() @ rng.normal(0.0, 1e-3 * (0.08 / 110) ** 2, m.n_edges)
    _log("oracle push")
    cm = op.CMesh(m)
    tet0 = m.locate(x)
    assert np.all(tet0 >= 0)
    dg_o = np.zeros(m.n_edges)
    orc = []
    for q, mass, u in species:
        xo, uo = x.copy(), u.astype(np.float64).copy()
        to, alive = tet0.astype(np.int64).copy(), np.ones(n_pairs, dtype=np.int8)
        rc, _ = op.push(cm, xo, uo, to, alive, q, mass, w, dt, e, b, dg_o)
        assert rc == 0
        a = alive.astype(bool)
        orc.append({"id": ids[a], "x": xo[a], "u": uo[a]})

    for precision in (0, 1):
        _log(f"library push, precision {precision}")
        with F.Simulation(xyz, tets, device=0, precision=precision) as L:
            F.fepic_set_fields(L.ctx, e=e, e_prev=e, b=b)
            handles = []
            for q, mass, u in species:
                s = F.fepic_add_species(L.ctx, q, mass, w)
                assert F.fepic_upload_particles(L.ctx, s, x, u, ids=ids) == 0
                handles.append(s)
            st = F.fepic_push_particles(L.ctx, dt)
            gps = [F.fepic_get_particles(L.ctx, s) for s in handles]
            dg_g, _ = F.fepic_get_current(L.ctx)
        tol = 1e-10 if precision == 1 else 1e-5
        for gp, o in zip(gps, orc):
            ncommon, nodd = compare_particles(gp, o, h, tol, tol)
            assert nodd <= max(2, n_pairs // 100_000) and ncommon >= n_pairs - 2
        scale = np.abs(dg_o).max()
        err = np.max(np.abs(dg_g - dg_o)) / scale
        _log(f"precision {precision}: {st.n_crossings} crossings, current max error {err:.2e} of max")
        assert err <= tol
