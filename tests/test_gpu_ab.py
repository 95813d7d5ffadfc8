"""GPU parity of the Adams-Bashforth pusher (fepic_push_particles_ab) against the oracle's
(oracle/ab.py): the same seeded particles in the same seeded fields, stepped with orders 1
to 5 for enough steps that the history reaches the full order.  Every step compares every
particle's position and velocity, the absorbed set, and the deposited current on every
edge, and checks charge continuity D^T dG = rho^{n+1} - rho^n on the library's own state.
"""
import numpy as np
import pytest

from gpu_common import announce, divfree_fields, have_gpu, jittered_kuhn, require_lib
from oracle import ab, fem
from oracle.constants import M_E, Q_E
from oracle.pic import OracleSim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    if not have_gpu():
        pytest.fail("GPU tests need an MI355X")
    return require_lib()


def _oracle_steps(m, e, b, x, v, q, mass, w, dt, order, n_steps):
    """Per particle: the oracle's AB step, curved walk and deposit; returns per step the
    alive ids, their positions and velocities, and the current vector."""
    n = len(x)
    tet = m.locate(x)
    r_hist = [[x[i].copy()] for i in range(n)]
    v_hist = [[v[i].copy()] for i in range(n)]
    a_hist = [[] for _ in range(n)]
    alive = tet >= 0
    out = []
    for _ in range(n_steps):
        g = np.zeros(m.n_edges)
        for i in range(n):
            if not alive[i]:
                continue
            t = int(tet[i])
            lam = m.barycentric(t, r_hist[i][0])
            E = fem.eval_E(m, e, t, lam)
            B = fem.eval_B(m, b, t, lam)
            vi = v_hist[i][0]
            a_hist[i].insert(0, (q / mass) * (E + np.cross(vi, B)))
            k = min(order, len(a_hist[i]))
            r_new, v_new = ab.ab_step(r_hist[i], v_hist[i], a_hist[i], dt, order)
            path = ab.step_path(r_new, r_hist[i][:k])
            pieces, last = ab.walk_curved(m, t, path, n_gl=k + 1)
            ab.deposit_curved(m, pieces, path, q * w, n_gl=k + 1, g=g)
            if last < 0:
                alive[i] = False
                continue
            tet[i] = last
            r_hist[i] = [r_new] + r_hist[i][:ab_max() - 1]
            v_hist[i] = [v_new] + v_hist[i][:ab_max() - 1]
            a_hist[i] = a_hist[i][:ab_max() - 1]
        ids = np.nonzero(alive)[0]
        out.append((ids, np.array([r_hist[i][0] for i in ids]), np.array([v_hist[i][0] for i in ids]), g))
    return out


def ab_max():
    return 5


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_ab_push_vs_oracle(F, order):
    announce(f"Adams-Bashforth pusher, order {order}")
    xyz, tets, h = jittered_kuhn(5, seed=21)
    osim = OracleSim(xyz, tets)
    m = osim.mesh
    e, b = divfree_fields(osim, 2.0, 5e-7, [0.0, 0.0, 3e-5], seed=22)
    n = 300
    rng = np.random.default_rng(23)
    x = rng.uniform(0.25, 0.75, size=(n, 3))
    v = rng.normal(0.0, 6e5, size=(n, 3))
    q, mass, w = -Q_E, M_E, 1e3
    dt = 6e-8                                   # about a third of a cell per step, w dt = 0.3 rad
    n_steps = order + 3
    ref = _oracle_steps(m, e, b, x, v, q, mass, w, dt, order, n_steps)
    interior = ~m.boundary_node
    with F.Simulation(xyz, tets, device=0, precision=F.FEPIC_ALL_FP64, sort_period=0) as L:
        F.fepic_set_fields(L.ctx, e=e, e_prev=e, b=b)
        sp = F.fepic_add_species(L.ctx, q, mass, w)
        assert F.fepic_upload_particles(L.ctx, sp, x, v, ids=np.arange(n)) == 0
        _, G_prev = F.fepic_get_current(L.ctx)
        rho_prev = F.fepic_get_rho(L.ctx, m.n_nodes)
        total_cross = 0
        for k, (ids, r_o, v_o, g_o) in enumerate(ref):
            st = F.fepic_push_particles_ab(L.ctx, sp, dt, order)
            total_cross += st.n_crossings
            gp = F.fepic_get_particles(L.ctx, sp)
            gi = np.argsort(gp["id"])
            assert np.array_equal(gp["id"][gi], ids), f"step {k}: absorbed sets differ"
            assert np.abs(gp["x"][gi] - r_o).max() <= 1e-10, f"step {k}"
            assert np.abs(gp["u"][gi] - v_o).max() <= 1e-10 * np.abs(v_o).max(), f"step {k}"
            dG, G = F.fepic_get_current(L.ctx)
            assert np.abs(dG - g_o).max() <= 1e-10 * np.abs(g_o).max(), f"step {k}"
            # continuity holds up to the walk's inside tolerance: a crossing point may sit up
            # to 1e-13 (in barycentric terms) outside its face, where the two cells'
            # barycentric coordinates differ by as much, once per crossing through a node
            rho = F.fepic_get_rho(L.ctx, m.n_nodes)
            cont = (rho - rho_prev) - osim.D.T @ (G - G_prev)
            assert np.abs(cont[interior]).max() <= 1e-13 * 200 * abs(q * w), f"step {k}"
            rho_prev, G_prev = rho, G
        assert total_cross > n
        print(f"\n[ab] order {order}: {n_steps} steps, {total_cross} crossings, {len(ref[-1][0])} of {n} left")


def test_ab_push_rejects_bad_calls(F):
    """Order outside 1..5, a non-positive dt or an unknown species is FEPIC_E_ARG; the
    pusher needs the all-FP64 particle path (FEPIC_E_STATE otherwise); nothing is pushed."""
    announce("Adams-Bashforth pusher: argument and state errors")
    xyz, tets, _ = jittered_kuhn(3, seed=5)
    x = np.full((4, 3), 0.5) + 0.01 * np.arange(12).reshape(4, 3)
    v = np.zeros((4, 3))
    for precision, bad in [(F.FEPIC_ALL_FP64, [(0, 0, 1e-9), (0, 6, 1e-9), (0, 2, 0.0), (0, 2, -1e-9), (3, 2, 1e-9)]),
                           (F.FEPIC_FP32_PUSH_FP64_ACC, [(0, 2, 1e-9)])]:
        with F.Simulation(xyz, tets, device=0, precision=precision) as L:
            sp = F.fepic_add_species(L.ctx, -1.0, 1.0, 1.0)
            F.fepic_upload_particles(L.ctx, sp, x, v, ids=np.arange(4))
            want = "FEPIC_E_ARG" if precision == F.FEPIC_ALL_FP64 else "FEPIC_E_STATE"
            for species, order, dt in bad:
                with pytest.raises(F.FepicError) as ei:
                    F.fepic_push_particles_ab(L.ctx, species, dt, order)
                assert F.ERROR_NAMES[ei.value.code] == want
            gp = F.fepic_get_particles(L.ctx, sp)
            assert np.allclose(np.sort(gp["x"], axis=0), np.sort(x, axis=0), atol=1e-12)
