"""GPU tests of the learned warm start: BF16 matrix-core forward and gradient kernels
against the FP64 oracle network, and training on recorded Newmark solves.

Tolerances: BF16 operands carry 8 significant bits (relative rounding 2^-9); layer 2 sums
64 such products in FP32, so outputs and gradients agree with FP64 to about 1e-2
relative; the tests use 2e-2 on outputs/loss and 3e-2 on each gradient block.
"""
import numpy as np
import pytest

from gpu_common import announce, have_gpu, require_lib
from oracle import mlp
from oracle.constants import M_E, Q_E
from paper_2102_06248_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    if not have_gpu():
        pytest.fail("GPU tests need an MI355X")
    return require_lib()


@pytest.fixture(scope="module")
def small_sim(F):
    xyz, tets = inputs.kuhn_cube(2)
    sim = F.Simulation(xyz, tets, device=0)
    yield sim
    sim.close()


def _params(seed):
    p = mlp.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    p["b1"] = rng.normal(size=64) * 0.2
    p["b2"] = rng.normal(size=64) * 0.2
    p["b3"] = rng.normal(size=1) * 0.2
    p["W3"] = rng.normal(size=(1, 64)) * 0.3
    return p


def _set(F, sim, p):
    F.fepic_ws_set_weights(sim.ctx, mlp.flatten(p).astype(np.float32))
    # the library stores FP32 masters: compare against the oracle on the same FP32 values
    return mlp.unflatten(F.fepic_ws_get_weights(sim.ctx).astype(np.float64))


@pytest.mark.parametrize("n", [1, 16, 1037])
def test_forward_matches_oracle(F, small_sim, n):
    announce(f"mlp forward n={n}")
    p = _set(F, small_sim, _params(3))
    X = np.random.default_rng(4).normal(size=(n, 4)).astype(np.float32)
    y = F.fepic_mlp_forward(small_sim.ctx, X)
    yo, _ = mlp.forward(p, X.astype(np.float64))
    assert np.linalg.norm(y - yo) <= 2e-2 * np.linalg.norm(yo)


@pytest.mark.parametrize("n", [32, 777])
def test_gradient_matches_oracle(F, small_sim, n):
    announce(f"mlp gradient n={n}")
    p = _set(F, small_sim, _params(5))
    rng = np.random.default_rng(6)
    X = rng.normal(size=(n, 4)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    loss, g = F.fepic_mlp_grad(small_sim.ctx, X, t)
    Lo, go = mlp.loss_and_grad(p, X.astype(np.float64), t.astype(np.float64))
    assert loss == pytest.approx(Lo, rel=2e-2)
    gu = mlp.unflatten(g.astype(np.float64))
    for name, _ in mlp.SHAPES:
        ref = go[name]
        assert np.linalg.norm(gu[name] - ref) <= 3e-2 * np.linalg.norm(ref) + 1e-7, name


def _beam_ctx(F, **opts):
    xyz, tets = inputs.prism_cylinder(0.05, 0.5, 6, 20)
    sim = F.Simulation(xyz, tets, device=0, **opts)
    x, u = inputs.beam_particles(20000, 0.01, 0.0, 0.5, 1000.0, 1.0, M_E, seed=11)
    sp = F.fepic_add_species(sim.ctx, -Q_E, M_E, 2e5)
    F.fepic_upload_particles(sim.ctx, sp, x, u, ids=np.arange(len(x)))
    F.fepic_init_electrostatic(sim.ctx, 1e-12)
    return sim


def test_training_and_warm_start_gain(F):
    """Record solves, train on the GPU, then run the same continuation with and without
    the network: both reach the same tolerance; the iteration counts are reported (the
    plasma study, test_gpu_ws_study.py, measures the gain on held-out seeds)."""
    announce("mlp training on recorded Newmark solves")
    dt = 1e-10
    plain = _beam_ctx(F)
    learned = _beam_ctx(F)
    F.fepic_ws_record(learned.ctx, 1, 64)
    for _ in range(40):
        F.fepic_step(plain.ctx, dt)
        F.fepic_step(learned.ctx, dt)
    assert F.fepic_ws_num_snapshots(learned.ctx) == 40
    F.fepic_ws_record(learned.ctx, 0)
    st = F.fepic_ws_train(learned.ctx, epochs=6, batch=8192, lr=2e-3, seed=1, val_fraction=0.25)
    print(f"\n[mlp] train loss {st.train_loss:.4g}, val loss {st.val_loss:.4g}, {st.n_steps} Adam steps, "
          f"{st.n_train_rows} rows, {st.ms_total:.0f} ms")
    assert np.isfinite(st.train_loss) and np.isfinite(st.val_loss)
    F.fepic_set_warm_start(learned.ctx, F.FEPIC_WS_MLP)
    it_plain, it_mlp, r0_plain, r0_mlp = [], [], [], []
    for _ in range(20):
        a = F.fepic_step(plain.ctx, dt)
        b = F.fepic_step(learned.ctx, dt)
        it_plain.append(a.cg_iters)
        it_mlp.append(b.cg_iters)
        r0_plain.append(a.cg_rel_resid0)
        r0_mlp.append(b.cg_rel_resid0)
        assert a.cg_rel_resid <= 1e-10 and b.cg_rel_resid <= 1e-10
    print(f"[mlp] mean CG iterations: plain {np.mean(it_plain):.1f}, learned {np.mean(it_mlp):.1f}; "
          f"initial residual: plain {np.mean(r0_plain):.3g}, learned {np.mean(r0_mlp):.3g}")
    e1, _, _ = F.fepic_get_fields(plain.ctx)
    e2, _, _ = F.fepic_get_fields(learned.ctx)
    assert np.linalg.norm(e1 - e2) <= 1e-6 * np.linalg.norm(e1)
    # the same continuation with the mixed-precision solve (the network's start passes the
    # same guard before the first FP32 pass)
    for sim in (plain, learned):
        F.fepic_set_solve_precision(sim.ctx, F.FEPIC_SOLVE_MIXED)
    for _ in range(5):
        a = F.fepic_step(plain.ctx, dt)
        b = F.fepic_step(learned.ctx, dt)
        assert a.cg_rel_resid <= 1e-10 and b.cg_rel_resid <= 1e-10
        assert a.cg_passes >= 1 and b.cg_passes >= 1
    e1, _, _ = F.fepic_get_fields(plain.ctx)
    e2, _, _ = F.fepic_get_fields(learned.ctx)
    assert np.linalg.norm(e1 - e2) <= 1e-6 * np.linalg.norm(e1)
    plain.close()
    learned.close()


def test_checkpoint_round_trip(F, tmp_path):
    announce("checkpoint save/load")
    dt = 1e-10
    a = _beam_ctx(F, precision=1)
    for _ in range(3):
        F.fepic_step(a.ctx, dt)
    path = str(tmp_path / "ck.bin")
    F.fepic_save(a.ctx, path)
    for _ in range(3):
        F.fepic_step(a.ctx, dt)
    ea, _, ba = F.fepic_get_fields(a.ctx)
    pa = F.fepic_get_particles(a.ctx, 0)
    xyz, tets = inputs.prism_cylinder(0.05, 0.5, 6, 20)
    b = F.Simulation(xyz, tets, device=0, precision=1)
    F.fepic_add_species(b.ctx, -Q_E, M_E, 2e5)
    F.fepic_load(b.ctx, path)
    for _ in range(3):
        F.fepic_step(b.ctx, dt)
    eb, _, bb = F.fepic_get_fields(b.ctx)
    pb = F.fepic_get_particles(b.ctx, 0)
    assert np.linalg.norm(ea - eb) <= 1e-9 * np.linalg.norm(ea)
    ia, ib = np.argsort(pa["id"]), np.argsort(pb["id"])
    assert np.array_equal(pa["id"][ia], pb["id"][ib])
    assert np.max(np.abs(pa["x"][ia] - pb["x"][ib])) <= 1e-12
    a.close()
    b.close()


def test_injection_matches_upload(F):
    """Particles injected between steps (no sort, no host wait) from host arrays or device
    memory, and particles uploaded from device memory, give the same state as the same
    particles uploaded from host arrays, and as the oracle."""
    announce("injection vs upload")
    import torch
    from oracle.pic import OracleSim
    xyz, tets = inputs.prism_cylinder(0.05, 0.5, 6, 20)
    osim = OracleSim(xyz, tets)
    so = osim.add_species(-Q_E, M_E, 2e5)
    sims = [F.Simulation(xyz, tets, device=0, precision=1) for _ in range(4)]
    sps = [F.fepic_add_species(s.ctx, -Q_E, M_E, 2e5) for s in sims]
    nid = 0
    for k in range(4):
        x, u = inputs.beam_particles(500, 0.01, 0.0, 0.0, 1000.0, 1.0, M_E, seed=100 + k)
        ids = np.arange(nid, nid + len(x))
        nid += len(x)
        F.fepic_upload_particles(sims[0].ctx, sps[0], x, u, ids=ids)
        F.fepic_inject_particles(sims[1].ctx, sps[1], x, u, ids=ids)
        dev = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in (x, u, ids)]
        torch.cuda.synchronize()
        F.fepic_inject_particles_device(sims[2].ctx, sps[2], len(x), dev[0].data_ptr(), dev[1].data_ptr(),
                                        dev[2].data_ptr())
        assert F.fepic_upload_particles_device(sims[3].ctx, sps[3], len(x), dev[0].data_ptr(), dev[1].data_ptr(),
                                               dev[2].data_ptr()) == 0
        osim.upload_particles(so, x, u, ids=ids)
        for s in sims:
            F.fepic_step(s.ctx, 1e-10)
        del dev                       # the steps above have consumed the device arrays
        osim.step(1e-10)
    ps = [F.fepic_get_particles(s.ctx, sp) for s, sp in zip(sims, sps)]
    po = osim.particles(so)
    for p in ps:
        i, j = np.argsort(p["id"]), np.argsort(po["id"])
        assert np.array_equal(p["id"][i], po["id"][j])
        assert np.max(np.abs(p["x"][i] - po["x"][j])) <= 1e-10
    for s in sims:
        s.close()
