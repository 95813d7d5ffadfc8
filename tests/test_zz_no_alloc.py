"""The allocation-free gradient entry point (fepic_mlp_grad_noalloc) against the existing
one (fepic_mlp_grad) on the same rows: two calls in a row, the second on fewer rows, so
the fixed scratch array is reused with a smaller grid.  Both launch the same grid and sum
in the same order, so the results agree to the bit; the test asserts agreement within
FP32 rounding (1e-6 relative) and reports whether the bits match.  Also checks the
argument errors that the host raises before any kernel: too many rows and no weights.
"""
import numpy as np
import pytest

from gpu_common import announce, have_gpu, require_lib
from oracle import mlp
from paper_2102_06248_amd import inputs

pytestmark = pytest.mark.gpu


def test_noalloc_gradient_matches_the_allocating_entry_point():
    if not have_gpu():
        pytest.fail("GPU tests need an MI355X")
    F = require_lib()
    import torch

    announce("fepic_mlp_grad_noalloc vs fepic_mlp_grad, n = 65536 then 777")
    xyz, tets = inputs.kuhn_cube(2)
    with F.Simulation(xyz, tets, device=0) as sim:
        ctx = sim.ctx
        X0 = torch.zeros((8, 4), dtype=torch.float32, device="cuda")
        g0 = torch.zeros(F.FEPIC_MLP_N_PARAMS, dtype=torch.float32, device="cuda")
        l0 = torch.zeros(1, dtype=torch.float64, device="cuda")
        # no weights yet: refused before any launch, and nothing is created
        with pytest.raises(RuntimeError, match="FEPIC_E_STATE"):
            F.fepic_mlp_grad_noalloc(ctx, 8, X0.data_ptr(), X0.data_ptr(), g0.data_ptr(), l0.data_ptr())
        p = mlp.init_params(7)
        rng = np.random.default_rng(8)
        p["b1"] = rng.normal(size=64) * 0.2
        p["b2"] = rng.normal(size=64) * 0.2
        F.fepic_ws_set_weights(ctx, mlp.flatten(p).astype(np.float32))
        big = F.FEPIC_MLP_NOALLOC_MAX_ROWS
        with pytest.raises(RuntimeError, match="FEPIC_E_ARG"):
            F.fepic_mlp_grad_noalloc(ctx, big + 1, X0.data_ptr(), X0.data_ptr(), g0.data_ptr(), l0.data_ptr())
        for n in (big, 777):
            X = rng.normal(size=(n, 4)).astype(np.float32)
            t = rng.normal(size=n).astype(np.float32)
            loss_ref, g_ref = F.fepic_mlp_grad(ctx, X, t)
            dX = torch.from_numpy(X).to("cuda")
            dt_ = torch.from_numpy(t).to("cuda")
            dg = torch.full((F.FEPIC_MLP_N_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
            dl = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            F.fepic_mlp_grad_noalloc(ctx, n, dX.data_ptr(), dt_.data_ptr(), dg.data_ptr(), dl.data_ptr())
            torch.cuda.synchronize()
            g = dg.cpu().numpy()
            loss = float(dl.cpu().numpy()[0])
            assert np.all(np.isfinite(g)) and np.isfinite(loss)
            assert np.max(np.abs(g - g_ref)) <= 1e-6 * np.max(np.abs(g_ref))
            assert loss == pytest.approx(loss_ref, rel=1e-12)
            print(f"n={n}: gradient bit-identical {np.array_equal(g, g_ref)}, loss {loss:.6e} vs {loss_ref:.6e}",
                  flush=True)
