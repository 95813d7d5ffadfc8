"""The learned warm start's study protocol (paper_2102_06248_amd/ws_study.py) on a small
plasma ball: record plain solves over training seeds with one edge in two per snapshot,
train on the GPU, then advance held-out seeds from e^n, from the quadratic extrapolation
and from the network side by side.  Every solve reaches the same residual 1e-10 (the
study raises otherwise) and the fields of the learned and plain runs agree; the measured
iterations and Newmark times of the three starts are reported, whatever they show."""
import numpy as np
import pytest

from gpu_common import announce, have_gpu, require_lib
from paper_2102_06248_amd import ws_study

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    if not have_gpu():
        pytest.fail("GPU tests need an MI355X")
    return require_lib()


def test_small_study(F, tmp_path):
    announce("learned warm start study, small plasma ball")
    res = ws_study.run([1, 2, 3], 60, [11], 40, stride=2, epochs=4, n_pairs=100_000, n_cells=16,
                       workdir=str(tmp_path))
    # steps whose target RMS exceeds 10 (a history near zero) are left out
    assert 3 * 60 - 3 <= res["recorded_solves"] <= 3 * 60
    assert res["train_rows"] > 0 and np.isfinite(res["train_loss"]) and np.isfinite(res["val_loss"])
    seed = res["per_seed"][0]
    assert seed["fields_rel_diff_learned_vs_plain"] <= 1e-6
    print(f"\n[ws study small] iterations {res['cg_iters']}, Newmark ms {res['newmark_ms']}, "
          f"validation loss {res['val_loss']:.3g}")
