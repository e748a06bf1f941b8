"""What the trained preconditioner gains over the method without it: on a
held-out model (seed 6001, 401 x 201, 2 shots, 1500 steps) flexible CG with
the learned correction reaches a relative residual of 1e-3 (true residual
included) within 400 iterations, and plain CG (Algorithm 1) does not reach
it in the same budget or wall time.  The analytic scale alone is run and
printed beside them."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2211_06300_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2211_06300_amd", "weights", "precond_unet.npy")


@pytest.fixture(scope="module")
def esi():
    from paper_2211_06300_amd import esi as _esi
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    _esi.load_library()
    return _esi


def test_learned_preconditioner_gain(esi):
    from paper_2211_06300_amd import precond
    theta = torch.from_numpy(np.load(WEIGHTS)).to(DEV)
    cfg = inputs.cfg_precond(6001, nshots=2)
    out = precond.compare_solvers(cfg, theta, rtol=1e-3, max_iter=400, log=print)
    print(json.dumps(out))
    plain, lrn = out["plain"], out["learned"]
    assert lrn["converged"] and not plain["converged"]
    assert sum(lrn["iters"]) < sum(plain["iters"])
    assert lrn["seconds"] < plain["seconds"]
    assert max(lrn["true_residual"]) < 1.5e-3 < min(plain["true_residual"])
