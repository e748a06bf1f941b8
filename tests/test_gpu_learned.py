"""What the trained preconditioner gains over the method without it, on a
held-out model (seed 6003, 801 x 401, 2 shots, 2000 steps, not in training):

* flexible CG with the learned correction (the network re-evaluated every
  10 iterations) reaches a relative residual of 1e-3, true residual included;
* it needs fewer iterations and less wall time than flexible CG with the
  analytic scale alone (the method without the network), and no shot gives
  up the network on the way;
* plain CG (Algorithm 1) does not reach the tolerance in 400 iterations (in
  float32 it stalls near a relative residual of 1e-2 on these systems)."""
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
    cfg = inputs.cfg_precond(6003, nx=801, nz=401, nshots=2, nt=2000)
    out = precond.compare_solvers(cfg, theta, rtol=1e-3, max_iter=500, plain_max_iter=400, log=print)
    print(json.dumps(out))
    plain, an, lrn = out["plain"], out["analytic"], out["learned"]
    assert lrn["converged"] and an["converged"] and not plain["converged"]
    assert max(lrn["true_residual"]) < 1.5e-3 < min(plain["true_residual"])
    assert sum(lrn["iters"]) < sum(an["iters"])
    assert lrn["seconds"] < an["seconds"]
    assert all(f == -1 for f in lrn["fallback"]), lrn["fallback"]
