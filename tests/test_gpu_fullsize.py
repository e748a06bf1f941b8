"""The single-solve workload at full size (801 x 401 cells, nb 20, 2000 steps,
401 receivers per shot) in the launch configuration the bench times: 32
point-source shots in one forward launch for the observed data, and groups of
16 shots per launch, two time steps per launch, for the normal operator and
CG.  Sampled shots are compared with the FP64 oracle, which runs one full-size
propagation in a few seconds on the host cores.

Tolerances as for the small sizes: modelling and N p 1e-5, p.Np 1e-7 (a float64
sum of 642 M float32 products), CG iterate 1e-4.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core
from paper_2211_06300_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GROUP = 16


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def esi():
    from paper_2211_06300_amd import esi as _esi
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    _esi.load_library()
    return _esi


@pytest.fixture(scope="module")
def work():
    cfg = inputs.cfg_single_solve()
    g = core.Grid(2, cfg.nz, cfg.nx, nb=cfg.nb, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt)
    return cfg, g, core.make_model(g, cfg.v_true), core.make_model(g, cfg.v_start)


def _release():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_fullsize_forward_32_shots(esi, work):
    """The observed-data launch: 32 shots of point sources in one call; the
    first and the last shot against the oracle."""
    cfg, g, mt, _ = work
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(DEV))
    wav = torch.from_numpy(np.tile(cfg.wavelet, (cfg.nshots, 1))).to(DEV)
    d = plan.forward(wav, esi.SRC_POINT).cpu().numpy()
    plan.close()
    nrec = int(cfg.rec_ptr[1] - cfg.rec_ptr[0])
    d = d.reshape(cfg.nshots, cfg.nt, nrec)
    for s in (0, cfg.nshots - 1):
        ref = core.forward(mt, cfg.wavelet.astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
        assert _rel(d[s], ref) < 1e-5, s
    _release()


def test_fullsize_normal_apply_group(esi, work):
    """N p and p.Np for a group of 16 shots in one launch series; shots 0 and
    15 against the oracle (the same seeded p for every shot: the systems are
    independent, and the shots differ in source and receivers' reach)."""
    cfg, g, _, m0 = work
    p1 = inputs.random_field((1, cfg.nt, cfg.nz, cfg.nx), 91)
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(DEV))
    p = torch.from_numpy(p1).to(DEV).expand(GROUP, -1, -1, -1).contiguous()
    Np, pAp = plan.normal_apply(p, shot0=0, nshots=GROUP)
    pAp = pAp.cpu().numpy()
    got = {s: Np[s].cpu().numpy() for s in (0, GROUP - 1)}
    del p, Np
    plan.close()
    _release()
    p64 = p1[0].astype(np.float64)
    for s, Ns in got.items():
        ref = core.normal_apply(m0, cfg.shot_rec(s), core.annihilator_sq(g, cfg.src[s]), cfg.beta, p64)
        assert _rel(Ns, ref) < 1e-5, s
        ref_pAp = core.dot(p64, ref)
        assert abs(pAp[s] - ref_pAp) < 1e-7 * abs(ref_pAp), s


def test_fullsize_cg_two_iterations(esi, work):
    """Two CG iterations on a group of 16 shots (iteration 1 runs the fused
    residual update): shot 0's iterate and residual history against the
    oracle's.  Shot 0's data come from the oracle; the other shots, whose
    systems are independent of shot 0's, reuse them."""
    cfg, g, mt, m0 = work
    d0 = core.forward(mt, cfg.wavelet.astype(np.float64), cfg.shot_rec(0), src_pos=cfg.src[0])
    d0 = d0.astype(np.float32)
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(DEV))
    d = torch.from_numpy(np.tile(d0.ravel(), GROUP)).to(DEV)
    x, rep = plan.cg_solve(d, max_iter=2, shot0=0, nshots=GROUP)
    x0 = x[0].cpu().numpy()
    del x
    plan.close()
    _release()
    ref = core.esi_cg(m0, cfg.src[0], cfg.shot_rec(0), d0.astype(np.float64), cfg.beta, 2)
    assert rep["iters"] == 2
    assert _rel(x0, ref.x) < 1e-4
    np.testing.assert_allclose(rep["res_hist"][0], ref.res_hist, rtol=1e-4)
