"""The outer loop of Algorithm 2 on the GPU (esi_invert) against the FP64
oracle's loop (oracle.outer) on the same float32 data: objective, line-search
decisions, step lengths, penalty schedule and the updated model, for ESI and
WRI.

Tolerances: objective and data misfit 1e-4 (they come from 8-iteration CG
iterates), model update 1e-3 relative to the change of the model.  The inner
solves stop at 8 iterations: on these systems the FP64 CG trajectory itself
moves by percent at 15 iterations under relative perturbations of 5e-7 (the
float32 operator's rounding), against 2e-6 at 8.

The cases use beta = 100: at small beta the PENALTY gradient of a truncated
inner solve (Algorithm 2 uses lambda = beta B^T B q) does not predict the change
of the reduced objective, whose value is then dominated by the inner solve's
truncation, and line-search decisions are not a stable target.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core, outer
from paper_2211_06300_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


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


def _case(nt=300, seed=11):
    """30 x 40 grid, background 2000 m/s, a +300 m/s Gaussian anomaly at depth
    10 (its reflections reach the receivers within nt); two shots at depth 1
    with receivers along row 1."""
    nz, nx = 30, 40
    cfg = inputs.cfg_tiny(nz=nz, nx=nx, nt=nt, nb=6, nrec=5, seed=seed)
    zz, xx = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    v_bg = np.full((nz, nx), 2000.0, dtype=np.float32)
    v_true = (v_bg + 300.0 * np.exp(-((zz - 10) ** 2 + (xx - 20) ** 2) / 12.0)).astype(np.float32)
    cfg.v_true = v_true
    cfg.v_start = v_bg
    cfg.src = np.array([[8, 1], [31, 1]], dtype=np.int32)
    rec = np.stack([np.arange(nx), np.full(nx, 1)], axis=1)
    cfg.rec_ptr = np.array([0, nx, 2 * nx], dtype=np.int64)
    cfg.rec = np.concatenate([rec, rec]).astype(np.int32)
    cfg.beta = 100.0
    g = core.Grid(2, nz, nx, nb=cfg.nb, nt=nt, dx=cfg.dx, dt=cfg.dt)
    eta = core.eta_max_default(2000.0, g.nb, g.dx)       # the plan's, from the starting model
    mt = core.make_model(g, v_true.astype(np.float64), eta_max=eta)
    w = cfg.wavelet.astype(np.float64)
    d_obs = [core.forward(mt, w, rec, src_pos=tuple(cfg.src[s])).astype(np.float32) for s in range(2)]
    mask = np.ones((nz, nx), dtype=np.float32)
    mask[:3] = 0.0
    return cfg, g, eta, d_obs, mask


def _run_gpu(esi, cfg, d_obs, mask, wavelet=None, weight=None, **opts):
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(DEV))
    if weight is not None:
        plan.set_weight(weight)
    vel = torch.from_numpy(cfg.v_start.copy()).to(DEV)
    flat = torch.from_numpy(np.concatenate([d.ravel() for d in d_obs])).to(DEV)
    w = None if wavelet is None else torch.from_numpy(wavelet).to(DEV)
    rep = plan.invert(flat, vel, wavelet=w, mask=torch.from_numpy(mask).to(DEV), **opts)
    plan.close()
    return vel.cpu().numpy(), rep


def _run_oracle(cfg, g, eta, d_obs, mask, wavelet=None, cg_iters=8, beta=None, inner="cg", **opts):
    shots = [(tuple(cfg.src[s]), cfg.shot_rec(s), d_obs[s].astype(np.float64)) for s in range(2)]
    ev = outer.esi_objective(g, shots, cg_iters, eta_max=eta, mask=mask.astype(np.float64),
                             wavelet=None if wavelet is None else wavelet.astype(np.float64), inner=inner)
    m0 = 1.0 / cfg.v_start.astype(np.float64) ** 2
    return outer.minimize(ev, m0, cfg.beta if beta is None else beta,
                          outer.OuterOptions(cg_iters=cg_iters, **opts)), m0


@pytest.mark.parametrize("kind", ["esi", "wri"])
def test_objective_at_start(esi, kind):
    """outer_iters = 0: J and the data misfit of the starting model, ESI
    (eq. (esi)) and WRI (eq. (wridSf), B = I, u = A^{-1}(f + q))."""
    cfg, g, eta, d_obs, mask = _case()
    w = np.stack([cfg.wavelet, cfg.wavelet]).astype(np.float32) if kind == "wri" else None
    weight = esi.WEIGHT_IDENTITY if kind == "wri" else None
    _, rep = _run_gpu(esi, cfg, d_obs, mask, wavelet=w, weight=weight, outer_iters=0, cg_iters=8)
    ref, _ = _run_oracle(cfg, g, eta, d_obs, mask, wavelet=w, outer_iters=0)
    assert rep["evals"] == 1 and rep["outer_done"] == 0
    # WRI fits the data to ~1e-3: S(f + q) - d cancels, so float32 data error
    # (~1e-6 of ||d||) weighs in relative to the misfit
    tol = 1e-4 + 2e-6 / ref.misfit[0]
    assert abs(rep["J"][0] - ref.J[0]) < tol * ref.J[0]
    assert abs(rep["misfit"][0] - ref.misfit[0]) < tol * ref.misfit[0]


def test_esi_outer_loop_matches_oracle(esi):
    """Two outer iterations: the same accepted steps, trials and objective
    history, and the same model update."""
    cfg, g, eta, d_obs, mask = _case()
    opts = dict(outer_iters=2, first_step=0.03)
    vel, rep = _run_gpu(esi, cfg, d_obs, mask, cg_iters=8, **opts)
    ref, m0 = _run_oracle(cfg, g, eta, d_obs, mask, **opts)
    assert rep["status"] == 0 and ref.status == "ok"
    assert rep["trials"] == ref.trials
    assert rep["evals"] == ref.evals
    np.testing.assert_allclose(rep["step"], ref.step, rtol=1e-4)
    np.testing.assert_allclose(rep["J"], ref.J, rtol=1e-4)
    m = 1.0 / vel.astype(np.float64) ** 2
    assert _rel(m - m0, ref.m - m0) < 1e-3
    assert np.all(vel[:3] == cfg.v_start[:3])           # masked rows keep their model
    assert rep["J"][-1] < rep["J"][0]


def test_scaled_inner_solver_matches_oracle(esi):
    """Inner solves by flexible CG with the cell scale 1 / (beta B^2 + 0.03):
    objective at the start and one outer iteration."""
    cfg, g, eta, d_obs, mask = _case()
    opts = dict(outer_iters=1, first_step=0.03)
    vel, rep = _run_gpu(esi, cfg, d_obs, mask, cg_iters=8, inner=esi.INNER_FCG_SCALE, **opts)
    ref, m0 = _run_oracle(cfg, g, eta, d_obs, mask, inner="fcg", **opts)
    assert rep["trials"] == ref.trials and rep["status"] == 0
    np.testing.assert_allclose(rep["J"], ref.J, rtol=1e-4)
    np.testing.assert_allclose(rep["misfit"], ref.misfit, rtol=1e-4)
    m = 1.0 / vel.astype(np.float64) ** 2
    assert _rel(m - m0, ref.m - m0) < 1e-3


def test_dataspace_inner_solver_matches_oracle(esi):
    """Inner solves by the data-space CG (Sec. 5.1): two outer iterations."""
    cfg, g, eta, d_obs, mask = _case()
    opts = dict(outer_iters=2, first_step=0.03)
    vel, rep = _run_gpu(esi, cfg, d_obs, mask, cg_iters=8, inner=esi.INNER_DATASPACE, **opts)
    ref, m0 = _run_oracle(cfg, g, eta, d_obs, mask, inner="ds", **opts)
    assert rep["status"] == 0 and rep["trials"] == ref.trials
    np.testing.assert_allclose(rep["J"], ref.J, rtol=1e-4)
    np.testing.assert_allclose(rep["misfit"], ref.misfit, rtol=1e-4)
    m = 1.0 / vel.astype(np.float64) ** 2
    assert _rel(m - m0, ref.m - m0) < 1e-3


def test_outer_loop_deterministic_and_grouping(esi):
    """Two runs give the same bits; solving the shots one at a time gives the
    same result to rounding."""
    cfg, g, eta, d_obs, mask = _case()
    a, ra = _run_gpu(esi, cfg, d_obs, mask, outer_iters=1, cg_iters=8, first_step=0.03)
    b, rb = _run_gpu(esi, cfg, d_obs, mask, outer_iters=1, cg_iters=8, first_step=0.03)
    assert ra["status"] == 0 and ra["outer_done"] == 1
    assert np.array_equal(a, b) and ra["J"] == rb["J"]
    c, rc = _run_gpu(esi, cfg, d_obs, mask, outer_iters=1, cg_iters=8, first_step=0.03, shot_group=1)
    np.testing.assert_allclose(rc["J"], ra["J"], rtol=1e-6)
    m0 = 1.0 / cfg.v_start.astype(np.float64) ** 2
    dm = 1.0 / a.astype(np.float64) ** 2 - m0
    assert np.linalg.norm(dm) > 0
    assert _rel(1.0 / c.astype(np.float64) ** 2 - m0, dm) < 1e-4


def test_discrepancy_rule_matches_oracle(esi):
    """With a band above the starting misfit the rule raises beta as the
    oracle does (same number of changes, same beta)."""
    cfg, g, eta, d_obs, mask = _case(nt=80)
    _, r0 = _run_gpu(esi, cfg, d_obs, mask, outer_iters=0, cg_iters=8)
    e0 = r0["misfit"][0]
    opts = dict(outer_iters=1, beta_rule=1, misfit_lo=1.5 * e0, misfit_hi=3.0 * e0, beta_tries=3,
                first_step=0.03)
    _, rep = _run_gpu(esi, cfg, d_obs, mask, cg_iters=8, **opts)
    opts["beta_rule"] = "discrepancy"
    ref, _ = _run_oracle(cfg, g, eta, d_obs, mask, cg_iters=8, **opts)
    np.testing.assert_allclose(rep["beta_iter"], ref.beta_iter, rtol=1e-12)
    assert rep["beta_iter"][0] > cfg.beta
    assert rep["evals"] == ref.evals


def test_invert_argument_errors(esi):
    cfg, g, eta, d_obs, mask = _case(nt=20)
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(DEV))
    vel = torch.from_numpy(cfg.v_start.copy()).to(DEV)
    flat = torch.from_numpy(np.concatenate([d.ravel() for d in d_obs])).to(DEV)
    for bad in [dict(cg_iters=0), dict(v_min=3000.0, v_max=2000.0), dict(beta_factor=1.0),
                dict(armijo_c1=1.5), dict(beta_rule=5)]:
        with pytest.raises(esi.EsiError):
            plan.invert(flat, vel, outer_iters=1, **bad)
    # any finite beta is accepted (a negative one makes the normal operator
    # indefinite, which CG reports as a breakdown); a non-finite one is not
    for beta in (float("nan"), float("inf")):
        with pytest.raises(esi.EsiError):
            plan.set_beta(beta)
    plan.close()
