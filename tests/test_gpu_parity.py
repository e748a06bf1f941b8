"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded float32 inputs.

Tolerances (relative L2 against the oracle): modelling 1e-5, adjoint dot test
1e-6, CG solutions 1e-4; gradients 1e-4 (float32 correlation sums over nt
steps).  Sizes span several 64 x 32 tiles with ragged tails.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core
from paper_2211_06300_amd import inputs

pytestmark = pytest.mark.gpu


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


DEV = "cuda:0"


def _oracle_model(cfg, v=None):
    g = core.Grid(cfg.ndim, cfg.nz, cfg.nx, ny=cfg.ny, nb=cfg.nb, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt)
    return g, core.make_model(g, cfg.v_true if v is None else v)


def _ragged_cfg(nshots=3, nt=70, seed=21):
    """37 x 70 physical, nb 8 -> 53 x 86 padded: 2 x 2 tiles with ragged tails;
    shots with different receiver sets, duplicates in one cell, corner cells and
    a shot without receivers."""
    rng = np.random.default_rng(seed)
    nz, nx = 37, 70
    cfg = inputs.cfg_tiny(nz=nz, nx=nx, nt=nt, nb=8, nrec=5, seed=seed)
    src = np.array([[5, 2], [35, 20], [69, 36]][:nshots], dtype=np.int32)
    recs = [np.array([[0, 0], [69, 0], [0, 36], [69, 36], [30, 2], [30, 2], [31, 2]]),
            np.stack([rng.integers(0, nx, 40), rng.integers(0, nz, 40)], axis=1),
            np.zeros((0, 2), dtype=np.int64)][:nshots]
    ptr = np.zeros(nshots + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in recs])
    cfg.src = src
    cfg.rec_ptr = ptr
    cfg.rec = np.concatenate(recs).astype(np.int32)
    cfg.v_true = (1800.0 + 900.0 * rng.random((nz, nx))).astype(np.float32)
    cfg.v_start = cfg.v_true
    cfg.beta = 0.05
    return cfg


def _plan(esi, cfg, v=None, **kw):
    vel = torch.from_numpy(np.ascontiguousarray(cfg.v_true if v is None else v)).to(DEV)
    return esi.Plan.from_config(cfg, vel=vel, **kw)


def _split(cfg, data_flat, shot0=0, nshots=None):
    nshots = cfg.nshots - shot0 if nshots is None else nshots
    out, off = [], 0
    for s in range(shot0, shot0 + nshots):
        n = int(cfg.rec_ptr[s + 1] - cfg.rec_ptr[s])
        out.append(data_flat[off:off + cfg.nt * n].reshape(cfg.nt, n))
        off += cfg.nt * n
    return out


def test_forward_point_small_config(esi):
    """201 x 201, v = 2000, 10 Hz Ricker at (100, 5), 201 receivers on row 5, 500 steps."""
    cfg = inputs.cfg_small()
    plan = _plan(esi, cfg)
    d = plan.forward(torch.from_numpy(cfg.wavelet[None].copy()).to(DEV), esi.SRC_POINT)
    g, m = _oracle_model(cfg)
    d_ref = core.forward(m, cfg.wavelet.astype(np.float64), cfg.shot_rec(0), src_pos=cfg.src[0])
    assert _rel(d.cpu().numpy().reshape(cfg.nt, -1), d_ref) < 1e-5


def test_forward_dense_ragged(esi):
    cfg = _ragged_cfg()
    plan = _plan(esi, cfg)
    q = inputs.random_field((cfg.nshots, cfg.nt, cfg.nz, cfg.nx), 1)
    d = plan.forward(torch.from_numpy(q).to(DEV), esi.SRC_DENSE).cpu().numpy()
    g, m = _oracle_model(cfg)
    for s, ds in enumerate(_split(cfg, d)):
        if ds.size == 0:
            continue
        ref = core.forward(m, q[s].astype(np.float64), cfg.shot_rec(s))
        assert _rel(ds, ref) < 1e-5, s


def test_adjoint_ragged(esi):
    cfg = _ragged_cfg()
    plan = _plan(esi, cfg)
    dd = inputs.random_field(plan.data_shape(), 2)
    out = plan.adjoint(torch.from_numpy(dd).to(DEV)).cpu().numpy()
    g, m = _oracle_model(cfg)
    for s, ds in enumerate(_split(cfg, dd)):
        ref = core.adjoint(m, cfg.shot_rec(s), ds.astype(np.float64))
        if ds.size == 0:
            assert np.all(out[s] == 0.0)
            continue
        assert _rel(out[s], ref) < 1e-5, s


def test_dot_test_small_config(esi):
    """<S q, d> = <q, S^T d> on the GPU in float32, judged in float64: <= 1e-6."""
    cfg = inputs.cfg_small()
    plan = _plan(esi, cfg)
    q = torch.from_numpy(inputs.random_field((1, cfg.nt, cfg.nz, cfg.nx), 0)).to(DEV)
    dd = torch.from_numpy(inputs.random_field(plan.data_shape(), 1)).to(DEV)
    Sq = plan.forward(q, esi.SRC_DENSE)
    Std = plan.adjoint(dd)
    lhs = torch.dot(Sq.double().ravel(), dd.double().ravel()).item()
    rhs = torch.dot(q.double().ravel(), Std.double().ravel()).item()
    assert abs(lhs - rhs) / max(abs(lhs), abs(rhs)) < 1e-6


def test_normal_apply_ragged(esi):
    cfg = _ragged_cfg()
    plan = _plan(esi, cfg)
    p = inputs.random_field((cfg.nshots, cfg.nt, cfg.nz, cfg.nx), 3)
    Np, pAp = plan.normal_apply(torch.from_numpy(p).to(DEV))
    Np = Np.cpu().numpy()
    pAp = pAp.cpu().numpy()
    g, m = _oracle_model(cfg)
    for s in range(cfg.nshots):
        w2 = core.annihilator_sq(g, cfg.src[s])
        ref = core.normal_apply(m, cfg.shot_rec(s), w2, cfg.beta, p[s].astype(np.float64))
        assert _rel(Np[s], ref) < 1e-5, s
        ref_pAp = core.dot(p[s].astype(np.float64), Np[s].astype(np.float64))
        assert abs(pAp[s] - ref_pAp) < 1e-9 * abs(pAp[s])


def _cg_case(esi, cfg, iters, shots=None):
    plan = _plan(esi, cfg, v=cfg.v_start)
    g, m_true = _oracle_model(cfg)
    _, m0 = _oracle_model(cfg, cfg.v_start)
    shots = range(cfg.nshots) if shots is None else shots
    d_obs = [core.forward(m_true, cfg.wavelet.astype(np.float64), cfg.shot_rec(s),
                          src_pos=cfg.src[s]).astype(np.float32) for s in shots]
    flat = np.concatenate([d.ravel() for d in d_obs]).astype(np.float32)
    x, rep = plan.cg_solve(torch.from_numpy(flat).to(DEV), max_iter=iters)
    return plan, g, m0, d_obs, x.cpu().numpy(), rep


def test_cg_small_config(esi):
    """CG, 5 iterations, beta = 1e-2 on the 201 x 201 workload: x_5 within 1e-4."""
    cfg = inputs.cfg_small()
    plan, g, m0, d_obs, x, rep = _cg_case(esi, cfg, 5)
    ref = core.esi_cg(m0, cfg.src[0], cfg.shot_rec(0), d_obs[0].astype(np.float64), cfg.beta, 5)
    assert rep["iters"] == 5
    assert _rel(x[0], ref.x) < 1e-4
    np.testing.assert_allclose(rep["res_hist"][0], ref.res_hist, rtol=1e-4)


def test_cg_multishot_ragged(esi):
    """Batched per-shot CG on shots of uneven receiver counts, one shot with no
    receivers (b = 0, x = 0)."""
    cfg = _ragged_cfg(nt=50)
    cfg.v_start = (cfg.v_true * 1.03).astype(np.float32)
    plan, g, m0, d_obs, x, rep = _cg_case(esi, cfg, 6)
    for s in range(cfg.nshots):
        if d_obs[s].size == 0:
            assert np.all(x[s] == 0.0)
            assert rep["shot_iters"][s] == 0
            continue
        ref = core.esi_cg(m0, cfg.src[s], cfg.shot_rec(s), d_obs[s].astype(np.float64), cfg.beta, 6)
        assert _rel(x[s], ref.x) < 1e-4, s


def test_cg_early_exit_per_shot(esi):
    """Each shot leaves after the iteration where ||r|| < rtol ||r0||."""
    cfg = _ragged_cfg(nshots=2, nt=40)
    plan = _plan(esi, cfg)
    g, m = _oracle_model(cfg)
    d_obs = [core.forward(m, cfg.wavelet.astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
             .astype(np.float32) for s in range(2)]
    flat = torch.from_numpy(np.concatenate([d.ravel() for d in d_obs])).to(DEV)
    x, rep = plan.cg_solve(flat, max_iter=30, rtol=0.2)
    for s in range(2):
        ref = core.esi_cg(m, cfg.src[s], cfg.shot_rec(s), d_obs[s].astype(np.float64), cfg.beta, 30,
                          rtol=0.2)
        assert rep["shot_iters"][s] == ref.iters, s
        assert _rel(x.cpu().numpy()[s], ref.x) < 1e-4


def test_cg_deterministic(esi):
    cfg = _ragged_cfg(nt=40)
    a = _cg_case(esi, cfg, 4)[4]
    b = _cg_case(esi, cfg, 4)[4]
    assert np.array_equal(a, b)


def test_gradient_penalty_ragged(esi):
    cfg = _ragged_cfg()
    plan = _plan(esi, cfg)
    q = inputs.random_field((cfg.nshots, cfg.nt, cfg.nz, cfg.nx), 4)
    gm = plan.gradient(esi.GRAD_PENALTY, torch.from_numpy(q).to(DEV)).cpu().numpy()
    g, m = _oracle_model(cfg)
    ref = sum(core.gradient_penalty(m, q[s].astype(np.float64), core.annihilator_sq(g, cfg.src[s]),
                                    cfg.beta) for s in range(cfg.nshots))
    assert _rel(gm, ref) < 1e-4


@pytest.mark.parametrize("ckpt", [0, 7])
def test_gradient_adjoint_ragged(esi, ckpt):
    cfg = _ragged_cfg()
    plan = _plan(esi, cfg)
    q = inputs.random_field((cfg.nshots, cfg.nt, cfg.nz, cfg.nx), 5)
    dd = inputs.random_field(plan.data_shape(), 6)
    gm = plan.gradient(esi.GRAD_ADJOINT, torch.from_numpy(q).to(DEV), torch.from_numpy(dd).to(DEV),
                       ckpt_every=ckpt).cpu().numpy()
    g, m = _oracle_model(cfg)
    ref = sum(core.gradient_adjoint(m, q[s].astype(np.float64), cfg.shot_rec(s),
                                    ds.astype(np.float64))
              for s, ds in enumerate(_split(cfg, dd)))
    assert _rel(gm, ref) < 1e-4


def test_gradient_checkpointed_bitwise(esi):
    """Checkpointed recompute equals full storage bit for bit (same kernels)."""
    cfg = _ragged_cfg()
    plan = _plan(esi, cfg)
    q = torch.from_numpy(inputs.random_field((cfg.nshots, cfg.nt, cfg.nz, cfg.nx), 7)).to(DEV)
    dd = torch.from_numpy(inputs.random_field(plan.data_shape(), 8)).to(DEV)
    full = plan.gradient(esi.GRAD_ADJOINT, q, dd, ckpt_every=0).cpu().numpy()
    for K in (1, 7, 25, 69):
        ck = plan.gradient(esi.GRAD_ADJOINT, q, dd, ckpt_every=K).cpu().numpy()
        assert np.array_equal(ck, full), K


def test_gradient_seed_point(esi):
    cfg = _ragged_cfg(nshots=2)
    plan = _plan(esi, cfg)
    w = np.stack([cfg.wavelet, 0.5 * cfg.wavelet]).astype(np.float32)
    G = inputs.random_field(plan.data_shape(), 9)
    gsrc = torch.zeros((2, cfg.nt), dtype=torch.float32, device=DEV)
    gm = plan.gradient(esi.GRAD_SEED, torch.from_numpy(w).to(DEV), torch.from_numpy(G).to(DEV),
                       kind=esi.SRC_POINT, grad_src=gsrc, ckpt_every=11).cpu().numpy()
    g, m = _oracle_model(cfg)
    ref_m = np.zeros(g.phys_shape)
    for s, Gs in enumerate(_split(cfg, G)):
        rm, rs = core.gradient_seed(m, w[s].astype(np.float64), cfg.shot_rec(s),
                                    Gs.astype(np.float64), src_pos=cfg.src[s])
        ref_m += rm
        assert _rel(gsrc.cpu().numpy()[s], rs) < 1e-5, s
    assert _rel(gm, ref_m) < 1e-4


def test_batched_equals_per_shot(esi):
    """Several shots in one launch give bit-identical results to one shot per call."""
    cfg = _ragged_cfg()
    plan = _plan(esi, cfg)
    q = torch.from_numpy(inputs.random_field((cfg.nshots, cfg.nt, cfg.nz, cfg.nx), 10)).to(DEV)
    all_d = plan.forward(q, esi.SRC_DENSE).cpu().numpy()
    one = np.concatenate([plan.forward(q[s:s + 1].contiguous(), esi.SRC_DENSE, shot0=s, nshots=1)
                          .cpu().numpy() for s in range(cfg.nshots)])
    assert np.array_equal(all_d, one)
    Np_all, _ = plan.normal_apply(q)
    for s in range(cfg.nshots):
        Np_s, _ = plan.normal_apply(q[s:s + 1].contiguous(), shot0=s, nshots=1)
        assert torch.equal(Np_s[0], Np_all[s])


def test_single_step_and_errors(esi):
    cfg = _ragged_cfg(nshots=1, nt=1)
    cfg.src = np.array([[30, 2]], dtype=np.int32)      # a receiver sits on the source
    plan = _plan(esi, cfg)
    d = plan.forward(torch.from_numpy(cfg.wavelet[None, :1].copy()).to(DEV), esi.SRC_POINT)
    g, m = _oracle_model(cfg)
    ref = core.forward(m, cfg.wavelet[:1].astype(np.float64), cfg.shot_rec(0), src_pos=cfg.src[0])
    assert _rel(d.cpu().numpy().reshape(1, -1), ref) < 1e-6
    buf = torch.zeros(4, device=DEV)
    import ctypes
    rc = plan._lib.esi_forward(plan._h, 1, 1, esi.SRC_POINT, ctypes.c_void_p(buf.data_ptr()),
                               ctypes.c_void_p(buf.data_ptr()))
    assert rc == 1 and b"shot range" in plan._lib.esi_last_error()
    fast = np.full((cfg.nz, cfg.nx), 9000.0, dtype=np.float32)
    with pytest.raises(esi.EsiError) as e:
        _plan(esi, cfg, v=fast)
    assert e.value.code == 3


def test_time_block_bitwise(esi):
    """Every launch shape (one step per launch; two steps per launch on tiles
    of 32, 24 and 40 rows) gives the same bits for modelling, adjoint
    modelling, N p and the gradients (odd nt: the last step of each pass runs
    alone)."""
    cfg = _ragged_cfg(nt=41)
    q = torch.from_numpy(inputs.random_field((cfg.nshots, cfg.nt, cfg.nz, cfg.nx), 11)).to(DEV)
    w = torch.from_numpy(np.stack([cfg.wavelet] * cfg.nshots).astype(np.float32)).to(DEV)
    outs = []
    for shape in (1, 2, 3, 4):
        plan = _plan(esi, cfg)
        plan.set_launch_shape(shape, shape)
        dd = torch.from_numpy(inputs.random_field(plan.data_shape(), 12)).to(DEV)
        r = [plan.forward(w, esi.SRC_POINT), plan.forward(q, esi.SRC_DENSE), plan.adjoint(dd),
             plan.normal_apply(q)[0], plan.gradient(esi.GRAD_PENALTY, q),
             plan.gradient(esi.GRAD_ADJOINT, q, dd), plan.gradient(esi.GRAD_ADJOINT, q, dd, ckpt_every=5)]
        r.append(plan.forward_ckpt(w, 7))
        r.append(plan.gradient(esi.GRAD_SEED_REUSE, w, dd, kind=esi.SRC_POINT, ckpt_every=7))
        outs.append([t.cpu().numpy() for t in r])
        plan.close()
    for other in outs[1:]:
        for i, (a, b) in enumerate(zip(outs[0], other)):
            assert np.array_equal(a, b), i


def test_time_block_cg(esi):
    """CG with two-step launches matches one-step launches (p.Np partials are
    summed in another order, so the match is to rounding, not bitwise)."""
    cfg = _ragged_cfg(nt=40)
    xs = []
    for tb in (1, 2):
        plan = _plan(esi, cfg)
        plan.set_time_block(tb)
        g, m = _oracle_model(cfg)
        d_obs = [core.forward(m, cfg.wavelet.astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
                 .astype(np.float32) for s in range(cfg.nshots)]
        flat = torch.from_numpy(np.concatenate([d.ravel() for d in d_obs])).to(DEV)
        xs.append(plan.cg_solve(flat, max_iter=5)[0].cpu().numpy())
        plan.close()
    for s in range(2):
        assert _rel(xs[1][s], xs[0][s]) < 1e-6


@pytest.mark.parametrize("tb", [1, 2])
def test_cg_fused_residual(esi, tb):
    """The residual update fused into the adjoint pass (p.Np taken as
    ||S p||^2 + beta ||B p||^2 from the forward pass, r updated in place) and
    the separate pass: both within 1e-4 of the oracle's iterate and history, and
    within float32 rounding of each other, on ragged shots with one shot that
    has no receivers."""
    cfg = _ragged_cfg(nt=50)
    cfg.v_start = (cfg.v_true * 1.03).astype(np.float32)
    g, m_true = _oracle_model(cfg)
    _, m0 = _oracle_model(cfg, cfg.v_start)
    d_obs = [core.forward(m_true, cfg.wavelet.astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
             .astype(np.float32) for s in range(cfg.nshots)]
    flat = torch.from_numpy(np.concatenate([d.ravel() for d in d_obs])).to(DEV)
    res = {}
    for fuse in (True, False):
        plan = _plan(esi, cfg, v=cfg.v_start)
        plan.set_time_block(tb)
        plan.set_cg_rfuse(fuse)
        x, rep = plan.cg_solve(flat, max_iter=6)
        res[fuse] = (x.cpu().numpy(), rep)
        plan.close()
    for s in range(cfg.nshots):
        if d_obs[s].size == 0:
            assert np.all(res[True][0][s] == 0.0) and res[True][1]["shot_iters"][s] == 0
            continue
        ref = core.esi_cg(m0, cfg.src[s], cfg.shot_rec(s), d_obs[s].astype(np.float64), cfg.beta, 6)
        for fuse in (True, False):
            x, rep = res[fuse]
            assert _rel(x[s], ref.x) < 1e-4, (s, fuse)
            np.testing.assert_allclose(rep["res_hist"][s], ref.res_hist, rtol=1e-4)
        assert _rel(res[True][0][s], res[False][0][s]) < 1e-5, s
