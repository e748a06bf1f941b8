"""3D kernels and differentiation on the GPU against the FP64 oracle.

Sizes: 20 x 27 x 70 physical cells with an 6-cell absorbing layer, i.e. a
32 x 39 x 82 padded grid: two 64-wide column blocks (one ragged), five 8-deep
blocks (one ragged) and a single 32-plane chunk.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core
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


def _cfg3(nt=40, seed=31, nshots=2):
    rng = np.random.default_rng(seed)
    nz, ny, nx = 20, 27, 70
    v = (1900.0 + 800.0 * rng.random((nz, ny, nx))).astype(np.float32)
    src = np.array([[5, 3, 4], [60, 10, 20]][:nshots], dtype=np.int32)     # (ix, iz, iy)
    recs = [np.array([[0, 0, 0], [69, 19, 26], [30, 2, 13], [30, 2, 13], [31, 2, 13],
                      [10, 2, 25], [65, 5, 1]]),
            np.stack([rng.integers(0, nx, 30), rng.integers(0, nz, 30), rng.integers(0, ny, 30)],
                     axis=1)][:nshots]
    ptr = np.zeros(nshots + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in recs])
    w = inputs.ricker_samples(nt, 1e-3, 25.0)
    return inputs.Config("test3d", 3, nz, nx, ny, 10.0, 1e-3, nt, 6, 25.0, 0.05, 0, v, v, src,
                         ptr, np.concatenate(recs).astype(np.int32), w)


def _model(cfg, v=None):
    g = core.Grid(3, cfg.nz, cfg.nx, ny=cfg.ny, nb=cfg.nb, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt)
    return g, core.make_model(g, cfg.v_true if v is None else v)


def _plan(esi, cfg):
    return esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(DEV))


def _split(cfg, flat):
    out, off = [], 0
    for s in range(cfg.nshots):
        n = int(cfg.rec_ptr[s + 1] - cfg.rec_ptr[s])
        out.append(flat[off:off + cfg.nt * n].reshape(cfg.nt, n))
        off += cfg.nt * n
    return out


def test_3d_forward_point_and_dense(esi):
    cfg = _cfg3()
    plan = _plan(esi, cfg)
    g, m = _model(cfg)
    w = np.stack([cfg.wavelet, -0.5 * cfg.wavelet]).astype(np.float32)
    d = plan.forward(torch.from_numpy(w).to(DEV), esi.SRC_POINT).cpu().numpy()
    for s, ds in enumerate(_split(cfg, d)):
        ref = core.forward(m, w[s].astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
        assert _rel(ds, ref) < 1e-5, s
    q = inputs.random_field((cfg.nshots, cfg.nt, *cfg.phys_shape), 41)
    d = plan.forward(torch.from_numpy(q).to(DEV), esi.SRC_DENSE).cpu().numpy()
    for s, ds in enumerate(_split(cfg, d)):
        ref = core.forward(m, q[s].astype(np.float64), cfg.shot_rec(s))
        assert _rel(ds, ref) < 1e-5, s


def test_3d_adjoint_normal_dot(esi):
    cfg = _cfg3()
    plan = _plan(esi, cfg)
    g, m = _model(cfg)
    dd = inputs.random_field(plan.data_shape(), 42)
    out = plan.adjoint(torch.from_numpy(dd).to(DEV)).cpu().numpy()
    for s, ds in enumerate(_split(cfg, dd)):
        assert _rel(out[s], core.adjoint(m, cfg.shot_rec(s), ds.astype(np.float64))) < 1e-5, s
    p = inputs.random_field((cfg.nshots, cfg.nt, *cfg.phys_shape), 43)
    Np, pAp = plan.normal_apply(torch.from_numpy(p).to(DEV))
    for s in range(cfg.nshots):
        w2 = core.annihilator_sq(g, cfg.src[s])
        ref = core.normal_apply(m, cfg.shot_rec(s), w2, cfg.beta, p[s].astype(np.float64))
        assert _rel(Np.cpu().numpy()[s], ref) < 1e-5, s
    # GPU dot test
    q = torch.from_numpy(p).to(DEV)
    dt_ = torch.from_numpy(dd).to(DEV)
    lhs = torch.dot(plan.forward(q, esi.SRC_DENSE).double(), dt_.double()).item()
    rhs = torch.dot(q.double().ravel(), plan.adjoint(dt_).double().ravel()).item()
    assert abs(lhs - rhs) / max(abs(lhs), abs(rhs)) < 1e-6


def test_3d_cg_fused_residual(esi):
    """CG (Algorithm 1) in 3D, 4 iterations from a model 3% off: the residual
    update fused into the adjoint pass and as a separate pass, both within 1e-4
    of the oracle's iterate and history."""
    cfg = _cfg3(nt=40)
    g, m = _model(cfg)
    v0 = (cfg.v_true * 1.03).astype(np.float32)
    _, m0 = _model(cfg, v0)
    d_obs = [core.forward(m, cfg.wavelet.astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
             .astype(np.float32) for s in range(cfg.nshots)]
    flat = torch.from_numpy(np.concatenate([d.ravel() for d in d_obs])).to(DEV)
    refs = [core.esi_cg(m0, cfg.src[s], cfg.shot_rec(s), d_obs[s].astype(np.float64), cfg.beta, 4)
            for s in range(cfg.nshots)]
    for fuse in (True, False):
        plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(v0).to(DEV))
        plan.set_cg_rfuse(fuse)
        x, rep = plan.cg_solve(flat, max_iter=4)
        x = x.cpu().numpy()
        for s in range(cfg.nshots):
            assert _rel(x[s], refs[s].x) < 1e-4, (s, fuse)
            np.testing.assert_allclose(rep["res_hist"][s], refs[s].res_hist, rtol=1e-4)
        plan.close()


def _cplx(a):
    return a[..., 0].astype(np.float64) + 1j * a[..., 1].astype(np.float64)


def _rel_c(a, b):
    a = np.asarray(a).astype(np.complex128).ravel()
    b = np.asarray(b).astype(np.complex128).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_3d_dtft(esi):
    """The DTFT variant on a 3D plan, slices met per block of steps (the
    per-step path is 2D only and refused here): M p within 1e-5 and 3 CG
    iterations within 1e-4 of the oracle."""
    from oracle import dtft
    cfg = _cfg3(nt=40)
    g, m = _model(cfg)
    freqs = np.array([20.0, 45.0, 70.0])
    plan = _plan(esi, cfg)
    plan.dtft_set_freqs(freqs)
    plan.set_dtft_block(16)
    p = inputs.random_field(plan.dtft_shape(cfg.nshots), 46)
    Mp, pMp = plan.dtft_normal_apply(torch.from_numpy(p).to(DEV))
    Mp = Mp.cpu().numpy()
    for s in range(cfg.nshots):
        ref = dtft.normal_apply(m, cfg.shot_rec(s), core.annihilator_sq(g, tuple(cfg.src[s])), cfg.beta,
                                _cplx(p[s]), freqs)
        assert _rel_c(_cplx(Mp[s]), ref) < 1e-5, s
    d_obs = [core.forward(m, cfg.wavelet.astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
             .astype(np.float32) for s in range(cfg.nshots)]
    flat = torch.from_numpy(np.concatenate([d.ravel() for d in d_obs])).to(DEV)
    x, rep = plan.dtft_cg_solve(flat, 3)
    x = x.cpu().numpy()
    for s in range(cfg.nshots):
        ref = dtft.cg(m, tuple(cfg.src[s]), cfg.shot_rec(s), d_obs[s].astype(np.float64), cfg.beta, freqs, 3)
        assert _rel_c(_cplx(x[s]), ref.x) < 1e-4, s
    plan.set_dtft_block(0)
    with pytest.raises(esi.EsiError):
        plan.dtft_normal_apply(torch.from_numpy(p).to(DEV))
    plan.close()


def test_3d_dataspace(esi):
    """The data-space solver on a 3D plan: w within 1e-4 of the oracle after 4
    iterations, q from the GPU's own w within 1e-5, and the checkpointed
    adjoint field bit for bit equal to the resident one."""
    from oracle import dataspace
    cfg = _cfg3(nt=30)
    g, m = _model(cfg)
    v0 = (cfg.v_true * 1.03).astype(np.float32)
    _, m0 = _model(cfg, v0)
    d_obs = [core.forward(m, cfg.wavelet.astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
             .astype(np.float32) for s in range(cfg.nshots)]
    flat = torch.from_numpy(np.concatenate([d.ravel() for d in d_obs])).to(DEV)
    outs = []
    for every in (0, 7):
        plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(v0).to(DEV))
        plan.set_ds_ckpt(every)
        outs.append(plan.ds_cg_solve(flat, 4))
        plan.close()
    w, q, rep = outs[0]
    assert torch.equal(w, outs[1][0]) and torch.equal(q, outs[1][1])
    w, q = w.cpu().numpy(), q.cpu().numpy()
    for s, ws in enumerate(_split(cfg, w)):
        d64 = d_obs[s].astype(np.float64)
        rw, rq, res = dataspace.cg(m0, tuple(cfg.src[s]), cfg.shot_rec(s), d64, cfg.beta, 4)
        assert _rel(ws, rw) < 1e-4, s
        w2 = core.annihilator_sq(g, tuple(cfg.src[s]))
        q_of_w = core.adjoint(m0, cfg.shot_rec(s), d64 - ws.astype(np.float64)) / (cfg.beta * w2[None])
        assert _rel(q[s], q_of_w) < 1e-5, s


def test_3d_gradient_seed_ckpt(esi):
    cfg = _cfg3(nt=60)
    plan = _plan(esi, cfg)
    g, m = _model(cfg)
    w = np.stack([cfg.wavelet, 0.7 * cfg.wavelet]).astype(np.float32)
    G = inputs.random_field(plan.data_shape(), 44)
    gsrc = torch.zeros((2, cfg.nt), device=DEV)
    gm = plan.gradient(esi.GRAD_SEED, torch.from_numpy(w).to(DEV), torch.from_numpy(G).to(DEV),
                       kind=esi.SRC_POINT, grad_src=gsrc, ckpt_every=13).cpu().numpy()
    ref = np.zeros(cfg.phys_shape)
    for s, Gs in enumerate(_split(cfg, G)):
        rm, rs = core.gradient_seed(m, w[s].astype(np.float64), cfg.shot_rec(s),
                                    Gs.astype(np.float64), src_pos=cfg.src[s])
        ref += rm
        assert _rel(gsrc.cpu().numpy()[s], rs) < 1e-5
    assert _rel(gm, ref) < 1e-4


def test_autograd_matches_seed_and_reuses_checkpoints(esi):
    """Propagate.backward (checkpoints kept by the forward pass) equals the SEED
    gradient computed from scratch, bit for bit, in 2D and 3D."""
    from paper_2211_06300_amd.autograd import propagate
    for cfg in (_cfg3(nt=50), inputs.cfg_tiny(nz=30, nx=70, nt=90, nb=8, nrec=12)):
        plan = _plan(esi, cfg)
        vel = torch.from_numpy(cfg.v_true).to(DEV).requires_grad_(True)
        w = torch.from_numpy(np.stack([cfg.wavelet] * cfg.nshots)).to(DEV).requires_grad_(True)
        d = propagate(vel, w, plan, ckpt_every=7)
        G = torch.from_numpy(inputs.random_field(tuple(d.shape), 45)).to(DEV)
        (d * G).sum().backward()
        gm = plan.gradient(esi.GRAD_SEED, w.detach(), G, kind=esi.SRC_POINT, ckpt_every=0)
        gv = plan.grad_velocity(vel.detach(), gm)
        assert torch.equal(vel.grad, gv)
        gsrc = torch.zeros_like(w)
        plan.gradient(esi.GRAD_SEED, w.detach(), G, kind=esi.SRC_POINT, grad_src=gsrc)
        assert torch.equal(w.grad, gsrc)
        plan.close()


def _bump(cfg, centre, amp=20.0):
    """Gaussian velocity bump (sigma^2 = 15 cells^2), zero within 4 cells of
    the edges so the padded extension of the model is untouched."""
    zz, yy, xx = np.meshgrid(*[np.arange(n) for n in cfg.phys_shape], indexing="ij")
    c = centre
    bump = np.exp(-((zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2) / 30.0)
    inner = ((zz >= 4) & (zz < cfg.nz - 4) & (yy >= 4) & (yy < cfg.ny - 4)
             & (xx >= 4) & (xx < cfg.nx - 4))
    return (amp * bump * inner).astype(np.float32)


def test_autograd_fd_3d(esi):
    """<grad_v, dv> from Propagate.backward against central differences of
    L(v) = 1/2 ||S(v) w - d_obs||^2.

    The differences are taken with the FP64 oracle (float32 losses cannot
    resolve directional derivatives far below 1e-6 L); the bound is
    1e-3 |fd| + 1e-4 ||grad|| ||dv|| (the gradient's parity tolerance through
    Cauchy-Schwarz).  A bump on the source-receiver path, where the change is
    about 1 % of L, is also differenced on the GPU itself (bound 1e-2).
    """
    from paper_2211_06300_amd.autograd import propagate
    cfg = _cfg3(nt=120, nshots=1)
    plan = _plan(esi, cfg)
    v0 = torch.from_numpy(cfg.v_true).to(DEV)
    w = torch.from_numpy(cfg.wavelet[None].copy()).to(DEV)
    d_obs = plan.forward(w, esi.SRC_POINT) * 0.9
    vel = v0.clone().requires_grad_(True)
    d = propagate(vel, w, plan, ckpt_every=10)
    loss = 0.5 * ((d - d_obs) ** 2).sum()
    loss.backward()
    gv = vel.grad.double().cpu().numpy()

    g, m = _model(cfg)
    eta = m.eta_max
    rec, src = cfg.shot_rec(0), cfg.src[0]
    wd = cfg.wavelet.astype(np.float64)
    dobs_ref = d_obs.cpu().numpy().astype(np.float64).reshape(cfg.nt, -1)

    def L_ref(vv):
        dd = core.forward(core.make_model(g, vv, eta), wd, rec, src_pos=src)
        return 0.5 * float(np.sum((dd - dobs_ref) ** 2))

    rng = np.random.default_rng(46)
    centres = [[rng.uniform(5, n - 5) for n in cfg.phys_shape] for _ in range(3)] + [(8, 6, 8)]
    v64 = cfg.v_true.astype(np.float64)
    for k, c in enumerate(centres):
        dv = _bump(cfg, c).astype(np.float64)
        fd = (L_ref(v64 + dv) - L_ref(v64 - dv)) / 2.0
        an = float(np.sum(gv * dv))
        bound = 1e-3 * abs(fd) + 1e-4 * np.linalg.norm(gv) * np.linalg.norm(dv)
        assert abs(fd - an) <= bound, (k, fd, an, bound)

    dv = torch.from_numpy(_bump(cfg, (8, 6, 8))).to(DEV)

    def L_gpu(vv):
        plan.set_model(vv)
        r = plan.forward(w, esi.SRC_POINT) - d_obs
        return 0.5 * float((r.double() ** 2).sum())
    fd = (L_gpu(v0 + dv) - L_gpu(v0 - dv)) / 2.0
    an = float((vel.grad.double() * dv.double()).sum())
    assert abs(fd - an) / abs(fd) < 1e-2, (fd, an)


def _cfg3_deep(nt=33, seed=37):
    """70 x 27 in x and y, 75 planes deep with a 6-cell layer: 87 padded planes,
    two z chunks of the two-step kernel (64 + 23 planes) and ragged 56 x 24
    column blocks; receivers on several planes, one on the chunk boundary
    (physical plane 58 = padded 64), shared cells and grid corners."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = 75, 27, 70
    v = (1900.0 + 800.0 * rng.random((nz, ny, nx))).astype(np.float32)
    src = np.array([[5, 3, 4], [60, 57, 20]], dtype=np.int32)             # (ix, iz, iy)
    recs = [np.array([[0, 0, 0], [69, 74, 26], [30, 2, 13], [30, 2, 13], [31, 58, 13],
                      [10, 58, 25], [65, 63, 1], [40, 57, 12]]),
            np.stack([rng.integers(0, nx, 40), rng.integers(0, nz, 40), rng.integers(0, ny, 40)], axis=1)]
    ptr = np.zeros(3, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in recs])
    w = inputs.ricker_samples(nt, 1e-3, 25.0)
    return inputs.Config("test3d-deep", 3, nz, nx, ny, 10.0, 1e-3, nt, 6, 25.0, 0.05, 0, v, v, src,
                         ptr, np.concatenate(recs).astype(np.int32), w)


def test_3d_two_step_bitwise(esi):
    """Two time steps per launch (56 x 24 column blocks, 64-plane chunks, the
    first step on the block grown by one stencil radius) give the same bits as
    one step per launch for modelling, adjoint modelling, N p, the source
    gradient records and the checkpointed gradients (odd nt: the last step of
    each pass runs alone); CG agrees to rounding (p.Np partials are summed over
    another tiling)."""
    for cfg in (_cfg3_deep(), _cfg3(nt=41)):
        q = torch.from_numpy(inputs.random_field((cfg.nshots, cfg.nt, *cfg.phys_shape), 51)).to(DEV)
        w = torch.from_numpy(np.stack([cfg.wavelet, -0.6 * cfg.wavelet]).astype(np.float32)).to(DEV)
        outs, xs = [], []
        for shape in (1, 2):
            plan = _plan(esi, cfg)
            plan.set_launch_shape(shape, shape)
            dd = torch.from_numpy(inputs.random_field(plan.data_shape(), 52)).to(DEV)
            gsrc = torch.zeros((cfg.nshots, cfg.nt), device=DEV)
            gq = torch.zeros_like(q)
            r = [plan.forward(w, esi.SRC_POINT), plan.forward(q, esi.SRC_DENSE), plan.adjoint(dd),
                 *plan.normal_apply(q),
                 plan.gradient(esi.GRAD_ADJOINT, q, dd, ckpt_every=5),
                 plan.gradient(esi.GRAD_ADJOINT, q, dd, ckpt_every=0),
                 plan.gradient(esi.GRAD_SEED, w, dd, kind=esi.SRC_POINT, grad_src=gsrc, ckpt_every=6), gsrc,
                 plan.gradient(esi.GRAD_SEED, q, dd, kind=esi.SRC_DENSE, grad_src=gq, ckpt_every=7), gq,
                 plan.forward_ckpt(w, 8),
                 plan.gradient(esi.GRAD_SEED_REUSE, w, dd, kind=esi.SRC_POINT, ckpt_every=8)]
            outs.append([t.cpu().numpy() for t in r])
            xs.append(plan.cg_solve(dd, max_iter=3)[0].cpu().numpy())
            plan.close()
        for i, (a, b) in enumerate(zip(*outs)):
            if i == 4:   # p.Np (float64 partials over another tiling)
                np.testing.assert_allclose(a, b, rtol=1e-12)
            else:
                assert np.array_equal(a, b), (cfg.name, i)
        for s in range(cfg.nshots):
            assert _rel(xs[1][s], xs[0][s]) < 1e-6


def test_3d_deep_forward_matches_oracle(esi):
    """The two-step 3D kernel across z chunks against the FP64 oracle."""
    cfg = _cfg3_deep(nt=30)
    plan = _plan(esi, cfg)
    g, m = _model(cfg)
    w = np.stack([cfg.wavelet, 0.8 * cfg.wavelet]).astype(np.float32)
    d = plan.forward(torch.from_numpy(w).to(DEV), esi.SRC_POINT).cpu().numpy()
    for s, ds in enumerate(_split(cfg, d)):
        ref = core.forward(m, w[s].astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
        assert _rel(ds, ref) < 1e-5, s
    dd = inputs.random_field(plan.data_shape(), 53)
    out = plan.adjoint(torch.from_numpy(dd).to(DEV)).cpu().numpy()
    for s, ds in enumerate(_split(cfg, dd)):
        assert _rel(out[s], core.adjoint(m, cfg.shot_rec(s), ds.astype(np.float64))) < 1e-5, s


def test_3d_autotune_probe(esi):
    """The autotuner on a 3D plan times one and two steps per launch on its
    propagation probe (a forward pass, and a gradient's adjoint pass with the
    correlation over a two-slot store, in paired one-step launches or two-step
    ones); whatever it picks, the checkpointed gradient keeps its bits."""
    cfg = _cfg3(nt=41)
    plan = _plan(esi, cfg)
    w = torch.from_numpy(np.stack([cfg.wavelet, -0.6 * cfg.wavelet]).astype(np.float32)).to(DEV)
    dd = torch.from_numpy(inputs.random_field(plan.data_shape(), 53)).to(DEV)
    g0 = plan.gradient(esi.GRAD_SEED, w, dd, kind=esi.SRC_POINT, ckpt_every=7).clone()
    ch = plan.autotune(probe=True)
    table = plan.tune_table()
    assert ch[0] in (1, 2) and ch[1] in (1, 2)
    assert [r[0] for r in table] == [1, 2] and all(r[1] > 0 and r[2] > 0 for r in table)
    assert ch == (min(table, key=lambda r: r[1])[0], min(table, key=lambda r: r[2])[0])
    plan.forward_ckpt(w, 7)
    g1 = plan.gradient(esi.GRAD_SEED_REUSE, w, dd, kind=esi.SRC_POINT, ckpt_every=7)
    assert torch.equal(g1, g0)
    plan.close()
