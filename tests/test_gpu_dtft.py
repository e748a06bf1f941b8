"""The DTFT variant on the GPU (Sec. 5.2) against the FP64 oracle: the
frequency-domain normal operator (inverse DTFT fused into the forward pass,
DTFT accumulated in the adjoint pass), the right-hand side, CG on the
frequency vectors, the time-domain source and the PENALTY gradient; one- and
two-step launches give the same bits.

Tolerances: operators 1e-5, CG 1e-4, gradient 1e-4 (as for the time domain).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core, dtft
from paper_2211_06300_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
FREQS = np.array([1.0 / 0.06, 25.0, 40.0])      # the first on the DFT grid of nt dt = 0.06 s


def _rel(a, b):
    """Relative L2 difference; complex arrays keep both parts."""
    a = np.asarray(a).astype(np.complex128).ravel()
    b = np.asarray(b).astype(np.complex128).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def esi():
    from paper_2211_06300_amd import esi as _esi
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    _esi.load_library()
    return _esi


def _cfg(nt=60, seed=29):
    """37 x 70 grid, nb 8 (ragged tiles), two shots with uneven receivers."""
    rng = np.random.default_rng(seed)
    nz, nx = 37, 70
    cfg = inputs.cfg_tiny(nz=nz, nx=nx, nt=nt, nb=8, nrec=5, seed=seed)
    cfg.src = np.array([[5, 2], [50, 20]], dtype=np.int32)
    recs = [np.array([[0, 0], [69, 36], [30, 2], [30, 2], [31, 2]]),
            np.stack([rng.integers(0, nx, 30), rng.integers(0, nz, 30)], axis=1)]
    cfg.rec_ptr = np.concatenate([[0], np.cumsum([len(r) for r in recs])]).astype(np.int64)
    cfg.rec = np.concatenate(recs).astype(np.int32)
    cfg.v_true = (1800.0 + 900.0 * rng.random((nz, nx))).astype(np.float32)
    cfg.v_start = (cfg.v_true * 1.03).astype(np.float32)
    cfg.beta = 0.05
    return cfg


def _model(cfg, v):
    g = core.Grid(2, cfg.nz, cfg.nx, nb=cfg.nb, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt)
    return g, core.make_model(g, v)


def _plan(esi, cfg, v):
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(np.ascontiguousarray(v)).to(DEV))
    plan.dtft_set_freqs(FREQS)
    return plan


def _cplx(a):
    return a[..., 0].astype(np.float64) + 1j * a[..., 1].astype(np.float64)


def _split(cfg, flat):
    out, off = [], 0
    for s in range(cfg.nshots):
        n = int(cfg.rec_ptr[s + 1] - cfg.rec_ptr[s])
        out.append(flat[off:off + cfg.nt * n].reshape(cfg.nt, n))
        off += cfg.nt * n
    return out


@pytest.mark.parametrize("tb", [1, 2])
def test_dtft_normal_apply(esi, tb):
    cfg = _cfg()
    plan = _plan(esi, cfg, cfg.v_true)
    plan.set_time_block(tb)
    g, m = _model(cfg, cfg.v_true)
    p = inputs.random_field(plan.dtft_shape(cfg.nshots), 81)
    Mp, pMp = plan.dtft_normal_apply(torch.from_numpy(p).to(DEV))
    Mp, pMp = Mp.cpu().numpy(), pMp.cpu().numpy()
    for s in range(cfg.nshots):
        ref = dtft.normal_apply(m, cfg.shot_rec(s), core.annihilator_sq(g, tuple(cfg.src[s])), cfg.beta,
                                _cplx(p[s]), FREQS)
        assert _rel(_cplx(Mp[s]), ref) < 1e-5, s
        assert abs(pMp[s] - dtft.rdot(_cplx(p[s]), ref)) < 1e-5 * abs(pMp[s])
    plan.close()


def test_dtft_two_step_bitwise(esi):
    cfg = _cfg()
    p = torch.from_numpy(inputs.random_field((cfg.nshots, len(FREQS), cfg.nz, cfg.nx, 2), 82)).to(DEV)
    outs = []
    for tb in (1, 2):
        plan = _plan(esi, cfg, cfg.v_true)
        plan.set_time_block(tb)
        outs.append(plan.dtft_normal_apply(p)[0])
        plan.close()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("nf", [3, 12, 20])
def test_dtft_block_bitwise(esi, nf):
    """Blocks of K steps (sources formed per block, adjoint fields folded into
    the slices per block) give the same bits as the per-step kernels, for K
    dividing nt or not, K above nt, and nt odd (the last launch of a pass runs
    one step): normal operator, right-hand side, gradient and 3 CG iterations."""
    cfg = _cfg(nt=61)
    freqs = np.linspace(10.0, 70.0, nf)
    p = torch.from_numpy(inputs.random_field((cfg.nshots, nf, cfg.nz, cfg.nx, 2), 86)).to(DEV)
    outs = []
    for block in (0, 7, 32, 100):
        plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(DEV))
        plan.dtft_set_freqs(freqs)
        plan.set_dtft_block(block)
        dd = torch.from_numpy(inputs.random_field(plan.data_shape(), 87)).to(DEV)
        Mp, pMp = plan.dtft_normal_apply(p)
        x, rep = plan.dtft_cg_solve(dd, 3)
        # a loose tolerance: shots leave at different iterations, and the
        # passes skip the ones that left
        x2, rep2 = plan.dtft_cg_solve(dd, 8, rtol=0.6)
        outs.append([Mp, pMp, plan.dtft_rhs(dd), plan.dtft_gradient(p), x,
                     torch.from_numpy(np.asarray(rep["res_hist"])), x2,
                     torch.from_numpy(np.asarray(rep2["res_hist"])),
                     torch.from_numpy(np.asarray(rep2["shot_iters"]))])
        plan.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)


def test_dtft_rhs_and_to_time(esi):
    cfg = _cfg()
    plan = _plan(esi, cfg, cfg.v_start)
    g, m = _model(cfg, cfg.v_start)
    dd = inputs.random_field(plan.data_shape(), 83)
    b = plan.dtft_rhs(torch.from_numpy(dd).to(DEV)).cpu().numpy()
    for s, ds in enumerate(_split(cfg, dd)):
        ref = dtft.rhs(m, cfg.shot_rec(s), ds.astype(np.float64), FREQS)
        assert _rel(_cplx(b[s]), ref) < 1e-5, s
    x = inputs.random_field(plan.dtft_shape(cfg.nshots), 84)
    q = plan.dtft_to_time(torch.from_numpy(x).to(DEV)).cpu().numpy()
    for s in range(cfg.nshots):
        assert _rel(q[s], dtft.idtft(_cplx(x[s]), FREQS, cfg.dt, cfg.nt)) < 1e-6
    plan.close()


def test_dtft_cg(esi):
    """Algorithm 1 on the frequency vectors, 6 iterations, against the oracle."""
    cfg = _cfg(nt=50)
    g, mt = _model(cfg, cfg.v_true)
    d_obs = [core.forward(mt, cfg.wavelet.astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
             .astype(np.float32) for s in range(cfg.nshots)]
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(DEV))
    freqs = np.array([20.0, 40.0, 60.0])
    plan.dtft_set_freqs(freqs)
    flat = torch.from_numpy(np.concatenate([d.ravel() for d in d_obs])).to(DEV)
    x, rep = plan.dtft_cg_solve(flat, 6)
    x = x.cpu().numpy()
    _, m0 = _model(cfg, cfg.v_start)
    for s in range(cfg.nshots):
        ref = dtft.cg(m0, tuple(cfg.src[s]), cfg.shot_rec(s), d_obs[s].astype(np.float64), cfg.beta, freqs, 6)
        assert _rel(_cplx(x[s]), ref.x) < 1e-4, s
        np.testing.assert_allclose(rep["res_hist"][s], ref.res_hist, rtol=1e-4)
    plan.close()


def test_dtft_gradient(esi):
    cfg = _cfg()
    plan = _plan(esi, cfg, cfg.v_true)
    g, m = _model(cfg, cfg.v_true)
    x = inputs.random_field(plan.dtft_shape(cfg.nshots), 85)
    gm = plan.dtft_gradient(torch.from_numpy(x).to(DEV)).cpu().numpy()
    ref = sum(dtft.gradient_penalty(m, _cplx(x[s]), core.annihilator_sq(g, tuple(cfg.src[s])), cfg.beta, FREQS)
              for s in range(cfg.nshots))
    assert _rel(gm, ref) < 1e-4
    plan.close()


def test_dtft_argument_errors(esi):
    cfg = _cfg(nt=20)
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(DEV))
    p = torch.zeros((cfg.nshots, 2, cfg.nz, cfg.nx, 2), dtype=torch.float32, device=DEV)
    plan.dtft_freqs = np.zeros(2)
    with pytest.raises(esi.EsiError):                     # no frequencies set on the plan
        plan.dtft_normal_apply(p)
    with pytest.raises(esi.EsiError):
        plan.dtft_set_freqs(np.arange(40.0))
    with pytest.raises(esi.EsiError):
        plan.dtft_set_freqs([10.0, -1.0])
    with pytest.raises(esi.EsiError):
        plan.set_dtft_block(-1)
    with pytest.raises(esi.EsiError):
        plan.set_dtft_block(1025)
    plan.close()
