"""CG iterations replayed from captured HIP graphs against the same solve run
eagerly: identical bits in x, the residual history and the iteration counts,
on every replay, with eager work and synchronizations between replays."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core
from paper_2211_06300_amd import inputs
from tests.test_gpu_parity import _oracle_model, _plan, _ragged_cfg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def esi():
    from paper_2211_06300_amd import esi as _esi
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    _esi.load_library()
    return _esi


def _d_obs(cfg):
    g, m = _oracle_model(cfg)
    d = [core.forward(m, cfg.wavelet.astype(np.float64), cfg.shot_rec(s), src_pos=cfg.src[s])
         .astype(np.float32) for s in range(cfg.nshots)]
    return torch.from_numpy(np.concatenate([x.ravel() for x in d])).to(DEV)


@pytest.mark.parametrize("time_block", [1, 2])
def test_cg_graph_equals_eager(esi, time_block):
    cfg = _ragged_cfg(nt=50)
    cfg.v_start = (cfg.v_true * 1.03).astype(np.float32)
    d = _d_obs(cfg)
    plan = _plan(esi, cfg, v=cfg.v_start)
    plan.set_time_block(time_block)
    x0, rep0 = plan.cg_solve(d, max_iter=7, rtol=0.0)
    x0 = x0.clone()
    plan.set_cg_graph(True)
    x = plan.new_vec(cfg.nshots)
    work = torch.empty((3, *plan.vec_shape(cfg.nshots)), dtype=torch.float32, device=DEV)
    for rep_i in range(3):
        x.fill_(123.0)                                   # eager work between replays
        _, rep = plan.cg_solve(d, max_iter=7, rtol=0.0, x=x, work=work)
        torch.cuda.synchronize()
        assert torch.equal(x, x0), rep_i
        assert rep["iters"] == rep0["iters"]
        np.testing.assert_array_equal(rep["shot_iters"], rep0["shot_iters"])
        np.testing.assert_array_equal(rep["res_hist"], rep0["res_hist"])
        plan.normal_apply(work[1])                       # unrelated eager call in between
    plan.set_cg_graph(False)
    x2, _ = plan.cg_solve(d, max_iter=7, rtol=0.0)
    assert torch.equal(x2, x0)
    plan.close()


def test_cg_graph_early_exit(esi):
    """Shots retire on the device at different iterations; replays after every
    shot has left are no-ops."""
    cfg = _ragged_cfg(nshots=2, nt=40)
    d = _d_obs(cfg)
    plan = _plan(esi, cfg)
    x0, rep0 = plan.cg_solve(d, max_iter=30, rtol=0.2)
    x0 = x0.clone()
    plan.set_cg_graph(True)
    for _ in range(2):
        x, rep = plan.cg_solve(d, max_iter=30, rtol=0.2)
        assert torch.equal(x, x0)
        np.testing.assert_array_equal(rep["shot_iters"], rep0["shot_iters"])
        np.testing.assert_array_equal(rep["res_hist"], rep0["res_hist"])
    g, m = _oracle_model(cfg)
    for s in range(2):
        ref = core.esi_cg(m, cfg.src[s], cfg.shot_rec(s),
                          d.cpu().numpy()[int(cfg.nt * cfg.rec_ptr[s]):int(cfg.nt * cfg.rec_ptr[s + 1])]
                          .reshape(cfg.nt, -1).astype(np.float64), cfg.beta, 30, rtol=0.2)
        assert rep["shot_iters"][s] == ref.iters
    plan.close()


def test_cg_graph_small_config_timing(esi):
    """The small parity workload (201 x 201, 500 steps, 5 iterations), where
    launches are short: graph replay matches eager bit for bit; both timings
    are printed."""
    import time
    cfg = inputs.cfg_small()
    d = _d_obs(cfg)
    plan = _plan(esi, cfg)
    out = {}
    for mode in (False, True, True):
        plan.set_cg_graph(mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, rep = plan.cg_solve(d, max_iter=5)
        torch.cuda.synchronize()
        out.setdefault(mode, []).append((time.perf_counter() - t, x.clone()))
    print(f"eager {out[False][0][0] * 1e3:.1f} ms, graph first {out[True][0][0] * 1e3:.1f} ms "
          f"(captures), graph replay {out[True][1][0] * 1e3:.1f} ms")
    assert torch.equal(out[True][0][1], out[False][0][1])
    assert torch.equal(out[True][1][1], out[False][0][1])
    plan.close()


def test_autotune_choice_and_results(esi):
    """The autotuner times the four launch shapes for each direction on the
    plan's shapes, reports the table and caches the choice; CG results agree
    with the untuned ones to rounding (only the p.Np partials are summed over
    another tiling), and propagations are bitwise the same."""
    cfg = _ragged_cfg(nt=40)
    d = _d_obs(cfg)
    plan = _plan(esi, cfg)
    x0, _ = plan.cg_solve(d, max_iter=4)
    x0 = x0.clone()
    ch = plan.autotune()
    assert ch[0] in (1, 2, 3, 4) and ch[1] in (1, 2, 3, 4)
    table = plan.tune_table()
    assert [r[0] for r in table] == [1, 2, 3, 4] or [r[0] for r in table] == [1, 3, 2, 4]
    assert all(r[1] > 0 and r[2] > 0 for r in table)
    best_f = min(table, key=lambda r: r[1])[0]
    best_a = min(table, key=lambda r: r[2])[0]
    assert ch == (best_f, best_a)
    assert plan.autotune() == ch                     # cached
    assert plan.tune_table() == table
    # the propagation-only timing run (forward, and a gradient's adjoint): its own cache entry
    chp = plan.autotune(probe=True)
    assert chp[0] in (1, 2, 3, 4) and chp[1] in (1, 2, 3, 4) and len(plan.tune_table()) == 4
    plan.set_launch_shape(*ch)
    x1, _ = plan.cg_solve(d, max_iter=4)
    assert float(torch.linalg.norm(x1 - x0) / torch.linalg.norm(x0)) < 1e-6
    w = torch.from_numpy(np.tile(cfg.wavelet, (cfg.nshots, 1))).to(DEV)
    y0 = plan.forward(w, esi.SRC_POINT).clone()
    plan.set_time_block(1)
    assert torch.equal(plan.forward(w, esi.SRC_POINT), y0)
    # the probe's correlating adjoint pass uses gradient scratch only: the
    # checkpoints a forward pass keeps survive it
    G = torch.from_numpy(inputs.random_field(plan.data_shape(), 47)).to(DEV)
    plan.forward_ckpt(w, 6)
    plan.autotune(probe=True, force=True)
    g1 = plan.gradient(esi.GRAD_SEED_REUSE, w, G, kind=esi.SRC_POINT, ckpt_every=6).clone()
    g0 = plan.gradient(esi.GRAD_SEED, w, G, kind=esi.SRC_POINT, ckpt_every=6)
    assert torch.equal(g1, g0)
    plan.close()
