"""Pins of the outer-loop oracle (Algorithm 2, Sec. 2.4): the L-BFGS two-loop
recursion against the explicit BFGS inverse-Hessian update, convergence on a
convex quadratic, the Armijo condition along the accepted steps, the
monotonicity of the data misfit in beta behind the discrepancy rule, and a
small ESI inversion that moves the model towards the truth."""
import numpy as np
import pytest

from oracle import core, dense, outer
from paper_2211_06300_amd import inputs


def test_two_loop_equals_bfgs_matrix():
    """Nocedal & Wright Sec. 7.2: the two-loop recursion computes H g for
    H_k = V^T H_{k-1} V + rho s s^T, V = I - rho y s^T, H_0 = (s'y / y'y) I of
    the newest pair."""
    rng = np.random.default_rng(3)
    n = 7
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    pairs = []
    for _ in range(4):
        s = rng.standard_normal(n)
        pairs.append((s, A @ s + 0.1 * rng.standard_normal(n)))
    assert all(s @ y > 0 for s, y in pairs)
    g = rng.standard_normal(n)
    s_new, y_new = pairs[-1]
    H = (s_new @ y_new) / (y_new @ y_new) * np.eye(n)
    for s, y in pairs:
        rho = 1.0 / (y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    d = outer.lbfgs_direction(g, pairs)
    assert np.linalg.norm(d + H @ g) < 1e-12 * np.linalg.norm(H @ g)
    assert np.array_equal(outer.lbfgs_direction(g, []), -g)


def _quadratic(n=20, seed=4):
    rng = np.random.default_rng(seed)
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(np.geomspace(1.0, 100.0, n)) @ Q.T * 1e14
    m_star = rng.uniform(2e-7, 5e-7, n)

    def evaluate(m, beta):
        e = m - m_star
        return 0.5 * e @ A @ e, A @ e, 0.1
    return evaluate, m_star


def test_minimize_quadratic():
    """On a convex quadratic (condition number 100) the loop reaches the minimiser
    and J never increases."""
    evaluate, m_star = _quadratic()
    m0 = np.full_like(m_star, 3.5e-7)
    opts = outer.OuterOptions(outer_iters=60, lbfgs_mem=10, first_step=0.05)
    res = outer.minimize(evaluate, m0, 1.0, opts)
    assert res.status == "ok"
    assert np.linalg.norm(res.m - m_star) < 1e-6 * np.linalg.norm(m_star)
    assert all(b <= a for a, b in zip(res.J, res.J[1:]))
    assert len(res.step) == 60 and res.evals == 1 + sum(res.trials)


def test_minimize_clips_to_bounds():
    """A minimiser outside the velocity bounds ends on the bound."""
    evaluate, m_star = _quadratic(n=5, seed=5)
    m_star[2] = 2e-6                              # v = 707 m/s, below v_min = 1000
    opts = outer.OuterOptions(outer_iters=40, lbfgs_mem=5, first_step=0.05)
    res = outer.minimize(evaluate, np.full(5, 3e-7), 1.0, opts)
    assert res.m[2] == pytest.approx(1e-6, rel=1e-12)
    assert all(b <= a for a, b in zip(res.J, res.J[1:]))


def _tiny_esi(nt=60, seed=9):
    cfg = inputs.cfg_tiny(nz=12, nx=14, nt=nt, nb=4, nrec=7, seed=seed)
    g = core.Grid(2, cfg.nz, cfg.nx, nb=cfg.nb, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt)
    eta = core.eta_max_default(3000.0, g.nb, g.dx)
    zz, xx = np.meshgrid(np.arange(cfg.nz), np.arange(cfg.nx), indexing="ij")
    v_bg = np.full((cfg.nz, cfg.nx), 2000.0)
    v_true = v_bg + 300.0 * np.exp(-((zz - 7) ** 2 + (xx - 7) ** 2) / 6.0)
    mt = core.make_model(g, v_true, eta_max=eta)
    srcs = [(3, 1), (10, 1)]
    rec = np.stack([np.arange(cfg.nx), np.full(cfg.nx, 1)], axis=1)
    w = cfg.wavelet.astype(np.float64)
    shots = [(s, rec, core.forward(mt, w, rec, src_pos=s)) for s in srcs]
    return g, eta, v_bg, v_true, shots, w


def test_data_misfit_grows_with_beta():
    """dJ^e/dbeta >= 0 (Sec. 2.4): with q solving the normal equation exactly,
    the data misfit is non-decreasing in beta, the property the discrepancy rule
    relies on."""
    g, eta, v_bg, v_true, shots, w = _tiny_esi(nt=30)
    m = core.make_model(g, v_bg, eta_max=eta)
    src, rec, d = shots[0]
    nin = g.nt * g.nz * g.nx
    S = dense.dense_matrix(lambda q: core.forward(m, q, rec), nin, (g.nt, g.nz, g.nx))
    W = np.tile(core.annihilator_sq(g, src).ravel(), g.nt)
    mis = []
    for beta in [1e-4, 1e-3, 1e-2, 1e-1, 1.0, 10.0]:
        q = dense.cholesky_solve(S.T @ S + beta * np.diag(W), S.T @ d.ravel())
        mis.append(np.linalg.norm(S @ q - d.ravel()))
    assert all(b >= a for a, b in zip(mis, mis[1:]))
    assert mis[-1] > 3 * mis[0]


def test_esi_inversion_moves_towards_truth():
    """Three outer iterations of the reduced ESI objective (20 CG iterations per
    solve) from the background model: J decreases and the model error shrinks."""
    g, eta, v_bg, v_true, shots, w = _tiny_esi()
    mask = np.ones(g.phys_shape)
    mask[:3] = 0.0                                # no update at the source/receiver rows
    ev = outer.esi_objective(g, shots, cg_iters=20, eta_max=eta, mask=mask)
    opts = outer.OuterOptions(outer_iters=3, first_step=0.03)
    m0 = 1.0 / v_bg ** 2
    res = outer.minimize(ev, m0, 0.05, opts)
    assert res.status == "ok"
    assert all(b < a for a, b in zip(res.J, res.J[1:]))
    mt = 1.0 / v_true ** 2
    assert np.linalg.norm(res.m - mt) < 0.9 * np.linalg.norm(m0 - mt)
    assert np.all(res.m[:3] == m0[:3])


def test_discrepancy_rule_moves_beta():
    """With a misfit band above the attainable misfit at the starting beta the
    rule raises beta (and clears the memory); with a band below it lowers beta."""
    g, eta, v_bg, v_true, shots, w = _tiny_esi(nt=40)
    ev = outer.esi_objective(g, shots, cg_iters=15, eta_max=eta)
    m0 = 1.0 / v_bg ** 2
    _, _, e0 = ev(m0.ravel(), 0.05)
    up = outer.minimize(ev, m0, 0.05, outer.OuterOptions(
        outer_iters=1, beta_rule="discrepancy", misfit_lo=2 * e0, misfit_hi=4 * e0, beta_tries=3))
    assert up.beta_iter[0] > 0.05
    down = outer.minimize(ev, m0, 0.05, outer.OuterOptions(
        outer_iters=1, beta_rule="discrepancy", misfit_lo=0.1 * e0, misfit_hi=0.5 * e0, beta_tries=3))
    assert down.beta_iter[0] < 0.05
    assert up.evals >= 3 and down.evals >= 3
