"""Pins of the oracle's WRI functions (Sec. 2.2: eq. (wridSf), eq. (normalwri),
eq. (wrieqfwi), Table (compare)) against dense matrices, direct solves, the
Sherman-Morrison-Woodbury route and finite differences."""
import numpy as np
import pytest

from oracle import core, dense
from paper_2211_06300_amd import inputs


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def test_point_source_is_dense_delta():
    """The wavelet injected at the source cell is the dense source that holds the
    wavelet in that cell and zero elsewhere (2D and 3D), so f + q is well defined."""
    cfg = inputs.cfg_tiny(nz=10, nx=12, nt=40)
    g = core.Grid(2, cfg.nz, cfg.nx, nb=cfg.nb, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt)
    m = core.make_model(g, cfg.v_true)
    rec = np.stack([np.arange(12), np.full(12, 7)], axis=1)
    w = cfg.wavelet.astype(np.float64)
    for src in [(5, 1), (0, 9), (11, 4)]:
        d_pt = core.forward(m, w, rec, src_pos=src)
        d_dn = core.forward(m, core.with_point_source(g, np.zeros((g.nt, *g.phys_shape)), w, src), rec)
        assert _rel(d_dn, d_pt) < 1e-14
    g3 = core.Grid(3, 6, 7, ny=5, nb=3, nt=20, dx=10.0, dt=1e-3)
    rng = np.random.default_rng(2)
    m3 = core.make_model(g3, 2000.0 + 300.0 * rng.random(g3.phys_shape))
    rec3 = np.array([[1, 2, 3], [5, 0, 1]])
    w3 = rng.standard_normal(g3.nt)
    src3 = (3, 1, 4)
    d_pt = core.forward(m3, w3, rec3, src_pos=src3)
    d_dn = core.forward(m3, core.with_point_source(g3, np.zeros((g3.nt, *g3.phys_shape)), w3, src3), rec3)
    assert _rel(d_dn, d_pt) < 1e-14


@pytest.fixture(scope="module")
def wri_system():
    """Tiny 2D system: data of a model 5% faster everywhere (the grid is too small
    for reflections within nt), so d - S f is the arrival-time misfit of the
    direct wave; S and S^T S + beta I formed densely."""
    cfg = inputs.cfg_tiny()
    g = core.Grid(2, cfg.nz, cfg.nx, nb=cfg.nb, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt)
    m = core.make_model(g, cfg.v_true)
    v_obs = cfg.v_true.astype(np.float64).copy()
    v_obs *= 1.05
    eta = core.eta_max_default(float(cfg.v_true.max()), g.nb, g.dx)
    m = core.make_model(g, cfg.v_true, eta_max=eta)
    m_obs = core.make_model(g, v_obs, eta_max=eta)
    rec = cfg.shot_rec(0)
    src = tuple(cfg.src[0])
    w = cfg.wavelet.astype(np.float64)
    d = core.forward(m_obs, w, rec, src_pos=src)
    nin = g.nt * g.nz * g.nx
    S = dense.dense_matrix(lambda q: core.forward(m, q, rec), nin, (g.nt, g.nz, g.nx))
    beta = 0.05
    N = S.T @ S + beta * np.eye(nin)
    d_f = S @ core.with_point_source(g, np.zeros((g.nt, g.nz, g.nx)), w, src).ravel()
    q_star = dense.cholesky_solve(N, S.T @ (d.ravel() - d_f))
    return dict(g=g, m=m, rec=rec, src=src, w=w, d=d, S=S, N=N, beta=beta, d_f=d_f,
                q_star=q_star.reshape(g.nt, g.nz, g.nx), eta=eta, cfg=cfg)


def test_wri_normal_operator_is_unit_weight(wri_system):
    """The WRI operator S^T S + beta I (eq. (normalwri)) is the ESI normal
    operator with B = I: the matrix-free form matches the dense one."""
    t = wri_system
    g = t["g"]
    ones = np.ones(g.phys_shape)
    Nm = dense.dense_matrix(lambda p: core.normal_apply(t["m"], t["rec"], ones, t["beta"], p),
                            t["N"].shape[0], (g.nt, g.nz, g.nx))
    assert np.max(np.abs(Nm - t["N"])) < 1e-12 * np.max(np.abs(t["N"]))


def test_wri_rhs_dense(wri_system):
    """wri_rhs = S^T (d - S f) with S and f taken from the dense matrix."""
    t = wri_system
    b = core.wri_rhs(t["m"], t["w"], t["src"], t["rec"], t["d"])
    # d - S f cancels part of d, which magnifies rounding
    assert np.linalg.norm(t["d"].ravel() - t["d_f"]) > 0.05 * np.linalg.norm(t["d"])
    assert _rel(b, t["S"].T @ (t["d"].ravel() - t["d_f"])) < 1e-10


def test_wri_solution_identities(wri_system):
    """At the solution q* of eq. (normalwri):
    * beta q* = S^T (d - S (f + q*)) (the WRI adjoint field of Table (compare));
    * J_WRI = 1/2 dd^T W1 dd with W1 = I + S S^T / beta (eq. (wrieqfwi));
    * q* = S^T (S S^T + beta I)^{-1} (d - S f) (data-space route);
    * CG (Algorithm 1) on the matrix-free operator reaches q*."""
    t = wri_system
    g, m, beta, q = t["g"], t["m"], t["beta"], t["q_star"]
    d_fq = core.forward(m, core.with_point_source(g, q, t["w"], t["src"]), t["rec"])
    dd = t["d"] - d_fq
    lam = core.adjoint(m, t["rec"], dd)
    assert _rel(beta * q, lam) < 1e-9
    S = t["S"]
    W1 = np.eye(S.shape[0]) + S @ S.T / beta
    J = core.misfit_wri(m, t["w"], t["src"], q, t["rec"], t["d"], beta)
    assert abs(J - 0.5 * dd.ravel() @ W1 @ dd.ravel()) < 1e-9 * J
    q_smw = dense.smw_extended_source(S, np.ones(S.shape[1]), beta, t["d"].ravel() - t["d_f"])
    assert _rel(q_smw, q) < 1e-8      # both direct routes carry ~cond(N) eps error
    res = core.wri_cg(m, t["w"], t["src"], t["rec"], t["d"], beta, max_iter=3000, rtol=1e-13)
    assert _rel(res.x, q) < 1e-8


def test_wri_penalty_equals_adjoint_at_optimum(wri_system):
    """With q = q*, lambda = beta q equals the adjoint field of the data residual,
    so the PENALTY and ADJOINT forms of the WRI gradient coincide; before
    convergence they differ."""
    t = wri_system
    m, beta = t["m"], t["beta"]
    gp = core.gradient_wri_penalty(m, t["w"], t["src"], t["q_star"], beta)
    ga = core.gradient_wri_adjoint(m, t["w"], t["src"], t["q_star"], t["rec"], t["d"])
    assert _rel(gp, ga) < 1e-8
    q2 = core.wri_cg(m, t["w"], t["src"], t["rec"], t["d"], beta, max_iter=2).x
    gp2 = core.gradient_wri_penalty(m, t["w"], t["src"], q2, beta)
    ga2 = core.gradient_wri_adjoint(m, t["w"], t["src"], q2, t["rec"], t["d"])
    assert _rel(gp2, ga2) > 1e-3
    # the physical source matters: leaving f out of u changes the gradient
    g0 = core.gradient_penalty(m, t["q_star"], np.ones(t["g"].phys_shape), beta)
    assert _rel(g0, gp) > 1e-2


def _model_m(g, mm, eta):
    return core.make_model(g, 1.0 / np.sqrt(mm), eta_max=eta)


def test_wri_gradient_adjoint_vs_fd():
    """d/dm of 1/2 ||S(m)(f + q) - d||^2 at fixed q (central differences in
    m = 1/v^2) against the ADJOINT form of the WRI gradient."""
    rng = np.random.default_rng(17)
    nz, nx = 22, 26
    g = core.Grid(2, nz, nx, nb=6, nt=140, dx=10.0, dt=1e-3)
    v0 = 2000.0 + 300.0 * rng.random((nz, nx))
    eta = core.eta_max_default(3000.0, g.nb, g.dx)
    m0 = 1.0 / v0 ** 2
    rec = np.stack([np.arange(1, nx, 3), np.full(9, 2)], axis=1)
    src = (13, 2)
    w = inputs.ricker_samples(g.nt, g.dt, 20.0).astype(np.float64)
    q = 0.3 * rng.standard_normal((g.nt, nz, nx))
    d_obs = rng.standard_normal((g.nt, len(rec))) * 1e-2
    grad = core.gradient_wri_adjoint(_model_m(g, m0, eta), w, src, q, rec, d_obs)
    zz, xx = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    # the perturbation stays off the edge cells, whose values the pad copies (the
    # gradient is taken with the pad held fixed)
    dm = np.exp(-((zz - 11) ** 2 + (xx - 12) ** 2) / 16.0) * rng.standard_normal((nz, nx)) \
        * (zz >= 4) * (zz < nz - 4) * (xx >= 4) * (xx < nx - 4)
    dm_s = dm * m0 * 1e-4

    def J(mm):
        return core.misfit_wri(_model_m(g, mm, eta), w, src, q, rec, d_obs, 0.7)
    fd = (J(m0 + dm_s) - J(m0 - dm_s)) / 2.0
    assert abs(fd - core.dot(grad, dm_s)) / abs(fd) < 1e-6


def test_wri_reduced_gradient_vs_fd(wri_system):
    """Variable projection: d/dm of J_WRI(m, q*(m)) equals the gradient at fixed
    q* (q* from a direct solve at every model), by central differences."""
    t = wri_system
    g, beta, eta = t["g"], t["beta"], t["eta"]
    m0 = 1.0 / t["cfg"].v_true.astype(np.float64) ** 2
    nin = g.nt * g.nz * g.nx

    def solve(mm):
        mod = _model_m(g, mm, eta)
        S = dense.dense_matrix(lambda q: core.forward(mod, q, t["rec"]), nin, (g.nt, g.nz, g.nx))
        d_f = S @ core.with_point_source(g, np.zeros((g.nt, g.nz, g.nx)), t["w"], t["src"]).ravel()
        q = dense.cholesky_solve(S.T @ S + beta * np.eye(nin), S.T @ (t["d"].ravel() - d_f))
        return mod, q.reshape(g.nt, g.nz, g.nx)

    mod, q = solve(m0)
    grad = core.gradient_wri_penalty(mod, t["w"], t["src"], q, beta)
    rng = np.random.default_rng(5)
    dm = np.zeros_like(m0)
    dm[2:6, 2:6] = rng.standard_normal((4, 4))
    dm_s = dm * m0 * 1e-4

    def Jred(mm):
        mo, qq = solve(mm)
        return core.misfit_wri(mo, t["w"], t["src"], qq, t["rec"], t["d"], beta)
    fd = (Jred(m0 + dm_s) - Jred(m0 - dm_s)) / 2.0
    assert abs(fd - core.dot(grad, dm_s)) / abs(fd) < 1e-6
