"""Pins of the data-space oracle (Sec. 5.1): the data-space operator against
its dense matrix, symmetry and definiteness, the extended source against the
wavefield-space direct solve, the synthetic data tending to d as beta -> 0,
and the WRI form (eq. (wriw))."""
import numpy as np

from oracle import core, dataspace, dense
from paper_2211_06300_amd import inputs


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _tiny():
    cfg = inputs.cfg_tiny()
    g = core.Grid(2, cfg.nz, cfg.nx, nb=cfg.nb, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt)
    m = core.make_model(g, cfg.v_true)
    rec = cfg.shot_rec(0)
    src = tuple(cfg.src[0])
    nin = g.nt * g.nz * g.nx
    S = dense.dense_matrix(lambda q: core.forward(m, q, rec), nin, (g.nt, g.nz, g.nx))
    return cfg, g, m, rec, src, S


def test_K_dense_symmetric():
    """S W^{-1} S^T formed matrix-free equals the dense product and is symmetric
    positive semi-definite."""
    cfg, g, m, rec, src, S = _tiny()
    w2 = core.annihilator_sq(g, src)
    nd = g.nt * len(rec)
    K = dense.dense_matrix(lambda w: dataspace.K_apply(m, rec, w2, w), nd, (g.nt, len(rec)))
    Kd = S @ (np.tile(1.0 / w2.ravel(), g.nt)[:, None] * S.T)
    assert np.max(np.abs(K - Kd)) < 1e-12 * np.max(np.abs(Kd))
    assert np.max(np.abs(K - K.T)) < 1e-12 * np.max(np.abs(K))
    assert np.min(np.linalg.eigvalsh(0.5 * (K + K.T))) > -1e-12 * np.max(np.abs(K))


def test_q_equals_wavefield_solution():
    """q from the data-space CG equals the wavefield-space direct solve of
    eq. (normalewi); the residual identity eq. (wd) holds at the solution."""
    cfg, g, m, rec, src, S = _tiny()
    w2 = core.annihilator_sq(g, src)
    beta = 0.05
    d = core.forward(m, cfg.wavelet.astype(np.float64), rec, src_pos=src)
    W = np.tile(w2.ravel(), g.nt)
    q_star = dense.cholesky_solve(S.T @ S + beta * np.diag(W), S.T @ d.ravel())
    w, q, res = dataspace.cg(m, src, rec, d, beta, max_iter=500, rtol=1e-13)
    # q = (beta W)^{-1} S^T (d - w) magnifies the solve's rounding by 1/beta and
    # by the cancellation in d - w
    assert _rel(q, q_star) < 1e-7
    # eq. (wd): (I + S (beta W)^{-1} S^T) w = S (beta W)^{-1} S^T d
    lhs = w.ravel() + S @ (S.T @ w.ravel() / (beta * W))
    rhs = S @ (S.T @ d.ravel() / (beta * W))
    assert _rel(lhs, rhs) < 1e-9
    # and w is the synthetic data of q: w = S q
    assert _rel(w.ravel(), S @ q.ravel()) < 1e-8


def test_w_tends_to_d_as_beta_vanishes():
    """The synthetic data w fit d ever more closely as beta -> 0 (Sec. 5.1)."""
    cfg, g, m, rec, src, S = _tiny()
    w2 = core.annihilator_sq(g, src)
    d = core.forward(m, cfg.wavelet.astype(np.float64), rec, src_pos=src)
    Winv = np.tile(1.0 / w2.ravel(), g.nt)
    K = S @ (Winv[:, None] * S.T)
    errs = []
    for beta in [1.0, 1e-1, 1e-2, 1e-3]:
        w = np.linalg.solve(beta * np.eye(len(K)) + K, K @ d.ravel())
        errs.append(np.linalg.norm(w - d.ravel()) / np.linalg.norm(d))
    assert all(b < a for a, b in zip(errs, errs[1:])) and errs[-1] < 0.1 * errs[0]


def test_wri_data_space():
    """WRI (B = I, d - S f): q from the data space equals the direct solve of
    eq. (normalwri), and R u = w + S f with u = A^{-1}(f + q) (Sec. 5.1)."""
    cfg, g, m, rec, src, S = _tiny()
    beta = 0.05
    v_obs = cfg.v_true.astype(np.float64) * 1.05
    d = core.forward(core.make_model(g, v_obs), cfg.wavelet.astype(np.float64), rec, src_pos=src)
    f = cfg.wavelet.astype(np.float64)
    d_f = core.forward(m, f, rec, src_pos=src)
    ones = np.ones(g.phys_shape)
    w, q, _ = dataspace.cg(m, src, rec, d - d_f, beta, max_iter=500, rtol=1e-13, w2=ones)
    q_star = dense.cholesky_solve(S.T @ S + beta * np.eye(S.shape[1]), S.T @ (d - d_f).ravel())
    # w fits d - S f to ~1e-3 here, so q = S^T (d - S f - w) / beta carries the
    # solve's error magnified about 1e3 times
    assert _rel(q, q_star) < 1e-5
    Ru = core.forward(m, core.with_point_source(g, q, f, src), rec)
    assert _rel(Ru, w + d_f) < 1e-8
