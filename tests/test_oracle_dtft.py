"""Pins of the DTFT oracle (Sec. 5.2): the transform against numpy's FFT on the
DFT grid, the adjoint relation G = F^* / nt under the real inner product,
F G = I / 2 on the grid, symmetry and definiteness of M = F N G, the dense
matrix of M, and a reconstruction of a band-limited signal through CG on
N_f frequencies (the paper's proof of concept, with an SPD Toeplitz matrix of
our own)."""
import numpy as np

from oracle import core, dense, dtft
from paper_2211_06300_amd import inputs


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def test_dtft_equals_fft_on_grid():
    """On the grid f = k / (nt dt), F u is the conjugate of numpy's FFT bin k
    (numpy uses exp(-j ...)); a cosine on the grid has F = nt / 2 at its own
    frequency and zero at the others."""
    rng = np.random.default_rng(1)
    nt, dt = 128, 2e-3
    u = rng.standard_normal(nt)
    ks = np.array([1, 5, 17, 40])
    freqs = ks / (nt * dt)
    assert np.max(np.abs(dtft.dtft(u, freqs, dt) - np.conj(np.fft.fft(u)[ks]))) < 1e-12 * np.linalg.norm(u) * nt
    c = np.cos(2 * np.pi * freqs[1] * np.arange(nt) * dt)
    F = dtft.dtft(c, freqs, dt)
    assert abs(F[1] - nt / 2) < 1e-9 and np.max(np.abs(np.delete(F, 1))) < 1e-9


def test_adjoint_relation():
    """<F u, s>_R = nt <u, G s> for any frequencies (on or off the grid)."""
    rng = np.random.default_rng(2)
    nt, dt = 90, 1e-3
    freqs = np.array([3.0, 7.3, 12.0, 29.9])
    u = rng.standard_normal((nt, 5))
    s = rng.standard_normal((4, 5)) + 1j * rng.standard_normal((4, 5))
    lhs = dtft.rdot(dtft.dtft(u, freqs, dt), s)
    rhs = nt * float(np.sum(u * dtft.idtft(s, freqs, dt, nt)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_FG_half_identity_on_grid():
    """F G s = s / 2 for grid frequencies other than 0 and Nyquist; off the grid
    it is not diagonal."""
    rng = np.random.default_rng(3)
    nt, dt = 200, 1.0 / 200
    s = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    on = np.array([1.0, 3.0, 5.0, 7.0, 9.0])
    assert np.max(np.abs(dtft.dtft(dtft.idtft(s, on, dt, nt), on, dt) - s / 2)) < 1e-12
    off = on + 0.37
    assert np.max(np.abs(dtft.dtft(dtft.idtft(s, off, dt, nt), off, dt) - s / 2)) > 1e-3


def _tiny(nt=30):
    cfg = inputs.cfg_tiny(nt=nt)
    g = core.Grid(2, cfg.nz, cfg.nx, nb=cfg.nb, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt)
    m = core.make_model(g, cfg.v_true)
    return cfg, g, m


def test_normal_operator_spd_and_dense():
    """M = F N G is symmetric and positive definite under the real inner product
    and equals F N F^* / nt formed densely."""
    cfg, g, m = _tiny()
    rec = cfg.shot_rec(0)
    src = tuple(cfg.src[0])
    w2 = core.annihilator_sq(g, src)
    freqs = np.array([20.0, 45.0, 80.0])
    rng = np.random.default_rng(4)
    a = rng.standard_normal((3, g.nz, g.nx)) + 1j * rng.standard_normal((3, g.nz, g.nx))
    b = rng.standard_normal((3, g.nz, g.nx)) + 1j * rng.standard_normal((3, g.nz, g.nx))
    Ma = dtft.normal_apply(m, rec, w2, cfg.beta, a, freqs)
    Mb = dtft.normal_apply(m, rec, w2, cfg.beta, b, freqs)
    assert abs(dtft.rdot(Ma, b) - dtft.rdot(a, Mb)) < 1e-12 * abs(dtft.rdot(Ma, b))
    assert dtft.rdot(Ma, a) > 0
    # dense: N (time domain) and F as a real 2 nf x nt map per cell
    nin = g.nt * g.nz * g.nx
    N = dense.dense_matrix(lambda p: core.normal_apply(m, rec, w2, cfg.beta, p), nin, (g.nt, g.nz, g.nx))
    E = dtft.twiddles(freqs, g.nt, g.dt)                     # [nt, nf]
    Fr = np.concatenate([E.real.T, E.imag.T])                # real rows then imaginary rows
    Fbig = np.kron(Fr, np.eye(g.nz * g.nx))                  # [2 nf cells, nt cells]
    M = Fbig @ N @ Fbig.T / g.nt
    av = np.concatenate([a.real.ravel(), a.imag.ravel()])
    Mv = M @ av
    k = len(freqs) * g.nz * g.nx
    assert _rel(Mv[:k] + 1j * Mv[k:], Ma.ravel()) < 1e-12


def test_band_limited_reconstruction():
    """Sec. 5.2's proof of concept: x(t) = sum_m sin(2 pi f_m t), f = 1, 3, 5, 7, 9
    Hz, nt = 200 samples on [0, 1); with an SPD Toeplitz N (here
    exp(-|i-j|/4) + 0.5 delta_ij) and b = N x, CG on F N G x_bar = F b over 5
    frequencies reconstructs x = G x_bar."""
    nt, dt = 200, 1.0 / 200
    freqs = np.array([1.0, 3.0, 5.0, 7.0, 9.0])
    t = np.arange(nt) * dt
    x = np.sum(np.sin(2 * np.pi * freqs[:, None] * t[None, :]), axis=0)
    idx = np.arange(nt)
    N = np.exp(-np.abs(idx[:, None] - idx[None, :]) / 4.0) + 0.5 * np.eye(nt)
    b = N @ x

    def M(xb):
        z = xb[..., 0] + 1j * xb[..., 1]
        y = dtft.dtft(N @ dtft.idtft(z, freqs, dt, nt), freqs, dt)
        return np.stack([y.real, y.imag], axis=-1)
    fb = dtft.dtft(b, freqs, dt)
    res = core.cg(M, np.stack([fb.real, fb.imag], axis=-1), max_iter=40, rtol=1e-14)
    xr = dtft.idtft(res.x[..., 0] + 1j * res.x[..., 1], freqs, dt, nt)
    assert _rel(xr, x) < 1e-10


def test_dtft_cg_and_gradient_shapes():
    """The frequency-domain CG reduces the residual, and the gradient with
    q = G q_bar is the time-domain PENALTY gradient of that source."""
    cfg, g, m = _tiny(nt=40)
    rec = cfg.shot_rec(0)
    src = tuple(cfg.src[0])
    d = core.forward(m, cfg.wavelet.astype(np.float64), rec, src_pos=src)
    freqs = np.array([15.0, 25.0, 35.0])
    res = dtft.cg(m, src, rec, d, cfg.beta, freqs, max_iter=12)
    assert res.res_hist[-1] < 0.5 and res.x.shape == (3, g.nz, g.nx)
    w2 = core.annihilator_sq(g, src)
    gp = dtft.gradient_penalty(m, res.x, w2, cfg.beta, freqs)
    ref = core.gradient_penalty(m, dtft.idtft(res.x, freqs, g.dt, g.nt), w2, cfg.beta)
    assert np.array_equal(gp, ref)


def test_rhs_dense():
    """F S^T G F d formed with the dense S and the DTFT as a real matrix."""
    cfg, g, m = _tiny(nt=30)
    rec = cfg.shot_rec(0)
    freqs = np.array([20.0, 45.0])
    rng = np.random.default_rng(6)
    d = rng.standard_normal((g.nt, len(rec)))
    b = dtft.rhs(m, rec, d, freqs)
    nin = g.nt * g.nz * g.nx
    S = dense.dense_matrix(lambda q: core.forward(m, q, rec), nin, (g.nt, g.nz, g.nx))
    E = dtft.twiddles(freqs, g.nt, g.dt)                     # [nt, nf]
    Fr = np.concatenate([E.real.T, E.imag.T])                # [2 nf, nt]
    band = Fr.T @ Fr / g.nt                                  # G F on one trace: nt x nt
    d_band = band @ d                                        # every receiver trace
    St_d = (S.T @ d_band.ravel()).reshape(g.nt, g.nz * g.nx)
    bv = Fr @ St_d                                           # [2 nf, cells]
    nf = len(freqs)
    assert _rel(bv[:nf] + 1j * bv[nf:], b.reshape(nf, -1)) < 1e-12
