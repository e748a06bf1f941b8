"""FP64 oracle of the frequency-domain ESI solved with time-domain modelling
(Sec. 5.2: eq. (dtft), eq. (idtft), eq. (normaldtft)).

TEST INFRASTRUCTURE ONLY.  Like ``core``, this is the plain definition the GPU
library is checked against; only ``tests/``, the smoke check and the bench
CPU baseline may use it.

Readings:
* F maps a time series to its DTFT at the chosen frequencies f_m,
  (F u)_m = sum_n u_n exp(+j 2 pi f_m n dt) (eq. (dtft)).
* The inverse of eq. (idtft) is read as its real part,
  (G s)_n = (1/nt) Re sum_m s_m exp(-j 2 pi f_m n dt): the modelling needs a
  real source.  Under the real inner product <a, b> = Re sum conj(a) b of the
  frequency vectors, G = F^* / nt (pinned), so M = F N G is symmetric positive
  definite and CG (Algorithm 1) runs on the N_f complex slices per cell with
  that inner product; the paper's remark that the 1/nt factor only scales M
  applies unchanged.
* The penalty term is applied exactly, F (beta W) G = beta W (F G), with
  F G an N_f x N_f real-linear map of each cell's slices (half the identity
  for frequencies on the DFT grid of nt dt, other than 0 and Nyquist).
* The data enter as d = G F d_obs (eq. (normaldtft): the observed data
  represented through the inverse DTFT of their DTFT), so the right-hand side
  is F S^T G F d_obs.
* The gradient is Algorithm 2's PENALTY form with the time-domain source
  q = G q_bar.
"""
from __future__ import annotations

import numpy as np

from . import core


def twiddles(freqs, nt: int, dt: float) -> np.ndarray:
    """exp(+j 2 pi f_m n dt), complex [nt, nf]."""
    n = np.arange(nt)[:, None]
    return np.exp(2j * np.pi * np.asarray(freqs, dtype=np.float64)[None, :] * n * dt)


def dtft(u: np.ndarray, freqs, dt: float) -> np.ndarray:
    """(F u)_m = sum_n u_n exp(+j 2 pi f_m n dt) along axis 0: complex [nf, ...]."""
    E = twiddles(freqs, u.shape[0], dt)
    return np.tensordot(E.T, u, axes=(1, 0))


def idtft(s: np.ndarray, freqs, dt: float, nt: int) -> np.ndarray:
    """(G s)_n = (1/nt) Re sum_m s_m exp(-j 2 pi f_m n dt): real [nt, ...]."""
    E = np.conj(twiddles(freqs, nt, dt))
    return np.real(np.tensordot(E, s, axes=(1, 0))) / nt


def rdot(a: np.ndarray, b: np.ndarray) -> float:
    """Real inner product Re sum conj(a) b of frequency vectors."""
    return float(np.real(np.vdot(a.ravel(), b.ravel())))


def normal_apply(m: core.Model, rec, w2: np.ndarray, beta: float, p_bar: np.ndarray, freqs) -> np.ndarray:
    """M p_bar = F (S^T S + beta W) G p_bar (eq. (normaldtft))."""
    g = m.g
    q = idtft(p_bar, freqs, g.dt, g.nt)
    return dtft(core.normal_apply(m, rec, w2, beta, q), freqs, g.dt)


def rhs(m: core.Model, rec, d_obs: np.ndarray, freqs) -> np.ndarray:
    """F S^T G F d_obs (eq. (normaldtft) with d = G F d_obs)."""
    g = m.g
    d = idtft(dtft(d_obs, freqs, g.dt), freqs, g.dt, g.nt)
    return dtft(core.adjoint(m, rec, d), freqs, g.dt)


def _real(z):
    return np.stack([z.real, z.imag], axis=-1)


def _cplx(x):
    return x[..., 0] + 1j * x[..., 1]


def cg(m: core.Model, src_pos, rec, d_obs, beta: float, freqs, max_iter: int, rtol: float = 0.0,
       eps: float = 1.0) -> core.CGResult:
    """Algorithm 1 on M q_bar = F S^T G F d_obs with the real inner product:
    core.cg on the (real, imaginary) pairs.  The result's x is complex [nf, *phys]."""
    w2 = core.annihilator_sq(m.g, src_pos, eps)
    b = _real(rhs(m, rec, d_obs, freqs))
    res = core.cg(lambda p: _real(normal_apply(m, rec, w2, beta, _cplx(p), freqs)), b, max_iter, rtol)
    res.x = _cplx(res.x)
    return res


def gradient_penalty(m: core.Model, q_bar: np.ndarray, w2: np.ndarray, beta: float, freqs) -> np.ndarray:
    """Algorithm 2's gradient with the time-domain extended source q = G q_bar."""
    g = m.g
    return core.gradient_penalty(m, idtft(q_bar, freqs, g.dt, g.nt), w2, beta)
