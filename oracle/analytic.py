"""Closed-form wavefields used to pin the oracle (test infrastructure only).

For A = (1/v^2) d_t^2 - Laplacian (eq. (wave), Sec. 2.1) in a homogeneous
medium the causal Green's function is

  2D:  G(r, t) = v H(v t - r) / (2 pi sqrt(v^2 t^2 - r^2))
  3D:  G(r, t) = delta(t - r / v) / (4 pi r)

A grid source of value w on one cell stands for a point source of strength
w dx^D, so the discrete field should approach dx^D (G * w)(r, t).  With
v t = r cosh(s) the 2D convolution becomes (1 / 2 pi) int_0^{acosh(vt/r)}
w(t - (r/v) cosh s) ds, which is smooth and is integrated by Gauss-Legendre.
"""
from __future__ import annotations

import numpy as np


def ricker(t: np.ndarray, f: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet of peak frequency f, delayed by t0 (default 1/f), zero for t < 0."""
    if t0 is None:
        t0 = 1.0 / f
    a = (np.pi * f * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    w = (1.0 - 2.0 * a) * np.exp(-a)
    return np.where(np.asarray(t) >= 0.0, w, 0.0)


def green2d_ricker(r: np.ndarray, t: np.ndarray, v: float, f: float, dx: float,
                   nodes: int = 400) -> np.ndarray:
    """dx^2 (G_2D * w)(r, t) for the Ricker w; r [nr] metres, t [nt] seconds -> [nt, nr]."""
    r = np.asarray(r, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    out = np.zeros((t.size, r.size))
    for j, rj in enumerate(r):
        ratio = v * t / rj
        live = ratio > 1.0
        smax = np.arccosh(np.where(live, ratio, 1.0))           # [nt]
        s = 0.5 * smax[:, None] * (xg[None, :] + 1.0)           # [nt, nodes]
        tau = t[:, None] - (rj / v) * np.cosh(s)
        val = ricker(tau, f) @ wg * 0.5 * smax
        out[:, j] = np.where(live, val, 0.0) / (2.0 * np.pi)
    return out * dx * dx


def green3d_ricker(r: np.ndarray, t: np.ndarray, v: float, f: float, dx: float) -> np.ndarray:
    """dx^3 w(t - r/v) / (4 pi r); r [nr] metres, t [nt] seconds -> [nt, nr]."""
    r = np.asarray(r, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return dx ** 3 * ricker(t[:, None] - r[None, :] / v, f) / (4.0 * np.pi * r[None, :])
