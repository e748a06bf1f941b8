"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws and shapes inputs: velocity models, acquisition
geometry, source wavelets and random test vectors.  It holds none of the
method's arithmetic (no propagation, no operator, no solver) and imports
nothing else from the package, so the FP64 oracle and the GPU path can both
consume its output.  Every generator works in float64 from
``numpy.random.default_rng(seed)`` and rounds once to float32; both sides use
those float32 values.

The paper's own workloads (Sec. 4: a two-layer reflection model, a 1D layered
landscape model and Marmousi-II with 28 surface shots, 641 receivers and a
5 Hz Ricker) are not available; the configurations below stand in for them
with the same acquisition style: surface sources and receivers, a 1500 m/s
top layer and Ricker sources.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def ricker_samples(nt: int, dt: float, f: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet of peak frequency f sampled at t_n = n dt, delay t0 = 1/f.

    w(t) = (1 - 2 pi^2 f^2 (t - t0)^2) exp(-pi^2 f^2 (t - t0)^2); float32 [nt].
    """
    if t0 is None:
        t0 = 1.0 / f
    t = np.arange(nt, dtype=np.float64) * dt
    a = (np.pi * f * (t - t0)) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


@dataclass
class Config:
    """One workload: grid, time axis, geometry, models and solver settings."""
    name: str
    ndim: int
    nz: int
    nx: int
    ny: int
    dx: float
    dt: float
    nt: int
    nb: int
    freq: float
    beta: float
    cg_iters: int
    v_true: np.ndarray                 # float32 [nz][(ny)][nx]
    v_start: np.ndarray                # float32, model the solve runs in
    src: np.ndarray                    # int32 [nshots][ndim] (ix, iz[, iy])
    rec_ptr: np.ndarray                # int64 [nshots+1]
    rec: np.ndarray                    # int32 [nrec_total][ndim]
    wavelet: np.ndarray                # float32 [nt]
    b_eps: float = 1.0
    notes: dict = field(default_factory=dict)
    window: np.ndarray | None = None    # int32 [nshots][2] physical columns [x0, x1) per shot

    @property
    def nshots(self) -> int:
        return int(self.src.shape[0])

    @property
    def phys_shape(self):
        return (self.nz, self.nx) if self.ndim == 2 else (self.nz, self.ny, self.nx)

    def shot_rec(self, s: int) -> np.ndarray:
        return self.rec[self.rec_ptr[s]:self.rec_ptr[s + 1]]


def _csr(recs):
    ptr = np.zeros(len(recs) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in recs])
    return ptr, np.concatenate(recs).astype(np.int32)


def cfg_small() -> Config:
    """201 x 201 grid, dx 10 m, v = 2000 m/s, one 10 Hz Ricker at (100, 5),
    201 receivers along row 5, 500 steps of 1 ms, 20-cell sponge, beta 1e-2,
    5 CG iterations (the small parity workload)."""
    nz = nx = 201
    v = np.full((nz, nx), 2000.0, dtype=np.float32)
    src = np.array([[100, 5]], dtype=np.int32)
    rec = np.stack([np.arange(nx), np.full(nx, 5)], axis=1).astype(np.int32)
    ptr, rr = _csr([rec])
    return Config("small-201x201", 2, nz, nx, 1, 10.0, 1e-3, 500, 20, 10.0, 1e-2, 5,
                  v, v.copy(), src, ptr, rr, ricker_samples(500, 1e-3, 10.0))


def layered_model(nz: int, nx: int, seed: int, water_cells: int = 40) -> np.ndarray:
    """1500 m/s water over 5 layers (sorted U[1700, 4500] m/s, tops at cell 40
    and at 4 sorted U[60, 380] depths) with 3 Gaussian anomalies of +-10 %
    (centres uniform below the water, sigma U[15, 40] cells); float64."""
    rng = np.random.default_rng(seed)
    vel = np.sort(rng.uniform(1700.0, 4500.0, 5))
    tops = np.concatenate([[water_cells], np.sort(rng.uniform(60.0, 0.95 * nz, 4))])
    z = np.arange(nz, dtype=np.float64)[:, None]
    v = np.full((nz, nx), 1500.0)
    for vk, tk in zip(vel, tops):
        v = np.where(z >= tk, vk, v)
    zz, xx = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(nx, dtype=np.float64),
                         indexing="ij")
    for _ in range(3):
        cz = rng.uniform(water_cells + 20, nz)
        cx = rng.uniform(0, nx)
        sig = rng.uniform(15.0, 40.0)
        amp = 0.1 * rng.choice([-1.0, 1.0])
        v = v * (1.0 + amp * np.exp(-((zz - cz) ** 2 + (xx - cx) ** 2) / (2 * sig * sig)))
    return v


def smooth_model(v: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian-smoothed start model (sigma in cells, nearest-edge boundary)."""
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(np.asarray(v, dtype=np.float64), sigma=sigma, mode="nearest")


def cfg_single_solve(nshots: int = 32, nx: int = 801, nz: int = 401, nt: int = 2000,
                     seed: int = 1) -> Config:
    """801 x 401 grid, dx 12.5 m, layered 1500-4500 m/s with 3 anomalies (seed 1),
    32 shots of an 8 Hz Ricker at depth cell 2 (x evenly 12..788), 401 receivers
    at depth cell 2 every 2nd cell, 2000 steps of 1 ms, start model smoothed
    with sigma 10 cells, 20 CG iterations, beta 1e-2 (the single-solve workload)."""
    v_true = layered_model(nz, nx, seed)
    v_start = smooth_model(v_true, 10.0)
    xs = np.round(np.linspace(12, nx - 13, nshots)).astype(np.int32)
    src = np.stack([xs, np.full(nshots, 2)], axis=1).astype(np.int32)
    rx = np.arange(0, nx, 2)
    rec1 = np.stack([rx, np.full(rx.size, 2)], axis=1).astype(np.int32)
    ptr, rr = _csr([rec1] * nshots)
    return Config("single-solve-801x401", 2, nz, nx, 1, 12.5, 1e-3, nt, 20, 8.0, 1e-2, 20,
                  v_true.astype(np.float32), v_start.astype(np.float32), src, ptr, rr,
                  ricker_samples(nt, 1e-3, 8.0))


def cfg_tiny(nz: int = 8, nx: int = 8, nt: int = 24, nb: int = 4, seed: int = 7,
             nrec: int = 4, dx: float = 10.0, dt: float = 1e-3) -> Config:
    """Tiny heterogeneous 2D grid on which dense operators can be formed."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(1800.0, 2600.0, (nz, nx))
    src = np.array([[nx // 2, 1]], dtype=np.int32)
    rx = np.linspace(0, nx - 1, nrec).round().astype(np.int32)
    rec = np.stack([rx, np.full(nrec, 1)], axis=1).astype(np.int32)
    ptr, rr = _csr([rec])
    return Config("tiny", 2, nz, nx, 1, dx, dt, nt, nb, 25.0, 1e-2, 10,
                  v.astype(np.float32), v.astype(np.float32), src, ptr, rr,
                  ricker_samples(nt, dt, 25.0))


def random_field(shape, seed: int) -> np.ndarray:
    """Seeded N(0, 1) float32 array (dot-test and parity vectors)."""
    return np.random.default_rng(seed).standard_normal(shape).astype(np.float32)


def gaussian_random_field(shape, sigma: float, seed: int) -> np.ndarray:
    """White N(0, 1) noise smoothed by a Gaussian of sigma cells (periodic FFT
    filter), standardized to zero mean and unit variance; float64."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    k = [np.fft.fftfreq(n) for n in shape]
    kk = np.zeros(shape)
    for ax, ka in enumerate(k):
        sh = [1] * len(shape)
        sh[ax] = -1
        kk = kk + (ka.reshape(sh)) ** 2
    field = np.real(np.fft.ifftn(np.fft.fftn(white) * np.exp(-2.0 * (np.pi * sigma) ** 2 * kk)))
    return (field - field.mean()) / field.std()


def cfg_diff3d(n: int = 256, nshots: int = 8, nt: int = 1500, rec_n: int = 128, seed: int = 3,
               dx: float = 10.0, dt: float = 1e-3, f: float = 10.0, nb: int = 20) -> Config:
    """3D n^3 grid, dx 10 m, v = 3000 + 300 * (Gaussian random field, sigma 16
    cells) clipped to [2000, 4000] m/s (seed 3); `nshots` shots at depth cell 2
    on a 2 x 4 lattice; a rec_n x rec_n receiver grid at depth cell 2, every
    2nd cell; 10 Hz Ricker, nt steps of 1 ms (the differentiation workload)."""
    field = gaussian_random_field((n, n, n), 16.0 * n / 256.0, seed)
    v = np.clip(3000.0 + 300.0 * field, 2000.0, 4000.0).astype(np.float32)   # [z][y][x]
    px = np.round(np.linspace(n / 8, n - n / 8, 4)).astype(int)
    py = np.round(np.linspace(n / 4, n - n / 4, 2)).astype(int)
    lattice = [(x, 2, y) for y in py for x in px][:nshots]
    src = np.array(lattice, dtype=np.int32)                                  # (ix, iz, iy)
    step = max(1, min(2, n // rec_n))
    r1 = np.arange(rec_n) * step + (n - (rec_n - 1) * step - 1) // 2
    ry, rx = np.meshgrid(r1, r1, indexing="ij")
    rec1 = np.stack([rx.ravel(), np.full(rx.size, 2), ry.ravel()], axis=1).astype(np.int32)
    ptr, rr = _csr([rec1] * len(src))
    return Config(f"diff3d-{n}^3", 3, n, n, n, dx, dt, nt, nb, f, 1e-2, 0, v, v.copy(), src, ptr,
                  rr, ricker_samples(nt, dt, f))


def crop3d(cfg: Config, n: int, nt: int, rec_n: int) -> Config:
    """Central n^3 block of a 3D workload with one shot at its top centre and a
    rec_n x rec_n receiver grid (every 2nd cell) at depth cell 2."""
    N = cfg.nz
    o = (N - n) // 2
    v = np.ascontiguousarray(cfg.v_true[o:o + n, o:o + n, o:o + n])
    src = np.array([[n // 2, 2, n // 2]], dtype=np.int32)
    r1 = np.arange(rec_n) * 2 + (n - (rec_n - 1) * 2 - 1) // 2
    ry, rx = np.meshgrid(r1, r1, indexing="ij")
    rec1 = np.stack([rx.ravel(), np.full(rx.size, 2), ry.ravel()], axis=1).astype(np.int32)
    ptr, rr = _csr([rec1])
    return Config(f"crop3d-{n}^3", 3, n, n, n, cfg.dx, cfg.dt, nt, min(cfg.nb, 12), cfg.freq,
                  cfg.beta, 0, v, v.copy(), src, ptr, rr, ricker_samples(nt, cfg.dt, cfg.freq))


def he_init(segments, seed: int) -> np.ndarray:
    """Seeded initial network parameters: for each (n_weights, fan_in, n_bias)
    segment, n_weights draws of N(0, 2 / fan_in) followed by n_bias zeros
    (He et al. 2015); float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for n, fan, nb in segments:
        parts.append(rng.standard_normal(n) * np.sqrt(2.0 / fan))
        parts.append(np.zeros(nb))
    return np.concatenate(parts).astype(np.float32)


def cfg_precond(seed: int, nx: int = 401, nz: int = 201, nshots: int = 4, nt: int = 1500,
                sigma: float | None = None) -> Config:
    """A model of the learned-preconditioner workloads: the single-solve
    recipe (water over 5 layers with 3 anomalies, dx 12.5 m, 8 Hz Ricker,
    receivers every 2nd cell and shots at depth cell 2, beta 1e-2) on an
    nx x nz grid with `nshots` evenly spaced shots and nt steps of 1 ms; start
    model smoothed with sigma = 10 nz / 401 cells.  Training models use seeds
    5000..5199 at 401 x 201, held-out models seeds 6000..6009 at 801 x 401."""
    v_true = layered_model(nz, nx, seed)
    v_start = smooth_model(v_true, 10.0 * nz / 401.0 if sigma is None else sigma)
    xs = np.round(np.linspace(12, nx - 13, nshots)).astype(np.int32)
    src = np.stack([xs, np.full(nshots, 2)], axis=1).astype(np.int32)
    rx = np.arange(0, nx, 2)
    rec1 = np.stack([rx, np.full(rx.size, 2)], axis=1).astype(np.int32)
    ptr, rr = _csr([rec1] * nshots)
    return Config(f"precond-{nx}x{nz}-seed{seed}", 2, nz, nx, 1, 12.5, 1e-3, nt, 20, 8.0, 1e-2, 0,
                  v_true.astype(np.float32), v_start.astype(np.float32), src, ptr, rr,
                  ricker_samples(nt, 1e-3, 8.0))


def layered_fault_model(nz: int, nx: int, seed: int, vmin: float = 1500.0, vmax: float = 5000.0,
                        nlayers: int = 8) -> np.ndarray:
    """nlayers layers from vmin at the top to vmax (velocities jittered by
    U[-5, 5] % and sorted, tops at sorted U[20, 0.95 nz] cells below a vmin
    layer) cut by one normal fault: dip U[20, 40] degrees, throw U[20, 40]
    cells, through a point at x U[0.3, 0.7] nx on the surface; the hanging
    wall (right of the fault plane) drops by the throw; float64."""
    rng = np.random.default_rng(seed)
    vel = np.linspace(vmin, vmax, nlayers) * (1.0 + rng.uniform(-0.05, 0.05, nlayers))
    vel = np.clip(np.sort(vel), vmin, vmax)
    tops = np.sort(rng.uniform(20.0, 0.95 * nz, nlayers - 1))
    dip = np.deg2rad(rng.uniform(20.0, 40.0))
    throw = rng.uniform(20.0, 40.0)
    xf = rng.uniform(0.3, 0.7) * nx
    zz, xx = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    hanging = xx > xf + zz / np.tan(dip)
    depth = np.where(hanging, zz - throw, zz)
    v = np.full((nz, nx), vel[0])
    for vk, tk in zip(vel[1:], tops):
        v = np.where(depth >= tk, vk, v)
    return v


def cfg_batching(nshots: int = 128, nx: int = 1601, nz: int = 601, nt: int = 4000, seed: int = 2,
                 dt: float = 0.8e-3, f: float = 10.0, margin: int = 50) -> Config:
    """The uneven-aperture batching workload: 1601 x 601 grid, dx 10 m, layered
    model with one normal fault, 1500-5000 m/s (seed 2); `nshots` shots at
    depth cell 2, x evenly from 50 to nx - 51; each shot records on a
    split spread of U{101..801} receivers at 1-cell spacing around its source
    (clipped to the grid); its aperture is the receiver span plus `margin`
    cells each side; 10 Hz Ricker, nt steps of 0.8 ms."""
    rng = np.random.default_rng(seed)
    v = layered_fault_model(nz, nx, seed).astype(np.float32)
    xs = np.round(np.linspace(50, nx - 51, nshots)).astype(np.int32)
    src = np.stack([xs, np.full(nshots, 2)], axis=1).astype(np.int32)
    recs, win = [], []
    for s in range(nshots):
        n = int(rng.integers(101, 802))
        lo = max(0, int(xs[s]) - n // 2)
        hi = min(nx, lo + n)
        lo = max(0, hi - n)
        rx = np.arange(lo, hi)
        recs.append(np.stack([rx, np.full(rx.size, 2)], axis=1))
        win.append([max(0, lo - margin), min(nx, hi + margin)])
    ptr, rr = _csr(recs)
    cfg = Config(f"batching-{nx}x{nz}-{nshots}shots", 2, nz, nx, 1, 10.0, dt, nt, 20, f, 1e-2, 0, v, v.copy(),
                 src, ptr, rr, ricker_samples(nt, dt, f))
    cfg.window = np.asarray(win, dtype=np.int32)
    return cfg
