"""FP64 CPU oracle for the time-domain ESI hot path (Yang & Zhou, arXiv 2211.06300).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
definition that the GPU library is checked against.  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may use
it.  It shares no code with the GPU path; the GPU path never imports it.

Every function cites the passage of the paper it follows.  Where the paper is
silent the reading taken is stated in the docstring.  The time loops are the C
file ``oracle/prop.c`` (double precision, serial reductions); this module builds
the padded model, the absorbing profile, the annihilator and the finite
difference weights, and writes out CG and the gradients step by step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "prop.c")


def build_oracle(force: bool = False) -> str:
    """Compile ``prop.c`` with gcc (plain -O2, no fast-math) into ``liboracle.so``."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("nz", ctypes.c_int), ("ny", ctypes.c_int),
                ("nx", ctypes.c_int), ("nb", ctypes.c_int), ("nt", ctypes.c_int),
                ("w", ctypes.c_double * 5), ("inv_dx2", ctypes.c_double),
                ("inv_dt2", ctypes.c_double)]


_lib = None


def _load(path: str | None = None):
    global _lib
    if path is not None:
        lib = ctypes.CDLL(path)
    else:
        if _lib is not None:
            return _lib
        lib = ctypes.CDLL(build_oracle())
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_long)
    lib.or_forward.argtypes = [ctypes.POINTER(_Grid), dp, dp, ctypes.c_int, dp, ctypes.c_long,
                               ctypes.c_int, lp, dp, dp]
    lib.or_adjoint.argtypes = [ctypes.POINTER(_Grid), dp, dp, ctypes.c_int, lp, dp, dp]
    lib.or_forward.restype = ctypes.c_int
    lib.or_adjoint.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------------------
# Discretisation (Sec. 4.1: O(dt^2, dx^8) scheme with an absorbing boundary)
# ---------------------------------------------------------------------------

def laplacian_weights(half_width: int = 4) -> tuple[Fraction, ...]:
    """Weights a_0..a_M of the centred second difference of order 2M.

    Sec. 4.1 fixes the spatial order at 8 (M = 4).  The weights solve the
    Taylor-matching system: with f(x+kh)+f(x-kh) = 2 sum_m (kh)^{2m} f^{(2m)}/(2m)!,
    require sum_k a_k k^2 = 1 and sum_k a_k k^{2m} = 0 for m = 2..M, and
    a_0 = -2 sum_k a_k (constants are annihilated).  Solved exactly in rationals.
    """
    M = half_width
    # rows m = 1..M: sum_{k=1..M} a_k k^{2m} = [m == 1]
    A = [[Fraction(k ** (2 * m)) for k in range(1, M + 1)] for m in range(1, M + 1)]
    b = [Fraction(1 if m == 1 else 0) for m in range(1, M + 1)]
    # Gauss-Jordan elimination in exact arithmetic
    n = M
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [ar - f * ac for ar, ac in zip(A[r], A[col])]
                b[r] -= f * b[col]
    a = [b[i] / A[i][i] for i in range(n)]
    a0 = -2 * sum(a)
    return (a0, *a)


@dataclass
class Grid:
    """Physical grid, pad and time axis.

    Readings (the paper gives only the FD order and "an absorbing boundary"):
    the absorbing layer is a damping term of width ``nb`` cells placed outside
    the physical grid on every side (this also removes the free surface, as
    Sec. 4.1 asks); beyond the pad the field is zero.  ``ndim`` 2 uses (z, x),
    3 uses (z, y, x); arrays are [z][y][x] with x fastest.
    """
    ndim: int
    nz: int
    nx: int
    ny: int = 1
    nb: int = 20
    nt: int = 500
    dx: float = 10.0
    dt: float = 1e-3

    @property
    def phys_shape(self):
        return (self.nz, self.nx) if self.ndim == 2 else (self.nz, self.ny, self.nx)

    @property
    def pad_shape(self):
        nb = self.nb
        if self.ndim == 2:
            return (self.nz + 2 * nb, self.nx + 2 * nb)
        return (self.nz + 2 * nb, self.ny + 2 * nb, self.nx + 2 * nb)

    def pad_index(self, pos) -> int:
        """Padded linear index of a physical position (ix, iz) or (ix, iz, iy)."""
        nb = self.nb
        if self.ndim == 2:
            ix, iz = int(pos[0]), int(pos[1])
            if not (0 <= ix < self.nx and 0 <= iz < self.nz):
                raise ValueError("position outside the physical grid")
            return (iz + nb) * (self.nx + 2 * nb) + ix + nb
        ix, iz, iy = int(pos[0]), int(pos[1]), int(pos[2])
        if not (0 <= ix < self.nx and 0 <= iz < self.nz and 0 <= iy < self.ny):
            raise ValueError("position outside the physical grid")
        nyp, nxp = self.ny + 2 * nb, self.nx + 2 * nb
        return ((iz + nb) * nyp + iy + nb) * nxp + ix + nb

    def _c(self) -> _Grid:
        g = _Grid()
        g.ndim, g.nz, g.ny, g.nx = self.ndim, self.nz, (self.ny if self.ndim == 3 else 1), self.nx
        g.nb, g.nt = self.nb, self.nt
        w = laplacian_weights(4)
        for k in range(5):
            g.w[k] = float(w[k])
        g.inv_dx2 = 1.0 / (self.dx * self.dx)
        g.inv_dt2 = 1.0 / (self.dt * self.dt)
        return g


def eta_max_default(vmax: float, nb: int, dx: float, reflection: float = 1e-3) -> float:
    """Peak damping of the absorbing layer, eta_max = 3 v_max ln(1/R) / (2 nb dx).

    Reading: the paper only says an absorbing boundary is used (Sec. 4.1); this
    is the usual quadratic damping profile for a target reflection R = 1e-3.
    """
    return 3.0 * vmax * np.log(1.0 / reflection) / (2.0 * nb * dx)


def pad_model(g: Grid, v: np.ndarray) -> np.ndarray:
    """Velocity on the padded grid by nearest-edge extension (reading)."""
    v = np.asarray(v, dtype=np.float64).reshape(g.phys_shape)
    return np.pad(v, g.nb, mode="edge")


def damping(g: Grid, eta_max: float) -> np.ndarray:
    """kappa = eta dt / 2 on the padded grid, eta = eta_max sum_d (delta_d / nb)^2.

    delta_d is the distance, in cells, of a padded index into the pad along
    axis d (zero in the physical grid).
    """
    prof = np.zeros(g.pad_shape)
    if g.nb == 0:
        return prof
    for axis, n in enumerate(g.phys_shape):
        i = np.arange(n + 2 * g.nb)
        delta = np.maximum(np.maximum(g.nb - i, i - (n + g.nb - 1)), 0).astype(np.float64)
        shape = [1] * g.ndim
        shape[axis] = -1
        prof = prof + (delta / g.nb).reshape(shape) ** 2
    return eta_max * prof * g.dt / 2.0


def annihilator_sq(g: Grid, src, eps: float = 1.0) -> np.ndarray:
    """W = B^2 on the physical grid, B(x) = ||x - x_s|| + eps in grid cells.

    Sec. 4 picks B = ||x - x_s|| plus a small positive number so that B does not
    vanish at the source; reading: distances in cells, eps = 1 cell.
    """
    if g.ndim == 2:
        iz, ix = np.meshgrid(np.arange(g.nz), np.arange(g.nx), indexing="ij")
        r = np.sqrt((ix - src[0]) ** 2 + (iz - src[1]) ** 2)
    else:
        iz, iy, ix = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx), indexing="ij")
        r = np.sqrt((ix - src[0]) ** 2 + (iz - src[1]) ** 2 + (iy - src[2]) ** 2)
    return (r + eps) ** 2


@dataclass
class Model:
    """Coefficients of one velocity model: c = v^2 dt^2 and kappa, padded."""
    g: Grid
    v_phys: np.ndarray
    c: np.ndarray
    kap: np.ndarray
    eta_max: float


def make_model(g: Grid, v: np.ndarray, eta_max: float | None = None) -> Model:
    """Padded c = v^2 dt^2 (eq. (wave) with m = 1/v^2) and the damping kappa.

    ``eta_max`` None takes the default from the physical v_max; 0 switches the
    absorbing layer off.
    """
    vp = pad_model(g, v)
    if eta_max is None:
        eta_max = eta_max_default(float(np.max(v)), g.nb, g.dx)
    c = np.ascontiguousarray(vp * vp * g.dt * g.dt, dtype=np.float64)
    kap = np.ascontiguousarray(damping(g, eta_max), dtype=np.float64)
    return Model(g, np.asarray(v, np.float64).reshape(g.phys_shape), c, kap, eta_max)


def window_model(m: Model, x0: int, x1: int) -> Model:
    """The model a 2D shot with aperture [x0, x1) propagates on (reading of the
    uneven-aperture workload: each shot is modelled on its window alone).

    Its physical columns are x0 .. x1-1; its absorbing layer of nb cells on
    every side holds the padded model beyond the window (the true model where
    the grid continues, edge copies beyond the grid), i.e. columns x0 ..
    x1 + 2 nb - 1 of the whole padded model; the damping profile surrounds
    the window, with the whole model's eta_max.  Positions in the window are
    the grid's minus x0.
    """
    g = m.g
    if g.ndim != 2:
        raise ValueError("apertures are 2D")
    gw = Grid(2, g.nz, x1 - x0, nb=g.nb, nt=g.nt, dx=g.dx, dt=g.dt)
    c = np.ascontiguousarray(m.c[:, x0:x1 + 2 * g.nb])
    kap = np.ascontiguousarray(damping(gw, m.eta_max))
    return Model(gw, np.ascontiguousarray(m.v_phys[:, x0:x1]), c, kap, m.eta_max)


# ---------------------------------------------------------------------------
# Modelling S = R A^{-1} and adjoint S^T (Sec. 2.1, eq. (wave), eq. (FWI_lambda);
# Sec. 3 first bullet: the right-hand side by adjoint modelling)
# ---------------------------------------------------------------------------

def _rec_idx(g: Grid, rec) -> np.ndarray:
    """Receiver positions -> padded linear indices.  ``rec`` is either physical
    positions [nrec, ndim] or, as a 1-D integer array, padded indices already
    (used by the energy pins to record the pad too)."""
    rec = np.asarray(rec)
    if rec.ndim == 1:
        return np.ascontiguousarray(rec, dtype=np.int64)
    return np.ascontiguousarray([g.pad_index(p) for p in rec.reshape(-1, g.ndim)],
                                dtype=np.int64)


def forward(m: Model, src, rec, *, src_pos=None, want_dtt: bool = False):
    """Forward modelling d = S q for one shot.

    ``src`` is either a wavelet [nt] injected at ``src_pos`` (the physical
    source f of eq. (fwi)) or a dense extended source [nt, *phys] (eq. (newq2)).
    Reading of the time axis: q^n enters step n and d^n = u^{n+1}(x_r), i.e. the
    sample at time (n+1) dt; zero initial state.  Returns d [nt, nrec] and, if
    asked, dtt [nt, *phys] = v^2 (L u^n + q^n) (= (dA/dm) u, Sec. 2.3 eq. (gradewi)).
    """
    g = m.g
    lib = _load()
    ridx = _rec_idx(g, rec)
    nrec = len(ridx)
    data = np.zeros((g.nt, nrec))
    src = np.ascontiguousarray(src, dtype=np.float64)
    if src.ndim == 1:
        kind, sidx = 0, g.pad_index(src_pos)
        assert src.shape[0] == g.nt
    else:
        kind, sidx = 1, -1
        assert src.shape == (g.nt, *g.phys_shape)
    dtt = np.zeros((g.nt, *g.phys_shape)) if want_dtt else None
    gc = g._c()
    rc = lib.or_forward(ctypes.byref(gc), _dptr(m.c), _dptr(m.kap), kind, _dptr(src), sidx,
                        nrec, ridx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dptr(data),
                        _dptr(dtt) if dtt is not None else None)
    if rc != 0:
        raise MemoryError("oracle forward: allocation failed")
    return (data, dtt) if want_dtt else data


def adjoint(m: Model, rec, data) -> np.ndarray:
    """Adjoint modelling S^T d for one shot: R^T injection, backward time loop,
    dense output on the physical grid [nt, *phys] (eq. (FWI_lambda), Sec. 3)."""
    g = m.g
    lib = _load()
    ridx = _rec_idx(g, rec)
    data = np.ascontiguousarray(data, dtype=np.float64)
    assert data.shape == (g.nt, len(ridx))
    out = np.zeros((g.nt, *g.phys_shape))
    gc = g._c()
    rc = lib.or_adjoint(ctypes.byref(gc), _dptr(m.c), _dptr(m.kap), len(ridx),
                        ridx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dptr(data), _dptr(out))
    if rc != 0:
        raise MemoryError("oracle adjoint: allocation failed")
    return out


# ---------------------------------------------------------------------------
# Normal operator and CG (Sec. 3, eq. (normalewi), eq. (axb), Algorithm 1)
# ---------------------------------------------------------------------------

def normal_apply(m: Model, rec, w2: np.ndarray, beta: float, p: np.ndarray) -> np.ndarray:
    """N p = S^T S p + beta B^T B p (Sec. 3, second bullet): forward modelling
    with p as the source, receiver extraction, adjoint modelling, plus the
    pointwise beta B^2 p term."""
    d = forward(m, p, rec)
    return adjoint(m, rec, d) + beta * w2[None] * p


def dot(a: np.ndarray, b: np.ndarray) -> float:
    """Plain inner product over cells and time steps (reading: unweighted sum;
    constant cell-volume weights would only rescale beta)."""
    return float(np.dot(np.ravel(a), np.ravel(b)))


@dataclass
class CGResult:
    x: np.ndarray
    iters: int
    res_hist: list          # ||r_k|| / ||r_0|| of the recursively updated residual
    alphas: list
    betas: list
    residuals: list | None = None   # r_0, r_1, ... when asked for
    iterates: list | None = None    # x_1, x_2, ... when asked for


def cg(apply_N, b: np.ndarray, max_iter: int, rtol: float = 0.0,
       keep_residuals: bool = False, keep_iterates: bool = False) -> CGResult:
    """Algorithm 1 (conjugate gradient for N x = b, N symmetric), step by step.

    x_0 = 0, r_0 = b, p_0 = r_0; for k = 0..K-1: alpha = r.r / p.Np,
    x += alpha p, r -= alpha Np; leave when ||r_{k+1}|| < tol ||r_0|| or
    k = K-1; beta = r'.r' / r.r; p = r' + beta p.  Returns x after the exit.
    """
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = dot(r, r)
    r0 = np.sqrt(rr)
    hist, alphas, betas = [1.0], [], []
    res = [r.copy()] if keep_residuals else None
    its = [] if keep_iterates else None
    k = 0
    for k in range(max_iter):
        Ap = apply_N(p)
        alpha = rr / dot(p, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = dot(r, r)
        alphas.append(alpha)
        if keep_residuals:
            res.append(r.copy())
        if keep_iterates:
            its.append(x.copy())
        hist.append(np.sqrt(rr_new) / r0 if r0 > 0 else 0.0)
        if np.sqrt(rr_new) < rtol * r0 or k == max_iter - 1:
            break
        beta = rr_new / rr
        betas.append(beta)
        p = r + beta * p
        rr = rr_new
    return CGResult(x, k + 1, hist, alphas, betas, res, its)


@dataclass
class FPCGResult:
    x: np.ndarray
    iters: int
    res_hist: list          # ||r_k|| / ||r_0||
    fallback_at: int | None  # iteration after which the first preconditioner was given up, or None
    cg_at: int | None        # iteration after which plain CG took over, or None


def fpcg(apply_N, b: np.ndarray, precond, max_iter: int, rtol: float = 0.0,
         stall: float = 0.99, window: int = 20, precond_fallback=None) -> FPCGResult:
    """Flexible CG with truncation 1 (Notay 2000, FCG(1)) for N x = b.

    x_0 = 0, r_0 = b, z_0 = M(r_0), p_0 = z_0; per iteration alpha = p.r / p.Np,
    x += alpha p, r -= alpha Np; leave when ||r|| < rtol ||r_0|| or at
    max_iter; z = M(r), beta = -z.Np / p.Np, p = z + beta p.  M may change from
    one call to the next.

    The preconditioner is given up when z.r <= 0, when z or z.r is not finite,
    or when the residual norm has not set a new best by the factor `stall` for
    `window` iterations (a preconditioned iteration minimises the error in the
    N-norm, so ||r|| may pause for a while and still converge).  It is then
    replaced by `precond_fallback` if given and by plain CG (M = I) after
    that; each switch restarts the direction at p = z, keeps the recursively
    updated residual and opens a fresh stall window.  With M = I the iteration
    is CG with the Hestenes-Stiefel form of beta, equal to Algorithm 1 in exact
    arithmetic.
    """
    stages = [precond] + ([precond_fallback] if precond_fallback is not None else []) + [None]
    stage = 0
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.sqrt(dot(b, b))
    hist = [1.0]
    marks = []                      # iterations of the switches

    def apply_m(res):
        m = stages[stage]
        return res.copy() if m is None else m(res)

    def usable(z, res):
        zr = dot(z, res)
        return bool(np.all(np.isfinite(z)) and np.isfinite(zr) and zr > 0)

    z = apply_m(r)
    while stages[stage] is not None and not usable(z, r):
        stage += 1
        marks.append(0)
        z = apply_m(r)
    p = z.copy()
    best, kbest = 1.0, 0
    k = 0
    for k in range(max_iter):
        Ap = apply_N(p)
        pAp = dot(p, Ap)
        alpha = dot(p, r) / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        hist.append(np.sqrt(dot(r, r)) / nb if nb > 0 else 0.0)
        if hist[-1] < rtol or k == max_iter - 1:
            break
        if hist[-1] < stall * best:
            best, kbest = hist[-1], k + 1
        z = apply_m(r)
        if stages[stage] is not None and (k + 1 - kbest >= window or not usable(z, r)):
            while True:                # give up this preconditioner: restart the direction
                stage += 1
                marks.append(k + 1)
                z = apply_m(r)
                if stages[stage] is None or usable(z, r):
                    break
            kbest, best = k + 1, hist[-1]
            p = z.copy()
            continue
        p = z - (dot(z, Ap) / pAp) * p
    fb = marks[0] if marks else None
    cg = marks[-1] if marks and stages[stage] is None else None
    return FPCGResult(x, k + 1, hist, fb, cg)


def esi_cg(m: Model, src_pos, rec, d_obs, beta: float, max_iter: int, rtol: float = 0.0,
           eps: float = 1.0, keep_iterates: bool = False) -> CGResult:
    """Solve (S^T S + beta B^T B) q = S^T d (eq. (normalewi)) for one shot by CG."""
    w2 = annihilator_sq(m.g, src_pos, eps)
    b = adjoint(m, rec, d_obs)
    return cg(lambda p: normal_apply(m, rec, w2, beta, p), b, max_iter, rtol, keep_iterates=keep_iterates)


# ---------------------------------------------------------------------------
# Gradients (eq. (gradient), eq. (gradewi), Algorithm 2 steps 4-6)
# ---------------------------------------------------------------------------

def gradient_penalty(m: Model, q: np.ndarray, w2: np.ndarray, beta: float) -> np.ndarray:
    """grad_m J = sum_n lambda^n (dA/dm) u^n with u = A^{-1} q and the adjoint
    field taken as lambda = beta B^T B q (Algorithm 2; the frequency sum printed
    there is read as the time sum of eq. (gradewi)).  m = 1/v^2."""
    g = m.g
    _, dtt = forward(m, q, np.zeros((0, g.ndim), dtype=np.int64), want_dtt=True)
    lam = beta * w2[None] * q
    return np.sum(lam * dtt, axis=0)


def gradient_adjoint(m: Model, q: np.ndarray, rec, d_obs) -> np.ndarray:
    """grad_m J = sum_n lambda^n (dA/dm) u^n with lambda = A^{-T} R^T (d - R u)
    (eq. (ewiadj), eq. (gradewi)) and u = A^{-1} q.  m = 1/v^2."""
    d_syn, dtt = forward(m, q, rec, want_dtt=True)
    lam = adjoint(m, rec, d_obs - d_syn)
    return np.sum(lam * dtt, axis=0)


def gradient_seed(m: Model, src, rec, seed, *, src_pos=None):
    """Gradients of a loss L(d), d = S(m) q, given G = dL/dd (eq. (gradient)).

    Returns (grad_m, grad_src): grad_m = -sum_n (S^T G)^n (dA/dm) u^n with
    m = 1/v^2, and grad_src = S^T G (dense source) or its trace at the source
    cell (point source).
    """
    g = m.g
    _, dtt = forward(m, src, rec, src_pos=src_pos, want_dtt=True)
    mu = adjoint(m, rec, seed)
    grad_m = -np.sum(mu * dtt, axis=0)
    if np.ndim(src) == 1:
        src_pos = np.asarray(src_pos)
        if g.ndim == 2:
            grad_src = mu[:, src_pos[1], src_pos[0]].copy()
        else:
            grad_src = mu[:, src_pos[1], src_pos[2], src_pos[0]].copy()
    else:
        grad_src = mu
    return grad_m, grad_src


def misfit_esi(m: Model, q: np.ndarray, rec, d_obs, w2: np.ndarray, beta: float) -> float:
    """J_ESI = 1/2 ||R u - d||^2 + beta/2 ||B q||^2 with u = A^{-1} q (eq. (esi))."""
    d = forward(m, q, rec)
    return 0.5 * dot(d - d_obs, d - d_obs) + 0.5 * beta * dot(w2[None] * q, q)


# ---------------------------------------------------------------------------
# WRI (Sec. 2.2: eq. (wridSf), eq. (normalwri), Table (compare), WRI row).
# The extension q is added to the physical source f (u = A^{-1}(f + q)) and
# penalised without a weight (B = I).
# ---------------------------------------------------------------------------

def with_point_source(g: Grid, q: np.ndarray, wavelet, src_pos) -> np.ndarray:
    """The dense source f + q: the wavelet added at the source cell of q (the
    point source of the forward modelling is that same dense source)."""
    out = np.array(q, dtype=np.float64, copy=True)
    sp = np.asarray(src_pos)
    if g.ndim == 2:
        out[:, sp[1], sp[0]] += wavelet
    else:
        out[:, sp[1], sp[2], sp[0]] += wavelet
    return out


def wri_rhs(m: Model, wavelet, src_pos, rec, d_obs) -> np.ndarray:
    """Right-hand side S^T (d - S f) of eq. (normalwri)."""
    d_f = forward(m, np.asarray(wavelet, np.float64), rec, src_pos=src_pos)
    return adjoint(m, rec, d_obs - d_f)


def wri_cg(m: Model, wavelet, src_pos, rec, d_obs, beta: float, max_iter: int,
           rtol: float = 0.0) -> CGResult:
    """Solve (S^T S + beta I) q = S^T (d - S f) (eq. (normalwri)) for one shot by
    CG (Algorithm 1)."""
    ones = np.ones(m.g.phys_shape)
    b = wri_rhs(m, wavelet, src_pos, rec, d_obs)
    return cg(lambda p: normal_apply(m, rec, ones, beta, p), b, max_iter, rtol)


def misfit_wri(m: Model, wavelet, src_pos, q: np.ndarray, rec, d_obs, beta: float) -> float:
    """J_WRI = 1/2 ||S (f + q) - d||^2 + beta/2 ||q||^2 (eq. (wridSf))."""
    d = forward(m, with_point_source(m.g, q, wavelet, src_pos), rec)
    return 0.5 * dot(d - d_obs, d - d_obs) + 0.5 * beta * dot(q, q)


def gradient_wri_penalty(m: Model, wavelet, src_pos, q: np.ndarray, beta: float) -> np.ndarray:
    """grad_m = sum_n lambda^n (dA/dm) u^n with lambda = beta q (the WRI adjoint
    field of Table (compare) at the solution of eq. (normalwri)) and
    u = A^{-1}(f + q).  m = 1/v^2."""
    g = m.g
    _, dtt = forward(m, with_point_source(g, q, wavelet, src_pos),
                     np.zeros((0, g.ndim), dtype=np.int64), want_dtt=True)
    return np.sum(beta * q * dtt, axis=0)


def gradient_wri_adjoint(m: Model, wavelet, src_pos, q: np.ndarray, rec, d_obs) -> np.ndarray:
    """grad_m = sum_n lambda^n (dA/dm) u^n with lambda = S^T (d - R u) and
    u = A^{-1}(f + q): the gradient of J_WRI in m at fixed q.  m = 1/v^2."""
    d_syn, dtt = forward(m, with_point_source(m.g, q, wavelet, src_pos), rec, want_dtt=True)
    lam = adjoint(m, rec, d_obs - d_syn)
    return np.sum(lam * dtt, axis=0)
