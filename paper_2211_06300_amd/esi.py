"""Python binding of the ESI C ABI (``include/esi.h``, ``libesi.so``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libesi.so``.  Device memory and streams come from PyTorch.  If the
library is missing this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesi.so")

SRC_POINT, SRC_DENSE = 0, 1
GRAD_PENALTY, GRAD_ADJOINT, GRAD_SEED, GRAD_SEED_REUSE = 0, 1, 2, 3
WEIGHT_ANNIHILATOR, WEIGHT_IDENTITY = 0, 1
BETA_FIXED, BETA_DISCREPANCY = 0, 1
LAUNCH_ONE_STEP, LAUNCH_TWO_STEP_32, LAUNCH_TWO_STEP_24, LAUNCH_TWO_STEP_40 = 1, 2, 3, 4
LAUNCH_NAMES = {1: "1 step, 64x32 tiles", 2: "2 steps, 56x32 tiles", 3: "2 steps, 56x24 tiles",
                4: "2 steps, 56x40 tiles"}
LAUNCH_TILES = {1: "64x32", 2: "56x32", 3: "56x24", 4: "56x40"}
LAUNCH_NAMES_3D = {1: "1 step, 64x16 columns, 32-plane chunks", 2: "2 steps, 56x24 columns, 64-plane chunks"}
INNER_CG, INNER_FCG_SCALE, INNER_DATASPACE = 0, 1, 2
_STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_SHAPE", 3: "ERR_CFL", 4: "ERR_OOM", 5: "ERR_HIP",
           6: "ERR_BREAKDOWN", 7: "ERR_NONFINITE"}


class EsiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nz", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nb", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("eta_max", ctypes.c_double),
                ("beta", ctypes.c_double), ("b_eps", ctypes.c_double)]


class _Geom(ctypes.Structure):
    _fields_ = [("nshots", ctypes.c_int32), ("src", ctypes.POINTER(ctypes.c_int32)),
                ("rec_ptr", ctypes.POINTER(ctypes.c_int64)), ("rec", ctypes.POINTER(ctypes.c_int32)),
                ("window", ctypes.POINTER(ctypes.c_int32))]


class _CgReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("shot_iters", ctypes.POINTER(ctypes.c_int32)),
                ("res_hist", ctypes.POINTER(ctypes.c_double)),
                ("shot_fallback", ctypes.POINTER(ctypes.c_int32)),
                ("shot_cg", ctypes.POINTER(ctypes.c_int32)),
                ("stat_xref", ctypes.c_void_p), ("stat_out", ctypes.c_void_p)]


class _CgState(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("rr0", ctypes.c_void_p), ("rr", ctypes.c_void_p), ("beta", ctypes.c_void_p),
                ("iterating", ctypes.c_void_p), ("iters", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("res_hist", ctypes.c_void_p), ("hist_cap", ctypes.c_int32)]


class CgState:
    """Host arrays of a saved CG solve (esi_cg_state_t)."""

    def __init__(self, nshots: int, hist_cap: int):
        self.k = 0
        self.rr0 = np.zeros(nshots)
        self.rr = np.zeros(nshots)
        self.beta = np.zeros(nshots)
        self.iterating = np.zeros(nshots, dtype=np.int32)
        self.iters = np.zeros(nshots, dtype=np.int32)
        self.status = np.zeros(nshots, dtype=np.int32)
        self.res_hist = np.full((nshots, hist_cap), -1.0)

    def _struct(self):
        return _CgState(self.k, self.rr0.ctypes.data, self.rr.ctypes.data, self.beta.ctypes.data,
                        self.iterating.ctypes.data, self.iters.ctypes.data, self.status.ctypes.data,
                        self.res_hist.ctypes.data, self.res_hist.shape[1])


class _InvertOpts(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("cg_iters", ctypes.c_int32), ("cg_rtol", ctypes.c_double),
                ("shot_group", ctypes.c_int32), ("lbfgs_mem", ctypes.c_int32), ("ls_max", ctypes.c_int32),
                ("armijo_c1", ctypes.c_double), ("first_step", ctypes.c_double), ("v_min", ctypes.c_double),
                ("v_max", ctypes.c_double), ("beta_rule", ctypes.c_int32), ("misfit_lo", ctypes.c_double),
                ("misfit_hi", ctypes.c_double), ("beta_factor", ctypes.c_double), ("beta_tries", ctypes.c_int32),
                ("inner", ctypes.c_int32), ("inner_gamma", ctypes.c_double)]


class _InvertReport(ctypes.Structure):
    _fields_ = [("outer_done", ctypes.c_int32), ("evals", ctypes.c_int32), ("status", ctypes.c_int32),
                ("beta_final", ctypes.c_double), ("J", ctypes.c_void_p), ("misfit", ctypes.c_void_p),
                ("beta", ctypes.c_void_p), ("beta_iter", ctypes.c_void_p), ("step", ctypes.c_void_p),
                ("trials", ctypes.c_void_p)]


_lib = None
EXPORTS = ["esi_plan_create", "esi_plan_set_model", "esi_plan_destroy", "esi_last_error",
           "esi_forward", "esi_adjoint", "esi_normal_apply", "esi_cg_solve", "esi_gradient",
           "esi_plan_profile", "esi_plan_profile_read", "esi_plan_set_time_block",
           "esi_forward_ckpt", "esi_grad_velocity", "esi_plan_set_cg_graph", "esi_plan_set_cg_rfuse",
           "esi_unet_num_params", "esi_unet_create", "esi_unet_destroy", "esi_unet_set_params",
           "esi_unet_get_params", "esi_unet_forward", "esi_unet_loss_grad", "esi_unet_adam",
           "esi_fpcg_solve", "esi_precond_features", "esi_unet_loss_weights", "esi_plan_autotune",
           "esi_plan_set_weight", "esi_data_residual", "esi_wri_gradient", "esi_plan_set_beta",
           "esi_invert", "esi_dtft_set_freqs", "esi_dtft_normal_apply", "esi_dtft_rhs", "esi_dtft_cg_solve",
           "esi_dtft_to_time", "esi_dtft_gradient", "esi_ds_cg_solve", "esi_plan_set_dtft_block",
           "esi_plan_set_ds_ckpt", "esi_forward_noalloc", "esi_precond_scale", "esi_plan_tune_table",
           "esi_plan_set_launch_shape", "esi_cg_solve_state"]
# time-step kernel variants (bit set of fused work), as in include/esi.h
K_FLAGS = {1: "SRC_POINT", 2: "SRC_DENSE", 4: "CG_FUSE", 8: "INJ", 16: "GATHER", 32: "OUT",
           64: "NORMAL", 128: "PENALTY", 256: "STORE", 512: "CORR", 1024: "SRC_REC",
           2048: "SCALE", 4096: "DTFT_SRC", 8192: "DTFT_ACC", 16384: "RUPD", 32768: "TWO_STEP"}


def load_library(path: str = LIB_PATH):
    """Load ``libesi.so`` and declare the signatures of ``include/esi.h``."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.esi_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Grid), ctypes.POINTER(_Geom),
                                  vp, vp]
    L.esi_plan_set_model.argtypes = [vp, vp]
    L.esi_plan_destroy.argtypes = [vp]
    L.esi_last_error.argtypes = []
    L.esi_last_error.restype = ctypes.c_char_p
    L.esi_forward.argtypes = [vp, i32, i32, i32, vp, vp]
    L.esi_adjoint.argtypes = [vp, i32, i32, vp, vp]
    L.esi_normal_apply.argtypes = [vp, i32, i32, vp, vp, vp]
    L.esi_cg_solve.argtypes = [vp, i32, i32, vp, vp, vp, i32, dbl, ctypes.POINTER(_CgReport)]
    L.esi_cg_solve_state.argtypes = [vp, i32, i32, vp, vp, vp, i32, dbl, ctypes.POINTER(_CgState),
                                     ctypes.POINTER(_CgState), ctypes.POINTER(_CgReport)]
    L.esi_gradient.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp, vp, i32]
    L.esi_plan_set_weight.argtypes = [vp, i32]
    L.esi_plan_set_beta.argtypes = [vp, dbl]
    L.esi_dtft_set_freqs.argtypes = [vp, i32, vp]
    L.esi_dtft_normal_apply.argtypes = [vp, i32, i32, vp, vp, vp]
    L.esi_dtft_rhs.argtypes = [vp, i32, i32, vp, vp]
    L.esi_dtft_cg_solve.argtypes = [vp, i32, i32, vp, vp, vp, i32, dbl, ctypes.POINTER(_CgReport)]
    L.esi_dtft_to_time.argtypes = [vp, i32, i32, vp, vp]
    L.esi_dtft_gradient.argtypes = [vp, i32, i32, vp, vp]
    L.esi_ds_cg_solve.argtypes = [vp, i32, i32, vp, vp, vp, vp, i32, dbl, ctypes.POINTER(_CgReport)]
    L.esi_invert.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(_InvertOpts),
                             ctypes.POINTER(_InvertReport)]
    L.esi_data_residual.argtypes = [vp, i32, i32, vp, vp, vp]
    L.esi_wri_gradient.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, i32]
    L.esi_plan_profile.argtypes = [vp, i32]
    L.esi_plan_set_time_block.argtypes = [vp, i32]
    L.esi_plan_set_cg_graph.argtypes = [vp, i32]
    L.esi_plan_set_cg_rfuse.argtypes = [vp, i32]
    L.esi_plan_set_dtft_block.argtypes = [vp, i32]
    L.esi_plan_set_ds_ckpt.argtypes = [vp, i32]
    L.esi_plan_autotune.argtypes = [vp, i32, i32, vp, vp, i32, vp]
    L.esi_forward_ckpt.argtypes = [vp, i32, i32, i32, vp, vp, i32]
    L.esi_forward_noalloc.argtypes = [vp, i32, i32, i32, vp, vp]
    L.esi_precond_scale.argtypes = [vp, i32, i32, dbl, vp]
    L.esi_plan_tune_table.argtypes = [vp, i32, vp, vp, vp, vp]
    L.esi_plan_set_launch_shape.argtypes = [vp, i32, i32]
    L.esi_grad_velocity.argtypes = [vp, vp, vp, vp]
    L.esi_plan_profile_read.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.esi_fpcg_solve.argtypes = [vp, i32, i32, vp, vp, vp, i32, dbl, vp, i32, vp, ctypes.POINTER(_CgReport)]
    L.esi_precond_features.argtypes = [vp, i32, i32, vp, vp, vp, i32, i32, vp, vp, vp]
    L.esi_unet_num_params.argtypes = []
    L.esi_unet_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, vp]
    L.esi_unet_destroy.argtypes = [vp]
    L.esi_unet_set_params.argtypes = [vp, vp]
    L.esi_unet_get_params.argtypes = [vp, vp]
    L.esi_unet_forward.argtypes = [vp, vp, vp, i32]
    L.esi_unet_loss_grad.argtypes = [vp, vp, vp, vp, vp, i32, vp, ctypes.POINTER(dbl)]
    L.esi_unet_loss_weights.argtypes = [vp, vp, i32, i64, vp, vp]
    L.esi_unet_adam.argtypes = [vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, i32,
                                ctypes.c_float]
    for f in EXPORTS:
        if f != "esi_last_error":
            getattr(L, f).restype = ctypes.c_int
    L.esi_unet_num_params.restype = i64
    if path == LIB_PATH:
        _lib = L
    return L


def _check(code: int):
    if code != 0:
        raise EsiError(code, load_library().esi_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("tensors must be contiguous and on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _f32(t, shape, name):
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return _ptr(t)


class Plan:
    """One grid, acquisition and velocity model (``esi_plan_create``).

    ``src`` is int [nshots, ndim] and ``rec`` int [nrec_total, ndim] of physical
    cells (ix, iz[, iy]); ``rec_ptr`` int [nshots+1] splits ``rec`` by shot.
    ``vel`` is a CUDA float32 tensor of the physical grid shape.
    """

    def __init__(self, *, ndim, nz, nx, ny=1, nb, nt, dx, dt, beta, b_eps=1.0, eta_max=-1.0,
                 src, rec_ptr, rec, vel: torch.Tensor, stream=None, window=None):
        self._lib = load_library()
        self.ndim, self.nz, self.nx, self.ny, self.nb, self.nt = ndim, nz, nx, ny, nb, nt
        self.dx, self.dt, self.beta = dx, dt, beta
        self.phys_shape = (nz, nx) if ndim == 2 else (nz, ny, nx)
        self.nphys = int(np.prod(self.phys_shape))
        self.src = np.ascontiguousarray(src, dtype=np.int32).reshape(-1, ndim)
        self.rec_ptr = np.ascontiguousarray(rec_ptr, dtype=np.int64)
        self.rec = np.ascontiguousarray(rec, dtype=np.int32).reshape(-1, ndim)
        self.nshots = self.src.shape[0]
        g = _Grid(ndim, nz, nx, ny, nb, nt, dx, dt, eta_max, beta, b_eps)
        self.window = None if window is None else np.ascontiguousarray(window, dtype=np.int32).reshape(-1, 2)
        geo = _Geom(self.nshots, self.src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    self.rec_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                    self.rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    None if self.window is None else self.window.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self.device = vel.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(vel.device)
        h = ctypes.c_void_p()
        _check(self._lib.esi_plan_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(geo),
                                         _f32(vel, self.phys_shape, "vel"),
                                         ctypes.c_void_p(self.stream.cuda_stream)))
        self._h = h

    @classmethod
    def from_config(cls, cfg, vel: torch.Tensor | None = None, device="cuda", **kw):
        if vel is None:
            vel = torch.from_numpy(np.ascontiguousarray(cfg.v_start)).to(device)
        kw.setdefault("window", getattr(cfg, "window", None))
        return cls(ndim=cfg.ndim, nz=cfg.nz, nx=cfg.nx, ny=cfg.ny, nb=cfg.nb, nt=cfg.nt,
                   dx=cfg.dx, dt=cfg.dt, beta=cfg.beta, b_eps=cfg.b_eps, src=cfg.src,
                   rec_ptr=cfg.rec_ptr, rec=cfg.rec, vel=vel, **kw)

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.esi_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- shapes ---------------------------------------------------------------
    def _range(self, shot0, nshots):
        if nshots is None:
            nshots = self.nshots - shot0
        return int(shot0), int(nshots)

    def data_shape(self, shot0=0, nshots=None):
        shot0, nshots = self._range(shot0, nshots)
        return (self.nt * int(self.rec_ptr[shot0 + nshots] - self.rec_ptr[shot0]),)

    def vec_shape(self, nshots):
        return (nshots, self.nt, *self.phys_shape)

    def new_data(self, shot0=0, nshots=None):
        return torch.zeros(self.data_shape(shot0, nshots), dtype=torch.float32, device=self.device)

    def new_vec(self, nshots):
        return torch.zeros(self.vec_shape(nshots), dtype=torch.float32, device=self.device)

    # -- calls ------------------------------------------------------------------
    def set_time_block(self, steps: int):
        _check(self._lib.esi_plan_set_time_block(self._h, int(steps)))

    def autotune(self, shot0=0, nshots=None, force=False, p=None, Ap=None, probe=False):
        """esi_plan_autotune; returns the (forward, adjoint) launch shapes.
        probe=True times a propagation-only pass (no wavefield-sized vectors)."""
        shot0, nshots = self._range(shot0, nshots)
        if probe:
            pp = ap = None
        else:
            p = self.new_vec(nshots) if p is None else p
            Ap = self.new_vec(nshots) if Ap is None else Ap
            pp = _f32(p, self.vec_shape(nshots), "p")
            ap = _f32(Ap, self.vec_shape(nshots), "Ap")
        ch = np.zeros(2, dtype=np.int32)
        _check(self._lib.esi_plan_autotune(self._h, shot0, nshots, pp, ap, int(bool(force)),
                                           ch.ctypes.data_as(ctypes.c_void_p)))
        return int(ch[0]), int(ch[1])

    def tune_table(self):
        """esi_plan_tune_table: [(shape, forward ms, adjoint ms)] of the last autotune."""
        cap = 8
        cnt = np.zeros(1, dtype=np.int32)
        sh = np.zeros(cap, dtype=np.int32)
        f = np.zeros(cap)
        a = np.zeros(cap)
        _check(self._lib.esi_plan_tune_table(self._h, cap, cnt.ctypes.data, sh.ctypes.data, f.ctypes.data,
                                             a.ctypes.data))
        return [(int(sh[i]), float(f[i]), float(a[i])) for i in range(min(int(cnt[0]), cap))]

    def set_launch_shape(self, forward: int, adjoint: int):
        """esi_plan_set_launch_shape (LAUNCH_* shapes)."""
        _check(self._lib.esi_plan_set_launch_shape(self._h, int(forward), int(adjoint)))

    def set_weight(self, kind: int):
        """esi_plan_set_weight: WEIGHT_ANNIHILATOR (ESI) or WEIGHT_IDENTITY (WRI, B = I)."""
        _check(self._lib.esi_plan_set_weight(self._h, int(kind)))

    def data_residual(self, wavelet, d_obs, shot0=0, nshots=None, out=None):
        """d_obs - S f for point wavelets f [nshots][nt] (the WRI right-hand side data)."""
        shot0, nshots = self._range(shot0, nshots)
        dshape = self.data_shape(shot0, nshots)
        out = self.new_data(shot0, nshots) if out is None else out
        _check(self._lib.esi_data_residual(self._h, shot0, nshots, _f32(wavelet, (nshots, self.nt), "wavelet"),
                                           _f32(d_obs, dshape, "d_obs"), _f32(out, dshape, "d_res")))
        return out

    def wri_gradient(self, mode, wavelet, q, d_obs=None, shot0=0, nshots=None, grad_m=None, ckpt_every=0):
        """esi_wri_gradient: gradient in m with u = A^{-1}(f + q), added to grad_m."""
        shot0, nshots = self._range(shot0, nshots)
        grad_m = torch.zeros(self.phys_shape, dtype=torch.float32, device=self.device) \
            if grad_m is None else grad_m
        dptr = None if d_obs is None else _f32(d_obs, self.data_shape(shot0, nshots), "d_obs")
        _check(self._lib.esi_wri_gradient(self._h, shot0, nshots, int(mode),
                                          _f32(wavelet, (nshots, self.nt), "wavelet"),
                                          _f32(q, self.vec_shape(nshots), "q"), dptr,
                                          _f32(grad_m, self.phys_shape, "grad_m"), int(ckpt_every)))
        return grad_m

    # -- DTFT variant (frequency vectors [nshots][nf][*phys][2] float32) ------------
    def dtft_set_freqs(self, freqs):
        f = np.ascontiguousarray(freqs, dtype=np.float64)
        _check(self._lib.esi_dtft_set_freqs(self._h, int(f.size), f.ctypes.data))
        self.dtft_freqs = f

    def dtft_shape(self, nshots):
        return (nshots, len(self.dtft_freqs), *self.phys_shape, 2)

    def dtft_normal_apply(self, p, shot0=0, nshots=None, out=None):
        shot0, nshots = self._range(shot0, nshots)
        sh = self.dtft_shape(nshots)
        out = torch.empty(sh, dtype=torch.float32, device=self.device) if out is None else out
        pMp = torch.zeros(nshots, dtype=torch.float64, device=self.device)
        _check(self._lib.esi_dtft_normal_apply(self._h, shot0, nshots, _f32(p, sh, "p"), _f32(out, sh, "Mp"),
                                               _ptr(pMp)))
        return out, pMp

    def dtft_rhs(self, d_obs, shot0=0, nshots=None):
        shot0, nshots = self._range(shot0, nshots)
        sh = self.dtft_shape(nshots)
        b = torch.empty(sh, dtype=torch.float32, device=self.device)
        _check(self._lib.esi_dtft_rhs(self._h, shot0, nshots, _f32(d_obs, self.data_shape(shot0, nshots), "d_obs"),
                                      _f32(b, sh, "b")))
        return b

    def dtft_cg_solve(self, d_obs, max_iter, rtol=0.0, shot0=0, nshots=None, x=None, work=None):
        shot0, nshots = self._range(shot0, nshots)
        sh = self.dtft_shape(nshots)
        x = torch.empty(sh, dtype=torch.float32, device=self.device) if x is None else x
        work = torch.empty((3, *sh), dtype=torch.float32, device=self.device) if work is None else work
        hist = np.zeros((nshots, max_iter + 1))
        iters = np.zeros(nshots, dtype=np.int32)
        rep = _CgReport(0, iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, None, None, None)
        _check(self._lib.esi_dtft_cg_solve(self._h, shot0, nshots,
                                           _f32(d_obs, self.data_shape(shot0, nshots), "d_obs"),
                                           _f32(x, sh, "x"), _f32(work, (3, *sh), "work"), int(max_iter),
                                           float(rtol), ctypes.byref(rep)))
        return x, {"iters": rep.iters, "shot_iters": iters, "res_hist": hist}

    def dtft_to_time(self, x, shot0=0, nshots=None):
        shot0, nshots = self._range(shot0, nshots)
        q = self.new_vec(nshots)
        _check(self._lib.esi_dtft_to_time(self._h, shot0, nshots, _f32(x, self.dtft_shape(nshots), "x"),
                                          _f32(q, self.vec_shape(nshots), "q")))
        return q

    def dtft_gradient(self, x, shot0=0, nshots=None, grad_m=None):
        shot0, nshots = self._range(shot0, nshots)
        grad_m = torch.zeros(self.phys_shape, dtype=torch.float32, device=self.device) \
            if grad_m is None else grad_m
        _check(self._lib.esi_dtft_gradient(self._h, shot0, nshots, _f32(x, self.dtft_shape(nshots), "x"),
                                           _f32(grad_m, self.phys_shape, "grad_m")))
        return grad_m

    def ds_cg_solve(self, d, max_iter, rtol=0.0, shot0=0, nshots=None, want_q=True, w=None, q=None, work=None):
        """esi_ds_cg_solve: data-space CG; returns (w, q or None, report)."""
        shot0, nshots = self._range(shot0, nshots)
        dsh = self.data_shape(shot0, nshots)
        w = self.new_data(shot0, nshots) if w is None else w
        if want_q and q is None:
            q = self.new_vec(nshots)
        work = torch.empty((3 * int(np.prod(dsh)),), dtype=torch.float32, device=self.device) if work is None else work
        hist = np.zeros((nshots, max_iter + 1))
        iters = np.zeros(nshots, dtype=np.int32)
        rep = _CgReport(0, iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, None, None, None)
        _check(self._lib.esi_ds_cg_solve(self._h, shot0, nshots, _f32(d, dsh, "d"), _f32(w, dsh, "w"),
                                         None if q is None else _f32(q, self.vec_shape(nshots), "q"),
                                         _f32(work, (3 * int(np.prod(dsh)),), "work"), int(max_iter), float(rtol),
                                         ctypes.byref(rep)))
        return w, q, {"iters": rep.iters, "shot_iters": iters, "res_hist": hist}

    def set_beta(self, beta: float):
        _check(self._lib.esi_plan_set_beta(self._h, float(beta)))

    def invert(self, d_obs, vel, *, wavelet=None, mask=None, shot0=0, nshots=None, shot_group=None,
               x=None, work=None, outer_iters=3, cg_iters=10, cg_rtol=0.0, lbfgs_mem=5, ls_max=6,
               armijo_c1=1e-4, first_step=0.02, v_min=1000.0, v_max=6000.0, beta_rule=BETA_FIXED,
               misfit_lo=0.05, misfit_hi=0.2, beta_factor=2.0, beta_tries=4, inner=INNER_CG, inner_gamma=0.03):
        """esi_invert: the outer loop of Algorithm 2.  vel (device [phys]) holds
        the starting model and receives the last accepted one; returns the
        report as a dict of counts and histories."""
        shot0, nshots = self._range(shot0, nshots)
        G = nshots if shot_group is None else int(shot_group)
        x = self.new_vec(G) if x is None else x
        if work is None:
            work = torch.empty((3, *self.vec_shape(G)), dtype=torch.float32, device=self.device)
        o = _InvertOpts(int(outer_iters), int(cg_iters), float(cg_rtol), G, int(lbfgs_mem), int(ls_max),
                        float(armijo_c1), float(first_step), float(v_min), float(v_max), int(beta_rule),
                        float(misfit_lo), float(misfit_hi), float(beta_factor), int(beta_tries), int(inner),
                        float(inner_gamma))
        k = int(outer_iters)
        h = {"J": np.zeros(k + 1), "misfit": np.zeros(k + 1), "beta": np.zeros(k + 1),
             "beta_iter": np.zeros(k), "step": np.zeros(k), "trials": np.zeros(k, dtype=np.int32)}
        r = _InvertReport(0, 0, 0, 0.0, *[a.ctypes.data if a.size else None for a in h.values()])
        _check(self._lib.esi_invert(self._h, shot0, nshots, _f32(d_obs, self.data_shape(shot0, nshots), "d_obs"),
                                    None if wavelet is None else _f32(wavelet, (nshots, self.nt), "wavelet"),
                                    _f32(vel, self.phys_shape, "vel"),
                                    None if mask is None else _f32(mask, self.phys_shape, "mask"),
                                    _f32(x, self.vec_shape(G), "x"), _f32(work, (3, *self.vec_shape(G)), "work"),
                                    ctypes.byref(o), ctypes.byref(r)))
        n = r.outer_done
        return {"outer_done": n, "evals": r.evals, "status": r.status, "beta_final": r.beta_final,
                "J": h["J"][:n + 1].tolist(), "misfit": h["misfit"][:n + 1].tolist(),
                "beta": h["beta"][:n + 1].tolist(),
                "beta_iter": h["beta_iter"][:n + (1 if r.status else 0)].tolist(),
                "step": h["step"][:n].tolist(),
                "trials": h["trials"][:n + (1 if r.status else 0)].tolist()}

    def set_cg_graph(self, enable: bool):
        _check(self._lib.esi_plan_set_cg_graph(self._h, int(bool(enable))))

    def set_ds_ckpt(self, every: int):
        """Data-space solver: adjoint field resident (0) or checkpointed every `every` steps."""
        _check(self._lib.esi_plan_set_ds_ckpt(self._h, int(every)))

    def set_dtft_block(self, block: int):
        """DTFT time loops meet the frequency slices per `block` steps (0: at every step)."""
        _check(self._lib.esi_plan_set_dtft_block(self._h, int(block)))

    def set_cg_rfuse(self, enable: bool):
        """CG with the residual update fused into the adjoint pass (default on)."""
        _check(self._lib.esi_plan_set_cg_rfuse(self._h, int(bool(enable))))

    def set_model(self, vel: torch.Tensor):
        _check(self._lib.esi_plan_set_model(self._h, _f32(vel, self.phys_shape, "vel")))

    def forward(self, src, kind=SRC_POINT, shot0=0, nshots=None, out=None):
        shot0, nshots = self._range(shot0, nshots)
        shape = (nshots, self.nt) if kind == SRC_POINT else self.vec_shape(nshots)
        out = self.new_data(shot0, nshots) if out is None else out
        _check(self._lib.esi_forward(self._h, shot0, nshots, kind, _f32(src, shape, "src"),
                                     _f32(out, self.data_shape(shot0, nshots), "data")))
        return out

    def precond_scale(self, gamma, shot0=0, nshots=None, out=None):
        """esi_precond_scale: the analytic cell scale 1 / (beta B^2 + gamma) per
        shot, float32 [nshots, *phys] on the device."""
        shot0, nshots = self._range(shot0, nshots)
        out = torch.empty((nshots, *self.phys_shape), dtype=torch.float32, device=self.device) \
            if out is None else out
        _check(self._lib.esi_precond_scale(self._h, shot0, nshots, float(gamma),
                                           _f32(out, (nshots, *self.phys_shape), "out")))
        return out

    def forward_noalloc(self, src, kind=SRC_POINT, shot0=0, nshots=None, out=None):
        """esi_forward_noalloc: forward modelling whose wavefield ring lives in
        the library's fixed device array (no device allocation by the call)."""
        shot0, nshots = self._range(shot0, nshots)
        shape = (nshots, self.nt) if kind == SRC_POINT else self.vec_shape(nshots)
        out = self.new_data(shot0, nshots) if out is None else out
        _check(self._lib.esi_forward_noalloc(self._h, shot0, nshots, kind, _f32(src, shape, "src"),
                                             _f32(out, self.data_shape(shot0, nshots), "data")))
        return out

    def forward_ckpt(self, src, ckpt_every, kind=SRC_POINT, shot0=0, nshots=None, out=None):
        """Forward modelling that keeps wavefield checkpoints every `ckpt_every`
        steps for a following gradient(GRAD_SEED_REUSE, ...)."""
        shot0, nshots = self._range(shot0, nshots)
        shape = (nshots, self.nt) if kind == SRC_POINT else self.vec_shape(nshots)
        out = self.new_data(shot0, nshots) if out is None else out
        _check(self._lib.esi_forward_ckpt(self._h, shot0, nshots, kind, _f32(src, shape, "src"),
                                          _f32(out, self.data_shape(shot0, nshots), "data"),
                                          int(ckpt_every)))
        return out

    def grad_velocity(self, vel, grad_m, out=None):
        """grad_v = -2 grad_m / v^3 (device kernel)."""
        out = torch.empty_like(grad_m) if out is None else out
        _check(self._lib.esi_grad_velocity(self._h, _f32(vel, self.phys_shape, "vel"),
                                           _f32(grad_m, self.phys_shape, "grad_m"),
                                           _f32(out, self.phys_shape, "grad_v")))
        return out

    def adjoint(self, data, shot0=0, nshots=None, out=None):
        shot0, nshots = self._range(shot0, nshots)
        out = self.new_vec(nshots) if out is None else out
        _check(self._lib.esi_adjoint(self._h, shot0, nshots,
                                     _f32(data, self.data_shape(shot0, nshots), "data"),
                                     _f32(out, self.vec_shape(nshots), "out")))
        return out

    def normal_apply(self, p, shot0=0, nshots=None, out=None, want_pAp=True):
        shot0, nshots = self._range(shot0, nshots)
        out = self.new_vec(nshots) if out is None else out
        pAp = torch.zeros(nshots, dtype=torch.float64, device=self.device) if want_pAp else None
        _check(self._lib.esi_normal_apply(self._h, shot0, nshots, _f32(p, self.vec_shape(nshots), "p"),
                                          _f32(out, self.vec_shape(nshots), "Ap"), _ptr(pAp)))
        return out, pAp

    def cg_solve(self, d_obs, max_iter, rtol=0.0, shot0=0, nshots=None, x=None, work=None):
        shot0, nshots = self._range(shot0, nshots)
        x = self.new_vec(nshots) if x is None else x
        if work is None:
            work = torch.empty((3, *self.vec_shape(nshots)), dtype=torch.float32, device=self.device)
        hist = np.zeros((nshots, max_iter + 1))
        iters = np.zeros(nshots, dtype=np.int32)
        rep = _CgReport(0, iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        _check(self._lib.esi_cg_solve(self._h, shot0, nshots,
                                      _f32(d_obs, self.data_shape(shot0, nshots), "d_obs"),
                                      _f32(x, self.vec_shape(nshots), "x"),
                                      _f32(work, (3, *self.vec_shape(nshots)), "work"),
                                      int(max_iter), float(rtol), ctypes.byref(rep)))
        return x, {"iters": int(rep.iters), "shot_iters": iters, "res_hist": hist}

    def cg_solve_state(self, d_obs, max_iter, rtol=0.0, shot0=0, nshots=None, x=None, work=None,
                       resume: "CgState | None" = None, save: bool = False):
        """esi_cg_solve_state: CG from x_0 = 0 or from `resume`; with save=True
        returns the state after the last iteration as a CgState."""
        shot0, nshots = self._range(shot0, nshots)
        x = self.new_vec(nshots) if x is None else x
        if work is None:
            work = torch.empty((3, *self.vec_shape(nshots)), dtype=torch.float32, device=self.device)
        hist = np.zeros((nshots, max_iter + 1))
        iters = np.zeros(nshots, dtype=np.int32)
        rep = _CgReport(0, iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        st = CgState(nshots, max_iter + 1) if save else None
        rs = resume._struct() if resume is not None else None
        ss = st._struct() if st is not None else None
        dptr = None if d_obs is None else _f32(d_obs, self.data_shape(shot0, nshots), "d_obs")
        code = self._lib.esi_cg_solve_state(self._h, shot0, nshots, dptr, _f32(x, self.vec_shape(nshots), "x"),
                                            _f32(work, (3, *self.vec_shape(nshots)), "work"), int(max_iter),
                                            float(rtol), None if rs is None else ctypes.byref(rs),
                                            None if ss is None else ctypes.byref(ss), ctypes.byref(rep))
        if st is not None:
            st.k = int(ss.k)
        _check(code)
        return x, {"iters": int(rep.iters), "shot_iters": iters, "res_hist": hist}, st

    def fpcg_solve(self, d_obs, max_iter, rtol=0.0, net=None, scale=None, shot0=0, nshots=None,
                   x=None, work=None, stat_xref=None, stat_out=None, net_every=0):
        """Flexible CG (esi_fpcg_solve); net is a Unet, scale a [nshots, *phys]
        tensor, or neither (M = I); the network runs on r_0 and every
        net_every-th iteration (0: once)."""
        shot0, nshots = self._range(shot0, nshots)
        x = self.new_vec(nshots) if x is None else x
        if work is None:
            work = torch.empty((3, *self.vec_shape(nshots)), dtype=torch.float32, device=self.device)
        hist = np.zeros((nshots, max_iter + 1))
        iters = np.zeros(nshots, dtype=np.int32)
        fb = np.zeros(nshots, dtype=np.int32)
        cg = np.zeros(nshots, dtype=np.int32)
        rep = _CgReport(0, iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        fb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        cg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        None if stat_xref is None else _f32(stat_xref, self.vec_shape(nshots), "stat_xref"),
                        None if stat_out is None else _f32(stat_out, (max_iter + 1, nshots, 2, self.nphys),
                                                           "stat_out"))
        sp = None if scale is None else _f32(scale, (nshots, *self.phys_shape), "scale")
        _check(self._lib.esi_fpcg_solve(self._h, shot0, nshots,
                                        _f32(d_obs, self.data_shape(shot0, nshots), "d_obs"),
                                        _f32(x, self.vec_shape(nshots), "x"),
                                        _f32(work, (3, *self.vec_shape(nshots)), "work"),
                                        int(max_iter), float(rtol), None if net is None else net._h,
                                        int(net_every), sp, ctypes.byref(rep)))
        return x, {"iters": int(rep.iters), "shot_iters": iters, "res_hist": hist, "fallback": fb, "cg_at": cg}

    def precond_features(self, a, Hp, Wp, cmap=None, base=None, shot0=0, nshots=None, pads=False):
        """Network input [nshots, 3, Hp, Wp] from a = sum_t r^2 [nshots, *phys];
        with pads=True also the zero-padded a base^2 and cmap base."""
        shot0, nshots = self._range(shot0, nshots)
        xin = torch.empty((nshots, 3, Hp, Wp), dtype=torch.float32, device=self.device)
        ap = torch.empty((nshots, Hp, Wp), dtype=torch.float32, device=self.device) if pads else None
        cp = torch.empty((nshots, Hp, Wp), dtype=torch.float32, device=self.device) if pads and cmap is not None else None
        _check(self._lib.esi_precond_features(self._h, shot0, nshots,
                                              _f32(a, (nshots, *self.phys_shape), "a"),
                                              None if cmap is None else _f32(cmap, (nshots, *self.phys_shape), "cmap"),
                                              None if base is None else _f32(base, (nshots, *self.phys_shape), "base"),
                                              int(Hp), int(Wp), _ptr(xin), _ptr(ap), _ptr(cp)))
        return (xin, ap, cp) if pads else xin

    def gradient(self, mode, src, data=None, kind=SRC_DENSE, shot0=0, nshots=None, grad_m=None,
                 grad_src=None, ckpt_every=0):
        shot0, nshots = self._range(shot0, nshots)
        grad_m = torch.zeros(self.phys_shape, dtype=torch.float32, device=self.device) \
            if grad_m is None else grad_m
        sshape = (nshots, self.nt) if kind == SRC_POINT else self.vec_shape(nshots)
        dptr = None if data is None else _f32(data, self.data_shape(shot0, nshots), "data")
        gsp = None if grad_src is None else _f32(grad_src, sshape, "grad_src")
        _check(self._lib.esi_gradient(self._h, shot0, nshots, mode, kind, _f32(src, sshape, "src"),
                                      dptr, _f32(grad_m, self.phys_shape, "grad_m"), gsp,
                                      int(ckpt_every)))
        return grad_m

    # -- timing ------------------------------------------------------------------
    def profile(self, enable=True):
        _check(self._lib.esi_plan_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """Per time-step kernel variant: launches, shot-weighted launches and the
        elapsed milliseconds of the time loops that ran it (hipEvents)."""
        cap = 32
        cnt = np.zeros(1, dtype=np.int32)
        fl = np.zeros(cap, dtype=np.uint32)
        la = np.zeros(cap, dtype=np.int64)
        sl = np.zeros(cap, dtype=np.int64)
        ms = np.zeros(cap, dtype=np.float64)
        _check(self._lib.esi_plan_profile_read(self._h, cap, cnt.ctypes.data, fl.ctypes.data,
                                               la.ctypes.data, sl.ctypes.data, ms.ctypes.data))
        out = {}
        for i in range(min(int(cnt[0]), cap)):
            f = int(fl[i])
            name = "|".join(v for k, v in K_FLAGS.items() if f & k)
            shape = (f >> 16) & 7
            if shape and self.ndim == 2:
                name += "@" + LAUNCH_TILES[shape]
            out[name] = {"flags": f, "launches": int(la[i]), "shot_launches": int(sl[i]), "ms": float(ms[i])}
        return out


class Unet:
    """The preconditioner network (``esi_unet_create``): images of H x W pixels
    (multiples of 8), batches of up to ``max_batch``; parameters as a flat
    float32 CUDA tensor in the layout of include/esi.h."""

    def __init__(self, H: int, W: int, max_batch: int, device="cuda", stream=None):
        self._lib = load_library()
        self.H, self.W, self.max_batch = int(H), int(W), int(max_batch)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.P = int(self._lib.esi_unet_num_params())
        h = ctypes.c_void_p()
        _check(self._lib.esi_unet_create(ctypes.byref(h), self.H, self.W, self.max_batch,
                                         ctypes.c_void_p(self.stream.cuda_stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.esi_unet_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta: torch.Tensor):
        _check(self._lib.esi_unet_set_params(self._h, _f32(theta, (self.P,), "theta")))

    def get_params(self) -> torch.Tensor:
        t = torch.empty(self.P, dtype=torch.float32, device=self.device)
        _check(self._lib.esi_unet_get_params(self._h, _ptr(t)))
        return t

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        b = int(x.shape[0])
        o = torch.empty((b, self.H, self.W), dtype=torch.float32, device=self.device)
        _check(self._lib.esi_unet_forward(self._h, _f32(x, (b, 3, self.H, self.W), "x"), _ptr(o), b))
        return o

    def loss_grad(self, x, a, c, grad=None, weight=None):
        b = int(x.shape[0])
        grad = torch.empty(self.P, dtype=torch.float32, device=self.device) if grad is None else grad
        loss = ctypes.c_double()
        shp = (b, self.H, self.W)
        _check(self._lib.esi_unet_loss_grad(self._h, _f32(x, (b, 3, self.H, self.W), "x"),
                                            _f32(a, shp, "a"), _f32(c, shp, "c"),
                                            None if weight is None else _f32(weight, (b,), "weight"), b,
                                            _f32(grad, (self.P,), "grad"), ctypes.byref(loss)))
        return grad, loss.value

    def loss_weights(self, a, c):
        """Default loss weights of whole images a, c [n, ...] (any size)."""
        n = int(a.shape[0])
        npix = int(a[0].numel())
        w = torch.empty(n, dtype=torch.float32, device=self.device)
        _check(self._lib.esi_unet_loss_weights(_f32(a, tuple(a.shape), "a"), _f32(c, tuple(c.shape), "c"), n,
                                               npix, _ptr(w), ctypes.c_void_p(self.stream.cuda_stream)))
        return w

    def adam(self, grad, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, clip=0.0):
        _check(self._lib.esi_unet_adam(self._h, _f32(grad, (self.P,), "grad"), float(lr), float(beta1),
                                       float(beta2), float(eps), int(step), float(clip)))
