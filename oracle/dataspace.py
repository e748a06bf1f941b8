"""FP64 oracle of the data-space solution of the ESI normal equation (Sec. 5.1:
eq. (wd), eq. (vd), eq. (wv), eq. (q)), the Sherman-Morrison-Woodbury route.

TEST INFRASTRUCTURE ONLY.  Like ``core``, this is the plain definition the GPU
library is checked against; only ``tests/``, the smoke check and the bench
CPU baseline may use it.

With W = B^T B invertible:
  v = S W^{-1} S^T d                      (eq. (vd): adjoint modelling of d,
                                           scaling by W^{-1}, forward modelling
                                           with the scaled field as source)
  (beta I + S W^{-1} S^T) w = v           (eq. (wv), solved by CG, Algorithm 1)
  q = (beta W)^{-1} S^T (d - w)           (eq. (q))
which equals the wavefield-space solution q = (S^T S + beta W)^{-1} S^T d.
For WRI (B = I) d is replaced by d - S f (eq. (wriw)).
"""
from __future__ import annotations

import numpy as np

from . import core


def K_apply(m: core.Model, rec, w2: np.ndarray, w: np.ndarray) -> np.ndarray:
    """S W^{-1} S^T w for a data vector w [nt, nrec]."""
    mu = core.adjoint(m, rec, w)
    return core.forward(m, mu / w2[None], rec)


def cg(m: core.Model, src_pos, rec, d: np.ndarray, beta: float, max_iter: int, rtol: float = 0.0,
       eps: float = 1.0, w2=None):
    """Returns (w, q, CGResult): CG on (beta I + S W^{-1} S^T) w = v with
    v = S W^{-1} S^T d, and q = (beta W)^{-1} S^T (d - w).  w2 defaults to the
    annihilator's B^2 of the shot (ones for WRI)."""
    if w2 is None:
        w2 = core.annihilator_sq(m.g, src_pos, eps)
    v = K_apply(m, rec, w2, d)
    res = core.cg(lambda p: beta * p + K_apply(m, rec, w2, p), v, max_iter, rtol)
    q = core.adjoint(m, rec, d - res.x) / (beta * w2[None])
    return res.x, q, res
