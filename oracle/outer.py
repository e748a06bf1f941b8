"""FP64 oracle of the outer loop of Algorithm 2 (nested loops for variable
projection between m and q), with the penalty schedule of Sec. 2.4.

TEST INFRASTRUCTURE ONLY.  Like ``core``, this is the plain definition the GPU
library is checked against; only ``tests/``, the smoke check and the bench
CPU baseline may use it.

Algorithm 2: for each outer iteration, solve the normal equation for q by CG
(the inner loop), form u = A^{-1} q and lambda = beta B^T B q, the gradient
sum_n lambda^n (dA/dm) u^n, a descent direction -H g with H the L-BFGS
approximation of the inverse Hessian, and a step length by line search.

Readings (the paper names L-BFGS and a line search, nothing more):
* the objective is the reduced J(m) = J_ESI(m, q(m)) with q(m) the CG iterate
  (the inner loop's output), evaluated as 1/2 ||S q - d||^2 + beta/2 ||B q||^2
  summed over shots (eq. (esi)); WRI uses eq. (wridSf);
* L-BFGS is the two-loop recursion (Nocedal & Wright, Numerical Optimization,
  Algorithm 7.4) with H0 = (s'y / y'y) I from the newest pair; a pair enters
  the memory only when s'y > 0;
* the line search is backtracking with the Armijo condition on the step
  actually taken after clipping m to the velocity bounds,
  J(m_t) <= J(m) + c1 g'(m_t - m), halving the step; the first trial is the
  full L-BFGS step, or, without curvature pairs, a steepest-descent step
  scaled so that max |dm| = first_step * max m;
* the penalty follows the discrepancy principle (Sec. 2.4, Sec. 4.3): before
  each outer iteration, while the relative data misfit ||S q - d|| / ||d|| is
  below `misfit_lo` beta is multiplied by `beta_factor` (the data are fitted
  too freely), while it is above `misfit_hi` beta is divided by it, at most
  `beta_tries` times; each change re-solves at the current model and clears
  the L-BFGS memory (J changes with beta).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import core, dataspace


@dataclass
class OuterOptions:
    outer_iters: int = 3
    cg_iters: int = 10           # inner CG iterations (Sec. 4 uses 10)
    cg_rtol: float = 0.0
    lbfgs_mem: int = 5
    ls_max: int = 6              # line-search trials per outer iteration
    armijo_c1: float = 1e-4
    first_step: float = 0.02     # steepest-descent step: max |dm| / max m
    v_min: float = 1000.0
    v_max: float = 6000.0
    beta_rule: str = "fixed"     # "fixed" or "discrepancy"
    misfit_lo: float = 0.05
    misfit_hi: float = 0.2
    beta_factor: float = 2.0
    beta_tries: int = 4


@dataclass
class OuterResult:
    m: np.ndarray
    J: list = field(default_factory=list)        # at the accepted models (J[0]: start)
    misfit: list = field(default_factory=list)   # relative data misfit at the accepted models
    beta: list = field(default_factory=list)     # penalty used for J[i]
    beta_iter: list = field(default_factory=list)  # penalty of each outer iteration (after the rule)
    step: list = field(default_factory=list)     # accepted step length per outer iteration
    trials: list = field(default_factory=list)   # line-search trials per outer iteration
    evals: int = 0                               # objective evaluations (inner solves)
    status: str = "ok"                           # or "line search failed"


def lbfgs_direction(g: np.ndarray, pairs) -> np.ndarray:
    """-H g by the two-loop recursion over the stored (s, y) pairs, oldest
    first; with no pairs, -g."""
    q = g.copy()
    alphas = []
    for s, y in reversed(pairs):
        rho = 1.0 / float(y @ s)
        a = rho * float(s @ q)
        q -= a * y
        alphas.append(a)
    if pairs:
        s, y = pairs[-1]
        q *= float(s @ y) / float(y @ y)
    for (s, y), a in zip(pairs, reversed(alphas)):
        rho = 1.0 / float(y @ s)
        b = rho * float(y @ q)
        q += (a - b) * s
    return -q


def minimize(evaluate, m0: np.ndarray, beta0: float, opts: OuterOptions) -> OuterResult:
    """The outer loop over a black-box objective: evaluate(m, beta) returns
    (J, gradient, relative data misfit) for the flattened model m.  m is
    clipped to [1/v_max^2, 1/v_min^2]."""
    lo, hi = 1.0 / opts.v_max ** 2, 1.0 / opts.v_min ** 2
    shape = np.shape(m0)
    m = np.clip(np.array(m0, dtype=np.float64).ravel(), lo, hi)
    beta = beta0
    res = OuterResult(m)
    J, g, e = evaluate(m, beta)
    res.evals += 1
    res.J.append(J)
    res.misfit.append(e)
    res.beta.append(beta)
    pairs = []
    for _ in range(opts.outer_iters):
        if opts.beta_rule == "discrepancy":
            tries = 0
            while tries < opts.beta_tries and (e < opts.misfit_lo or e > opts.misfit_hi):
                beta = beta * opts.beta_factor if e < opts.misfit_lo else beta / opts.beta_factor
                J, g, e = evaluate(m, beta)
                res.evals += 1
                pairs = []
                tries += 1
        res.beta_iter.append(beta)
        d = lbfgs_direction(g, pairs)
        if pairs and float(g @ d) >= 0.0:
            pairs = []
            d = -g
        alpha = 1.0 if pairs else opts.first_step * float(np.max(m)) / float(np.max(np.abs(g)))
        accepted = False
        for t in range(opts.ls_max):
            m_t = np.clip(m + alpha * d, lo, hi)
            J_t, g_t, e_t = evaluate(m_t, beta)
            res.evals += 1
            if J_t <= J + opts.armijo_c1 * float(g @ (m_t - m)):
                accepted = True
                break
            alpha *= 0.5
        res.trials.append(t + 1)
        if not accepted:
            res.status = "line search failed"
            break
        s, y = m_t - m, g_t - g
        if float(s @ y) > 0.0:
            pairs.append((s.ravel().copy(), y.ravel().copy()))
            pairs = pairs[-opts.lbfgs_mem:]
        m, J, g, e = m_t, J_t, g_t, e_t
        res.step.append(alpha)
        res.J.append(J)
        res.misfit.append(e)
        res.beta.append(beta)
    res.m = m.reshape(shape)
    return res


def esi_objective(g: core.Grid, shots, cg_iters: int, cg_rtol: float = 0.0, eta_max=None,
                  wavelet=None, mask=None, eps: float = 1.0, inner: str = "cg", gamma: float = 0.03):
    """evaluate(m, beta) of the reduced ESI (or, with `wavelet`, WRI) objective:
    per shot the CG iterate q of the normal equation, J = sum of eq. (esi) (or
    eq. (wridSf)), the PENALTY gradient of Algorithm 2 (lambda = beta W q with
    u = A^{-1} q, or A^{-1}(f + q) for WRI) times `mask`, and the relative data
    misfit ||S q - d|| / ||d|| over all shots.

    inner "cg" solves by Algorithm 1; "fcg" (ESI) by flexible CG (``core.fpcg``)
    preconditioned by the cell scale 1 / (beta B^2 + gamma), with its fallback to
    plain CG; "ds" by the data-space CG of ``dataspace.cg`` (Sec. 5.1).

    shots: list of (src_pos, rec, d_obs)."""
    dd = sum(core.dot(d, d) for _, _, d in shots)

    def evaluate(m, beta):
        mod = core.make_model(g, 1.0 / np.sqrt(m.reshape(g.phys_shape)), eta_max=eta_max)
        J, r2 = 0.0, 0.0
        grad = np.zeros(g.phys_shape)
        for s, (src, rec, d) in enumerate(shots):
            if wavelet is None:
                w2 = core.annihilator_sq(g, src, eps)
                if inner == "ds":
                    q = dataspace.cg(mod, src, rec, d, beta, cg_iters, cg_rtol, eps=eps)[1]
                elif inner == "fcg":
                    s0 = 1.0 / (beta * w2 + gamma)
                    q = core.fpcg(lambda p: core.normal_apply(mod, rec, w2, beta, p), core.adjoint(mod, rec, d),
                                  lambda r: s0[None] * r, cg_iters, cg_rtol).x
                else:
                    q = core.esi_cg(mod, src, rec, d, beta, cg_iters, cg_rtol, eps=eps).x
                d_syn = core.forward(mod, q, rec)
                J += 0.5 * core.dot(d_syn - d, d_syn - d) + 0.5 * beta * core.dot(w2[None] * q, q)
                grad += core.gradient_penalty(mod, q, w2, beta)
            else:
                f = wavelet[s]
                if inner == "ds":
                    d_f = core.forward(mod, f, rec, src_pos=src)
                    q = dataspace.cg(mod, src, rec, d - d_f, beta, cg_iters, cg_rtol, w2=np.ones(g.phys_shape))[1]
                else:
                    q = core.wri_cg(mod, f, src, rec, d, beta, cg_iters, cg_rtol).x
                d_syn = core.forward(mod, core.with_point_source(g, q, f, src), rec)
                J += 0.5 * core.dot(d_syn - d, d_syn - d) + 0.5 * beta * core.dot(q, q)
                grad += core.gradient_wri_penalty(mod, f, src, q, beta)
            r2 += core.dot(d_syn - d, d_syn - d)
        if mask is not None:
            grad = grad * mask
        return J, grad.ravel(), float(np.sqrt(r2 / dd))

    return evaluate
