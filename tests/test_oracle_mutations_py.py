"""The pins of the Python parts of the oracle catch plausible mistakes: each case
plants one mistake in a copy of an oracle module (WRI functions of ``core``,
``dtft``, ``dataspace``, ``outer``), runs it in place of the module inside the
pin tests, and checks that at least one pin fails."""
import os
import types

import numpy as np
import pytest

import oracle
import tests.test_oracle_dataspace as pins_ds
import tests.test_oracle_dtft as pins_dtft
import tests.test_oracle_outer as pins_outer
import tests.test_oracle_wri as pins_wri
from tests.test_oracle_wri import wri_system  # noqa: F401  (fixture for the WRI pins)

ORACLE_DIR = os.path.dirname(oracle.__file__)


def _mutant(modname, before, after):
    path = os.path.join(ORACLE_DIR, modname + ".py")
    text = open(path).read()
    assert text.count(before) == 1, "mutation anchor not found: " + before
    mod = types.ModuleType("oracle." + modname)
    mod.__file__ = path
    mod.__package__ = "oracle"
    exec(compile(text.replace(before, after), path, "exec"), mod.__dict__)
    if modname == "core":
        # share the loaded time-loop library and its ctypes types with the
        # original module, whose grids and models the pins also build
        from oracle import core
        for name in ("_load", "_Grid", "Grid", "Model", "CGResult"):
            setattr(mod, name, getattr(core, name))
    return mod


def _caught(pin_calls):
    failed = []
    with np.errstate(all="ignore"):
        for name, call in pin_calls:
            try:
                call()
            except (AssertionError, np.linalg.LinAlgError, FloatingPointError, ValueError):
                failed.append(name)
    return failed


WRI_MUTANTS = {
    "right-hand side sign": ("return adjoint(m, rec, d_obs - d_f)", "return adjoint(m, rec, d_obs + d_f)"),
    "f dropped from u": ("""    _, dtt = forward(m, with_point_source(g, q, wavelet, src_pos),
                     np.zeros((0, g.ndim), dtype=np.int64), want_dtt=True)""",
                         """    _, dtt = forward(m, q, np.zeros((0, g.ndim), dtype=np.int64), want_dtt=True)"""),
    "penalty without beta": ("return 0.5 * dot(d - d_obs, d - d_obs) + 0.5 * beta * dot(q, q)",
                             "return 0.5 * dot(d - d_obs, d - d_obs) + 0.5 * dot(q, q)"),
    "source cell transposed": ("out[:, sp[1], sp[0]] += wavelet", "out[:, sp[0], sp[1]] += wavelet"),
}


@pytest.mark.parametrize("name", sorted(WRI_MUTANTS))
def test_wri_pins_catch_mutant(name, monkeypatch, wri_system):  # noqa: F811
    monkeypatch.setattr(pins_wri, "core", _mutant("core", *WRI_MUTANTS[name]))
    failed = _caught([
        ("point source", pins_wri.test_point_source_is_dense_delta),
        ("rhs dense", lambda: pins_wri.test_wri_rhs_dense(wri_system)),
        ("identities", lambda: pins_wri.test_wri_solution_identities(wri_system)),
        ("penalty = adjoint", lambda: pins_wri.test_wri_penalty_equals_adjoint_at_optimum(wri_system)),
        ("fd", pins_wri.test_wri_gradient_adjoint_vs_fd),
    ])
    assert failed, "no pin caught the planted mistake: " + name


DTFT_MUTANTS = {
    "inverse exponent sign": ("    E = np.conj(twiddles(freqs, nt, dt))\n", "    E = twiddles(freqs, nt, dt)\n"),
    "missing 1/nt": ("return np.real(np.tensordot(E, s, axes=(1, 0))) / nt",
                     "return np.real(np.tensordot(E, s, axes=(1, 0)))"),
    "forward exponent sign": ("    E = twiddles(freqs, u.shape[0], dt)\n",
                              "    E = np.conj(twiddles(freqs, u.shape[0], dt))\n"),
    "data not band-limited": ("    d = idtft(dtft(d_obs, freqs, g.dt), freqs, g.dt, g.nt)\n", "    d = d_obs\n"),
    "imaginary part taken": ("return np.real(np.tensordot(E, s, axes=(1, 0))) / nt",
                             "return np.imag(np.tensordot(E, s, axes=(1, 0))) / nt"),
}


@pytest.mark.parametrize("name", sorted(DTFT_MUTANTS))
def test_dtft_pins_catch_mutant(name, monkeypatch):
    monkeypatch.setattr(pins_dtft, "dtft", _mutant("dtft", *DTFT_MUTANTS[name]))
    failed = _caught([(f.__name__, f) for f in (
        pins_dtft.test_dtft_equals_fft_on_grid, pins_dtft.test_adjoint_relation,
        pins_dtft.test_FG_half_identity_on_grid, pins_dtft.test_normal_operator_spd_and_dense,
        pins_dtft.test_band_limited_reconstruction, pins_dtft.test_rhs_dense)])
    assert failed, "no pin caught the planted mistake: " + name


DS_MUTANTS = {
    "W instead of W^-1": ("return core.forward(m, mu / w2[None], rec)", "return core.forward(m, mu * w2[None], rec)"),
    "q without beta": ("q = core.adjoint(m, rec, d - res.x) / (beta * w2[None])",
                       "q = core.adjoint(m, rec, d - res.x) / w2[None]"),
    "d - w sign": ("q = core.adjoint(m, rec, d - res.x) / (beta * w2[None])",
                   "q = core.adjoint(m, rec, d + res.x) / (beta * w2[None])"),
    "beta dropped from the system": ("res = core.cg(lambda p: beta * p + K_apply(m, rec, w2, p), v, max_iter, rtol)",
                                     "res = core.cg(lambda p: K_apply(m, rec, w2, p), v, max_iter, rtol)"),
}


@pytest.mark.parametrize("name", sorted(DS_MUTANTS))
def test_dataspace_pins_catch_mutant(name, monkeypatch):
    monkeypatch.setattr(pins_ds, "dataspace", _mutant("dataspace", *DS_MUTANTS[name]))
    failed = _caught([(f.__name__, f) for f in (
        pins_ds.test_K_dense_symmetric, pins_ds.test_q_equals_wavefield_solution, pins_ds.test_wri_data_space)])
    assert failed, "no pin caught the planted mistake: " + name


OUTER_MUTANTS = {
    "two-loop rho": ("        rho = 1.0 / float(y @ s)\n        a = rho * float(s @ q)",
                     "        rho = 1.0 / float(s @ s)\n        a = rho * float(s @ q)"),
    "H0 scale inverted": ("q *= float(s @ y) / float(y @ y)", "q *= float(y @ y) / float(s @ y)"),
    "second loop sign": ("q += (a - b) * s", "q += (b - a) * s"),
    "step doubled": ("            alpha *= 0.5\n", "            alpha *= 2.0\n"),
    "beta rule reversed": ("beta = beta * opts.beta_factor if e < opts.misfit_lo else beta / opts.beta_factor",
                           "beta = beta / opts.beta_factor if e < opts.misfit_lo else beta * opts.beta_factor"),
}


@pytest.mark.parametrize("name", sorted(OUTER_MUTANTS))
def test_outer_pins_catch_mutant(name, monkeypatch):
    monkeypatch.setattr(pins_outer, "outer", _mutant("outer", *OUTER_MUTANTS[name]))
    failed = _caught([(f.__name__, f) for f in (
        pins_outer.test_two_loop_equals_bfgs_matrix, pins_outer.test_minimize_quadratic,
        pins_outer.test_minimize_clips_to_bounds, pins_outer.test_discrepancy_rule_moves_beta)])
    assert failed, "no pin caught the planted mistake: " + name
