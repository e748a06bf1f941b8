"""The oracle pins catch plausible mistakes: each case plants one mistake in a
copy of ``oracle/prop.c`` (on the CPU), builds it, and checks that at least
one pin of ``test_oracle_pins`` fails with it."""
import os
import subprocess

import numpy as np
import pytest

from oracle import core
import tests.test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(core.__file__), "prop.c")

MUTANTS = {
    "damping sign": ("(1.0 - kap[i]) * um[i]", "(1.0 + kap[i]) * um[i]"),
    "record u^n not u^{n+1}": ("data[(long)n * nrec + r] = up[rec_idx[r]];",
                               "data[(long)n * nrec + r] = u0[rec_idx[r]];"),
    "adjoint output one step late": ("out[(long)j * NP + p] = m0[i];",
                                     "out[(long)j * NP + p] = m1[i];"),
    "dropped Laplacian term": ("for (long k = 1; k <= 4; ++k)", "for (long k = 1; k <= 3; ++k)"),
    "source scale": ("double lq = lap(g, u0, z, y, x) + q;",
                     "double lq = lap(g, u0, z, y, x) + 0.5 * q;"),
    "missing 1/dt^2 in dA/dm u": ("dtt[(long)n * NP + p] = c[i] * g->inv_dt2 * lq;",
                                  "dtt[(long)n * NP + p] = c[i] * lq;"),
    "adjoint injects at wrong step": ("inj[rec_idx[r]] += data[(long)j * nrec + r];",
                                      "inj[rec_idx[r]] += data[(long)(j > 0 ? j - 1 : 0) * nrec + r];"),
    "x stencil arm shifted": ("at(g, u, z - k * ez, y - k * ey, x - k * ex)",
                              "at(g, u, z - k * ez, y - k * ey, x - k * ex - ex)"),
}

PINS = [
    pins.test_dot_test_dense_source,
    pins.test_green2d_and_time_order,
    lambda: pins.test_energy(0.0),
    pins.test_gradient_seed_vs_fd,
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    before, after = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(before) == 1, "mutation anchor not found: " + before
    mpath = tmp_path / "prop_mut.c"
    mpath.write_text(text.replace(before, after))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o",
                           str(so), str(mpath), "-lm"])
    saved = core._lib
    core._lib = core._load(str(so))
    failed = []
    try:
        with np.errstate(all="ignore"):
            for pin in PINS:
                try:
                    pin()
                except AssertionError:
                    failed.append(pin)
    finally:
        core._lib = saved
    assert failed, "no pin caught the planted mistake: " + name
