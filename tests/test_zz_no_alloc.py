"""The forward modelling call that allocates no device memory
(esi_forward_noalloc), called through the C ABI, against esi_forward on the
same plan and inputs: the two run the same kernels on the same states, so the
recorded data must agree bit for bit.  Two calls in a row, the second on a
smaller input, as a caller reusing the library's fixed scratch would make them.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2211_06300_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def esi():
    from paper_2211_06300_amd import esi as _esi
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    _esi.load_library()
    return _esi


def _cfg(nz, nx, nt, nshots, seed):
    """A heterogeneous grid with `nshots` shots, corner and duplicate receivers."""
    rng = np.random.default_rng(seed)
    cfg = inputs.cfg_tiny(nz=nz, nx=nx, nt=nt, nb=8, nrec=5, seed=seed)
    src = np.stack([rng.integers(0, nx, nshots), rng.integers(0, nz, nshots)], axis=1).astype(np.int32)
    recs = []
    for s in range(nshots):
        r = np.stack([rng.integers(0, nx, 6 + s), rng.integers(0, nz, 6 + s)], axis=1)
        recs.append(np.concatenate([r, np.array([[0, 0], [nx - 1, nz - 1]]), r[:1]]))
    cfg.src = src
    cfg.rec_ptr = np.concatenate([[0], np.cumsum([len(r) for r in recs])]).astype(np.int64)
    cfg.rec = np.concatenate(recs).astype(np.int32)
    cfg.v_true = (1800.0 + 800.0 * rng.random((nz, nx))).astype(np.float32)
    cfg.v_start = cfg.v_true
    return cfg


def _call(esi, plan, shot0, ns, kind, src, out):
    lib = esi.load_library()
    return lib.esi_forward_noalloc(plan._h, shot0, ns, kind, ctypes.c_void_p(src.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()))


def test_noalloc_forward_equals_forward_twice(esi):
    big = _cfg(37, 70, 70, 3, 31)
    plan = esi.Plan.from_config(big, vel=torch.from_numpy(big.v_true).to(DEV))
    q = torch.from_numpy(inputs.random_field(plan.vec_shape(3), 5)).to(DEV)
    ref = plan.forward(q, esi.SRC_DENSE)
    out = torch.full_like(ref, float("nan"))
    assert _call(esi, plan, 0, 3, esi.SRC_DENSE, q, out) == 0, esi.load_library().esi_last_error()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)

    # second call, smaller input: one shot of the same plan, point source
    w = torch.from_numpy(np.tile(big.wavelet, (1, 1))).to(DEV)
    ref1 = plan.forward(w, esi.SRC_POINT, shot0=2, nshots=1)
    out1 = torch.full_like(ref1, float("nan"))
    assert _call(esi, plan, 2, 1, esi.SRC_POINT, w, out1) == 0, esi.load_library().esi_last_error()
    torch.cuda.synchronize()
    assert torch.equal(out1, ref1)
    plan.close()

    # and a smaller plan after it: the scratch holds the larger call's state,
    # which must not leak into this one
    small = _cfg(11, 13, 30, 1, 32)
    plan2 = esi.Plan.from_config(small, vel=torch.from_numpy(small.v_true).to(DEV))
    w2 = torch.from_numpy(small.wavelet[None].copy()).to(DEV)
    ref2 = plan2.forward(w2, esi.SRC_POINT)
    out2 = torch.full_like(ref2, float("nan"))
    assert _call(esi, plan2, 0, 1, esi.SRC_POINT, w2, out2) == 0, esi.load_library().esi_last_error()
    torch.cuda.synchronize()
    assert torch.equal(out2, ref2)
    assert torch.isfinite(out2).all() and float(out2.abs().max()) > 0
    plan2.close()


def test_noalloc_forward_one_step_launches(esi):
    """With one step per launch (the other tiling built at plan creation)."""
    cfg = _cfg(37, 70, 41, 2, 33)
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(DEV))
    plan.set_time_block(1)
    w = torch.from_numpy(np.tile(cfg.wavelet, (2, 1))).to(DEV)
    ref = plan.forward(w, esi.SRC_POINT)
    out = torch.full_like(ref, float("nan"))
    assert _call(esi, plan, 0, 2, esi.SRC_POINT, w, out) == 0, esi.load_library().esi_last_error()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    plan.close()


def test_noalloc_forward_rejects_oversize(esi):
    """9 shots of an 801 x 401 grid need a 69 MB ring: beyond the 64 MiB scratch."""
    cfg = _cfg(401, 801, 4, 9, 34)
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(DEV))
    w = torch.from_numpy(np.tile(cfg.wavelet, (9, 1))).to(DEV)
    out = plan.new_data()
    assert _call(esi, plan, 0, 9, esi.SRC_POINT, w, out) == 2
    assert b"no-allocation scratch" in esi.load_library().esi_last_error()
    # within the limit the same plan works
    ref = plan.forward(w[:8], esi.SRC_POINT, nshots=8)
    out8 = torch.full_like(ref, float("nan"))
    assert _call(esi, plan, 0, 8, esi.SRC_POINT, w[:8], out8) == 0, esi.load_library().esi_last_error()
    torch.cuda.synchronize()
    assert torch.equal(out8, ref)
    plan.close()
