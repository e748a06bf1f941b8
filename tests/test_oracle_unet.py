"""Pins of the learned-preconditioner oracle (network and flexible CG)."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import core, unet
from tests.test_oracle_pins import tiny_system  # noqa: F401  (fixture)


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_bf16_rounding_matches_torch():
    """Round-to-nearest-even to bfloat16 equals torch's conversion, ties included."""
    torch = pytest.importorskip("torch")
    rng = _rng(1)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        # exact ties: low 16 bits 0x8000 with even and odd bit 16
                        np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x40490000],
                                 dtype=np.uint32).view(np.float32)])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(unet.bf16(x), ref)


def test_conv3x3_is_cross_correlation():
    """Same-size 3x3 convolution = sum over input channels of scipy's 2D
    cross-correlation with zero fill."""
    rng = _rng(2)
    x = rng.standard_normal((2, 3, 7, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = unet.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, c], w[o, c], mode="same", boundary="fill")
                             for c in range(3))
            np.testing.assert_allclose(y[n, o], ref, rtol=1e-12, atol=1e-12)


def test_convT_and_pool_brute_force():
    rng = _rng(3)
    x = rng.standard_normal((2, 3, 4, 5))
    w = rng.standard_normal((3, 2, 2, 2))
    b = rng.standard_normal(2)
    y = unet.convT2(x, w, b)
    ref = np.zeros((2, 2, 8, 10))
    for n in range(2):
        for o in range(2):
            for i in range(8):
                for j in range(10):
                    ref[n, o, i, j] = b[o] + sum(w[c, o, i % 2, j % 2] * x[n, c, i // 2, j // 2]
                                                 for c in range(3))
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)
    z = rng.standard_normal((1, 2, 6, 4))
    p = unet.avgpool2(z)
    for i in range(3):
        for j in range(2):
            np.testing.assert_allclose(p[0, :, i, j], z[0, :, 2 * i:2 * i + 2, 2 * j:2 * j + 2]
                                       .reshape(2, 4).mean(axis=1), rtol=1e-14)


def test_layer_backward_adjoint_identities():
    """<conv(x), g> = <x, conv^T(g)> (bias off) and the same for convT and pool."""
    rng = _rng(4)
    x = rng.standard_normal((2, 3, 6, 8))
    w = rng.standard_normal((5, 3, 3, 3))
    g = rng.standard_normal((2, 5, 6, 8))
    y = unet.conv3x3(x, w, np.zeros(5))
    gx, gw, gb = unet.conv3x3_backward(x, w, g)
    assert abs(np.sum(y * g) - np.sum(x * gx)) < 1e-11 * abs(np.sum(y * g))
    assert abs(np.sum(y * g) - np.sum(w * gw)) < 1e-11 * abs(np.sum(y * g))
    np.testing.assert_allclose(gb, g.sum(axis=(0, 2, 3)))
    wt = rng.standard_normal((3, 4, 2, 2))
    gt = rng.standard_normal((2, 4, 12, 16))
    yt = unet.convT2(x, wt, np.zeros(4))
    gxt, gwt, _ = unet.convT2_backward(x, wt, gt)
    assert abs(np.sum(yt * gt) - np.sum(x * gxt)) < 1e-11 * abs(np.sum(yt * gt))
    assert abs(np.sum(yt * gt) - np.sum(wt * gwt)) < 1e-11 * abs(np.sum(yt * gt))
    gp = rng.standard_normal((2, 3, 3, 4))
    assert abs(np.sum(unet.avgpool2(x) * gp) - np.sum(x * unet.avgpool2_backward(gp))) < 1e-12


def _init(seed=5):
    from paper_2211_06300_amd import inputs
    return inputs.he_init(unet.fan_segments(), seed).astype(np.float64)


def test_param_count():
    assert unet.num_params() == 482033
    assert _init().size == unet.num_params()


def test_unet_gradient_vs_fd():
    """Backward of the whole network and the scaling loss against central
    differences in FP64 (no bf16 rounding) along random parameter directions."""
    rng = _rng(6)
    theta = _init()
    x = rng.standard_normal((2, 3, 16, 8))
    a = rng.random((2, 1, 16, 8)) + 0.1
    c = rng.standard_normal((2, 1, 16, 8)) * 0.3

    def loss(t):
        o, _ = unet.forward(t, x, bf=False)
        return unet.scaling_loss(o, a, c)[0]

    o, cache = unet.forward(theta, x, bf=False)
    L, go = unet.scaling_loss(o, a, c)
    g = unet.backward(theta, cache, go)
    for k in range(4):
        d = rng.standard_normal(theta.size)
        h = 1e-6
        fd = (loss(theta + h * d) - loss(theta - h * d)) / (2 * h)
        an = float(g @ d)
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9, (k, fd, an)


def test_scaling_loss_minimum():
    """For one sample the loss is minimised cell by cell at exp(o) = c / a; the
    best single scale sum c / sum a scores -1 and a vanishing correction 0;
    by Cauchy-Schwarz the cell optimum is at most -1."""
    rng = _rng(7)
    a = rng.random((1, 1, 4, 4)) + 0.5
    c = rng.random((1, 1, 4, 4)) + 0.1
    o = np.log(c / a)
    _, go = unet.scaling_loss(o, a, c)
    assert np.max(np.abs(go)) < 1e-15
    Lopt, _ = unet.scaling_loss(o, a, c)
    assert abs(Lopt + np.sum(c * c / a) * np.sum(a) / np.sum(c) ** 2) < 1e-13
    L1, _ = unet.scaling_loss(np.full_like(o, np.log(c.sum() / a.sum())), a, c)
    assert abs(L1 + 1.0) < 1e-13 and Lopt <= L1
    L0, _ = unet.scaling_loss(np.full_like(o, -50.0), a, c)
    assert abs(L0) < 1e-20


def test_loss_weights_tiles():
    """Explicit weights: the default weights reproduce the default loss, and
    the loss of an image equals the summed losses of its disjoint tiles
    weighted by the whole image's weight; non-positive sum c gives weight 0."""
    rng = _rng(9)
    o = rng.standard_normal((2, 1, 8, 8)) * 0.3
    a = rng.random((2, 1, 8, 8)) + 0.1
    c = rng.random((2, 1, 8, 8))
    L, g = unet.scaling_loss(o, a, c)
    L2, g2 = unet.scaling_loss(o, a, c, unet.loss_weights(a, c))
    assert L == L2 and np.array_equal(g, g2)
    w = unet.loss_weights(a, c)
    parts = [unet.scaling_loss(o[:, :, i:i + 4, j:j + 4], a[:, :, i:i + 4, j:j + 4], c[:, :, i:i + 4, j:j + 4], w)[0]
             for i in (0, 4) for j in (0, 4)]
    assert abs(sum(parts) - L) < 1e-12 * abs(L)
    assert unet.loss_weights(a, -c)[0] == 0.0


def test_bf16_forward_close_to_fp64():
    """bf16 emulation perturbs the output by about the bf16 unit roundoff."""
    rng = _rng(8)
    theta = _init()
    x = rng.standard_normal((1, 3, 16, 16))
    o64, _ = unet.forward(theta, x, bf=False)
    o16, _ = unet.forward(theta, x, bf=True)
    err = np.linalg.norm(o16 - o64) / np.linalg.norm(o64)
    assert 1e-4 < err < 5e-2


def test_adam_clip():
    """Clipping rescales the gradient to the given norm before the moments."""
    g = np.array([3.0, 4.0])
    a = unet.adam_step(np.zeros(2), g, np.zeros(2), np.zeros(2), 1, lr=0.1, clip=1.0)
    b = unet.adam_step(np.zeros(2), g / 5.0, np.zeros(2), np.zeros(2), 1, lr=0.1)
    for u, w in zip(a, b):
        np.testing.assert_allclose(u, w, rtol=1e-15)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are exact, so each
    step moves theta by lr g / (|g| + eps)."""
    g = np.array([1e-3, -2.0, 0.5])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 6):
        th, m, v = unet.adam_step(th, g, m, v, t, lr=0.01)
    np.testing.assert_allclose(th, -5 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_precond_inputs_constant_residual():
    r = np.full((5, 4, 6), 3.0)
    v = np.full((4, 6), 3000.0)
    w2 = np.full((4, 6), 400.0)
    x, a = unet.precond_inputs(r, v, w2)
    np.testing.assert_allclose(x[0], np.log(2.0))
    np.testing.assert_allclose(x[1], 1.0)
    np.testing.assert_allclose(x[2], np.log(20.0) / 4.0)
    np.testing.assert_allclose(a, 45.0)


# -- flexible CG -------------------------------------------------------------

def test_fpcg_identity_is_cg(tiny_system):
    """FCG(1) with M = I follows Algorithm 1 (beta in Hestenes-Stiefel form)."""
    N, b = tiny_system["N"], tiny_system["b"]
    ref = core.cg(lambda p: N @ p, b, 8)
    res = core.fpcg(lambda p: N @ p, b, lambda r: r.copy(), 8)
    assert res.fallback_at is None
    np.testing.assert_allclose(res.res_hist, ref.res_hist, rtol=1e-7)
    assert np.linalg.norm(res.x - ref.x) < 1e-7 * np.linalg.norm(ref.x)


def test_fpcg_fixed_spd_is_pcg(tiny_system):
    """With a fixed SPD diagonal M, FCG(1) equals textbook preconditioned CG
    (alpha = r.z / p.Np, beta = r'.z' / r.z), which it reduces to in exact
    arithmetic."""
    N, b = tiny_system["N"], tiny_system["b"]
    D = 1.0 / np.diag(N)
    res = core.fpcg(lambda p: N @ p, b, lambda r: D * r, 10)
    x, r = np.zeros_like(b), b.copy()
    z = D * r
    p, rz = z.copy(), r @ z
    for _ in range(10):
        Ap = N @ p
        al = rz / (p @ Ap)
        x, r = x + al * p, r - al * Ap
        z = D * r
        rz, rz_old = r @ z, rz
        p = z + rz / rz_old * p
    assert np.linalg.norm(res.x - x) < 1e-8 * np.linalg.norm(x)


def test_fpcg_exact_inverse_one_iteration(tiny_system):
    N, b = tiny_system["N"], tiny_system["b"]
    Ninv = np.linalg.inv(N)
    res = core.fpcg(lambda p: N @ p, b, lambda r: Ninv @ r, 5, rtol=1e-8)
    assert res.iters == 1
    assert np.linalg.norm(b - N @ res.x) < 1e-8 * np.linalg.norm(b)


def test_fpcg_fallback(tiny_system):
    """An indefinite preconditioner (z.r < 0) hands over at once, and one that
    stalls is replaced after 20 iterations without a new best residual: by the
    fallback preconditioner when given (which equals running with it from
    that point), then by plain CG; the result still converges."""
    N, b = tiny_system["N"], tiny_system["b"]
    ref = core.cg(lambda p: N @ p, b, 6)
    neg = core.fpcg(lambda p: N @ p, b, lambda r: -r, 6)
    assert neg.fallback_at == 0 and neg.cg_at == 0
    np.testing.assert_allclose(neg.res_hist, ref.res_hist, rtol=1e-7)
    D = 1.0 / np.diag(N)
    neg2 = core.fpcg(lambda p: N @ p, b, lambda r: -r, 6, precond_fallback=lambda r: D * r)
    pcg = core.fpcg(lambda p: N @ p, b, lambda r: D * r, 6)
    assert neg2.fallback_at == 0 and neg2.cg_at is None
    np.testing.assert_allclose(neg2.res_hist, pcg.res_hist, rtol=1e-7)
    e0 = np.zeros_like(b)
    e0[0] = 1.0
    stuck = core.fpcg(lambda p: N @ p, b, lambda r: e0 * (r @ e0) + 1e-30 * r, 80)
    assert stuck.fallback_at is not None and stuck.fallback_at >= 20 and stuck.cg_at == stuck.fallback_at
    assert stuck.res_hist[-1] < core.cg(lambda p: N @ p, b, 40).res_hist[-1]
