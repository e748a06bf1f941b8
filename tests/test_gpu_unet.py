"""The preconditioner network on the GPU against the FP64 oracle with bf16
emulation (same bf16 weights, activations rounded at every layer boundary):
forward output, loss, parameter gradient and one Adam step."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import unet as ounet
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


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(H, W, B, seed):
    rng = np.random.default_rng(seed)
    theta = inputs.he_init(ounet.fan_segments(), seed)
    theta[-17:] = rng.standard_normal(17).astype(np.float32) * 0.1   # output layer nonzero bias
    x = rng.standard_normal((B, 3, H, W)).astype(np.float32)
    a = (rng.random((B, H, W)) + 0.05).astype(np.float32)
    c = (rng.standard_normal((B, H, W)) * 0.5).astype(np.float32)
    return theta, x, a, c


@pytest.mark.parametrize("H,W,B", [(16, 24, 2), (40, 136, 2)])
def test_unet_forward_and_gradient(esi, H, W, B):
    theta, x, a, c = _case(H, W, B, 11)
    net = esi.Unet(H, W, B)
    net.set_params(torch.from_numpy(theta).to(DEV))
    o = net.forward(torch.from_numpy(x).to(DEV)).cpu().numpy()
    o_ref, cache = ounet.forward(theta.astype(np.float64), x.astype(np.float64), bf=True)
    err_o = _rel(o, o_ref[:, 0])
    L_ref, go = ounet.scaling_loss(o_ref, a[:, None].astype(np.float64), c[:, None].astype(np.float64))
    g_ref = ounet.backward(theta.astype(np.float64), cache, go)
    g, L = net.loss_grad(torch.from_numpy(x).to(DEV), torch.from_numpy(a).to(DEV),
                         torch.from_numpy(c).to(DEV))
    g = g.cpu().numpy()
    err_g = _rel(g, g_ref)
    print(f"H={H} W={W}: output {err_o:.2e}, loss {abs(L - L_ref) / abs(L_ref):.2e}, gradient {err_g:.2e}")
    assert err_o < 5e-3
    assert abs(L - L_ref) < 5e-3 * abs(L_ref)
    assert err_g < 5e-3
    # every layer's block of the gradient
    off = 0
    for name, kind, ci, co in ounet.layers():
        n = int(np.prod(ounet._wshape(kind, ci, co))) + co
        assert _rel(g[off:off + n], g_ref[off:off + n]) < 2e-2, name
        off += n
    net.close()


def test_unet_adam_step(esi):
    theta, x, a, c = _case(16, 16, 1, 12)
    net = esi.Unet(16, 16, 1)
    net.set_params(torch.from_numpy(theta).to(DEV))
    g, _ = net.loss_grad(torch.from_numpy(x).to(DEV), torch.from_numpy(a).to(DEV),
                         torch.from_numpy(c).to(DEV))
    gh = g.cpu().numpy().astype(np.float64)
    net.adam(g, lr=1e-3, step=1)
    net.adam(g, lr=1e-3, step=2, clip=0.5 * float(np.linalg.norm(gh)))
    th = net.get_params().cpu().numpy()
    ref, m, v = ounet.adam_step(theta.astype(np.float64), gh, 0 * gh, 0 * gh, 1, 1e-3)
    ref, m, v = ounet.adam_step(ref, gh, m, v, 2, 1e-3, clip=0.5 * float(np.linalg.norm(gh)))
    assert np.max(np.abs(th - ref)) < 1e-6
    net.close()


def test_unet_loss_weights(esi):
    """esi_unet_loss_weights equals the oracle's default weights (including
    the zero weight of a sample whose sum c is negative), and passing them
    explicitly reproduces the default loss."""
    theta, x, a, c = _case(16, 24, 3, 13)
    c[2] = -np.abs(c[2])
    net = esi.Unet(16, 24, 3)
    net.set_params(torch.from_numpy(theta).to(DEV))
    at, ct, xt = (torch.from_numpy(v).to(DEV) for v in (a, c, x))
    w = net.loss_weights(at, ct).cpu().numpy()
    np.testing.assert_allclose(w, ounet.loss_weights(a[:, None].astype(np.float64), c[:, None].astype(np.float64)),
                               rtol=1e-6)
    assert w[2] == 0.0
    g1, L1 = net.loss_grad(xt, at, ct)
    g2, L2 = net.loss_grad(xt, at, ct, weight=torch.from_numpy(w).to(DEV))
    assert abs(L1 - L2) <= 1e-6 * abs(L1)
    assert _rel(g2.cpu().numpy(), g1.cpu().numpy()) < 1e-6
    net.close()


def test_unet_batch_equals_single_images(esi):
    """At the solver's image size (408 x 808) a batch of 8 runs each workgroup
    of the persistent convolution kernels over several tiles (5304 full-
    resolution tiles, several per resident workgroup); one image alone nearly
    fits in one pass.  A tile's arithmetic does not depend on which workgroup
    takes it, so every image of the batch matches its own single-image forward
    bit for bit."""
    H, W, B = 408, 808, 8
    rng = np.random.default_rng(21)
    theta = inputs.he_init(ounet.fan_segments(), 21)
    x = torch.from_numpy(rng.standard_normal((B, 3, H, W)).astype(np.float32)).to(DEV)
    net = esi.Unet(H, W, B)
    net.set_params(torch.from_numpy(theta).to(DEV))
    ob = net.forward(x).clone()
    assert torch.isfinite(ob).all()
    for i in range(B):
        oi = net.forward(x[i:i + 1].contiguous())
        assert torch.equal(ob[i], oi[0]), i
    net.close()
