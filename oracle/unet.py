"""FP64 oracle of the learned preconditioner's network (test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline use this
module; the product path never imports it.

The paper leaves preconditioning open (Sec. 4.2, Sec. 6: fewer inner CG
iterations need an efficient preconditioner).  The network here is a
four-level U-Net, written out plainly in NumPy (NCHW, float64):

  encoder  conv3x3(3->16) relu conv3x3(16->16) relu        -> e1   (H, W)
           avgpool 2x2, conv(16->32) relu conv(32->32) relu  -> e2   (H/2)
           avgpool,     conv(32->64) relu conv(64->64) relu  -> e3   (H/4)
           avgpool,     conv(64->128) relu conv(128->128) relu -> b  (H/8)
  decoder  convT2x2(128->64), concat [up, e3], conv(128->64) relu conv(64->64) relu
           convT2x2(64->32),  concat [up, e2], conv(64->32) relu conv(32->32) relu
           convT2x2(32->16),  concat [up, e1], conv(32->16) relu conv(16->16) relu
           conv1x1(16->1) -> o

3x3 convolutions use zero padding (same size); H and W are multiples of 8.
With ``bf16=True`` every weight and every activation at a layer boundary is
rounded to bfloat16 (round to nearest even) and biases, accumulation and the
output o stay in float64; gradients of activations are rounded the same way
on the way back.  With ``bf16=False`` everything is float64 (used for the
finite-difference pins).

Flat parameter vector: layers in the order above, each layer's weight then
its bias.  Weight layouts: conv3x3 [co][ci][3][3], convT [ci][co][2][2],
conv1x1 [co][ci].

Loss of the scaling preconditioner: the network maps the inputs of one shot
to o(x) and the correction is z = exp(o) r.  With a(x) = sum_t r^2 and
c(x) = sum_t r e (e the error x_ref - x_k), the squared error sum_{x,t}
(exp(o) r - e)^2 equals sum_x a exp(2o) - 2 c exp(o) + const.  Per sample the
loss is that sum times a weight w, by default w = sum_x a / (sum_x c)^2 (0
when sum_x c <= 0): 0 for z = 0 and -1 for the best single scale sum c /
sum a, lower for a better cell scaling; the batch loss is the mean over
samples.  Tiles of a larger image take the weight of the whole image.
"""
from __future__ import annotations

import numpy as np

CONV3 = [("c1a", 3, 16), ("c1b", 16, 16), ("c2a", 16, 32), ("c2b", 32, 32),
         ("c3a", 32, 64), ("c3b", 64, 64), ("c4a", 64, 128), ("c4b", 128, 128)]


def layers():
    """(name, kind, cin, cout) in flat-vector order."""
    L = [(n, "conv3", ci, co) for n, ci, co in CONV3]
    L += [("u3", "convT", 128, 64), ("d3a", "conv3", 128, 64), ("d3b", "conv3", 64, 64),
          ("u2", "convT", 64, 32), ("d2a", "conv3", 64, 32), ("d2b", "conv3", 32, 32),
          ("u1", "convT", 32, 16), ("d1a", "conv3", 32, 16), ("d1b", "conv3", 16, 16),
          ("out", "conv1", 16, 1)]
    return L


def _wshape(kind, ci, co):
    return {"conv3": (co, ci, 3, 3), "convT": (ci, co, 2, 2), "conv1": (co, ci)}[kind]


def num_params() -> int:
    return sum(int(np.prod(_wshape(k, ci, co))) + co for _, k, ci, co in layers())


def fan_segments():
    """(weight count, fan-in, bias count) per layer, for the seeded initializer."""
    out = []
    for _, k, ci, co in layers():
        fan = {"conv3": 9 * ci, "convT": ci, "conv1": ci}[k]
        out.append((int(np.prod(_wshape(k, ci, co))), fan, co))
    return out


def unpack(flat):
    """Flat vector -> {name: (W, b)} views as float64."""
    flat = np.asarray(flat, dtype=np.float64)
    P, off = {}, 0
    for name, k, ci, co in layers():
        shp = _wshape(k, ci, co)
        n = int(np.prod(shp))
        P[name] = (flat[off:off + n].reshape(shp), flat[off + n:off + n + co])
        off += n + co
    assert off == flat.size
    return P


def pack(grads):
    return np.concatenate([np.concatenate([grads[n][0].ravel(), grads[n][1].ravel()])
                           for n, _, _, _ in layers()])


# ---------------------------------------------------------------------------
def bf16(x):
    """Round to the nearest bfloat16 (ties to even) and return float64.

    The value is first rounded to float32 (as the GPU holds it), then the low
    16 bits of the float32 pattern are rounded away.
    """
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _rb(x, on):
    return bf16(x) if on else x


def conv3x3(x, w, b):
    """y[n,o,i,j] = b[o] + sum_{c,dy,dx} w[o,c,dy,dx] x[n,c,i+dy-1,j+dx-1], zero outside."""
    n, c, h, wd = x.shape
    xp = np.zeros((n, c, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((n, w.shape[0], h, wd))
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + h, dx:dx + wd]                 # [n,c,h,w]
            y += np.einsum("oc,nchw->nohw", w[:, :, dy, dx], patch)
    return y + b[None, :, None, None]


def conv3x3_backward(x, w, gy):
    """Gradients of conv3x3 w.r.t. x, w and b given gy = dL/dy."""
    n, c, h, wd = x.shape
    xp = np.zeros((n, c, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + h, dx:dx + wd]
            gw[:, :, dy, dx] = np.einsum("nohw,nchw->oc", gy, patch)
            gxp[:, :, dy:dy + h, dx:dx + wd] += np.einsum("oc,nohw->nchw", w[:, :, dy, dx], gy)
    return gxp[:, :, 1:-1, 1:-1], gw, gy.sum(axis=(0, 2, 3))


def convT2(x, w, b):
    """y[n,o,2i+a,2j+d] = b[o] + sum_c w[c,o,a,d] x[n,c,i,j]."""
    n, c, h, wd = x.shape
    y = np.zeros((n, w.shape[1], 2 * h, 2 * wd))
    for a in range(2):
        for d in range(2):
            y[:, :, a::2, d::2] = np.einsum("co,nchw->nohw", w[:, :, a, d], x)
    return y + b[None, :, None, None]


def convT2_backward(x, w, gy):
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for a in range(2):
        for d in range(2):
            g = gy[:, :, a::2, d::2]
            gx += np.einsum("co,nohw->nchw", w[:, :, a, d], g)
            gw[:, :, a, d] = np.einsum("nchw,nohw->co", x, g)
    return gx, gw, gy.sum(axis=(0, 2, 3))


def avgpool2(x):
    n, c, h, w = x.shape
    return x.reshape(n, c, h // 2, 2, w // 2, 2).mean(axis=(3, 5))


def avgpool2_backward(gy):
    return np.repeat(np.repeat(gy, 2, axis=2), 2, axis=3) * 0.25


# ---------------------------------------------------------------------------
def forward(flat, x, bf=True):
    """U-Net output o [n,1,H,W] and the cache the backward pass needs."""
    P = unpack(flat)
    W = {k: (_rb(w, bf), b) for k, (w, b) in P.items()}
    cache = {"W": W, "bf": bf}
    h = _rb(x, bf)
    cache["x"] = h

    def cr(name, inp):                       # conv3x3 + relu, output rounded
        y = _rb(np.maximum(conv3x3(inp, *W[name]), 0.0), bf)
        cache[name] = (inp, y)
        return y

    e1 = cr("c1b", cr("c1a", h))
    p1 = _rb(avgpool2(e1), bf)
    e2 = cr("c2b", cr("c2a", p1))
    p2 = _rb(avgpool2(e2), bf)
    e3 = cr("c3b", cr("c3a", p2))
    p3 = _rb(avgpool2(e3), bf)
    bt = cr("c4b", cr("c4a", p3))
    cur = bt
    for up, da, db, skip in (("u3", "d3a", "d3b", e3), ("u2", "d2a", "d2b", e2),
                             ("u1", "d1a", "d1b", e1)):
        u = _rb(convT2(cur, *W[up]), bf)
        cache[up] = (cur, u)
        cat = np.concatenate([u, skip], axis=1)
        cur = cr(db, cr(da, cat))
    wo, bo = W["out"]
    o = np.einsum("oc,nchw->nohw", wo, cur) + bo[None, :, None, None]
    cache["out"] = (cur, o)
    return o, cache


def backward(flat, cache, go):
    """Flat gradient of the loss given go = dL/do (same layout as the params)."""
    W, bf = cache["W"], cache["bf"]
    G = {}
    cur, _ = cache["out"]
    wo, _ = W["out"]
    G["out"] = (np.einsum("nohw,nchw->oc", go, cur), go.sum(axis=(0, 2, 3)))
    g = _rb(np.einsum("oc,nohw->nchw", wo, go), bf)

    def bcr(name, gy):                       # back through relu + conv3x3
        inp, y = cache[name]
        gy = gy * (y > 0)
        gx, gw, gb = conv3x3_backward(inp, W[name][0], gy)
        G[name] = (gw, gb)
        return _rb(gx, bf)

    skips = {}
    for up, da, db, ch in (("u1", "d1a", "d1b", 16), ("u2", "d2a", "d2b", 32),
                           ("u3", "d3a", "d3b", 64)):
        gcat = bcr(da, bcr(db, g))
        gu, skips[up] = gcat[:, :ch], gcat[:, ch:]
        inp, _ = cache[up]
        gx, gw, gb = convT2_backward(inp, W[up][0], gu)
        G[up] = (gw, gb)
        g = _rb(gx, bf)
    g = bcr("c4a", bcr("c4b", g))
    g = _rb(avgpool2_backward(g), bf) + skips["u3"]
    g = bcr("c3a", bcr("c3b", g))
    g = _rb(avgpool2_backward(g), bf) + skips["u2"]
    g = bcr("c2a", bcr("c2b", g))
    g = _rb(avgpool2_backward(g), bf) + skips["u1"]
    g = bcr("c1a", bcr("c1b", g))
    return pack(G)


def loss_weights(a, c):
    """Default per-sample weight sum_x a / (sum_x c)^2, 0 when sum_x c <= 0."""
    n = a.shape[0]
    sa = a.reshape(n, -1).sum(axis=1)
    sc = c.reshape(n, -1).sum(axis=1)
    return np.where((sc > 0) & (sa > 0), sa / np.where(sc > 0, sc * sc, 1.0), 0.0)


def scaling_loss(o, a, c, w=None):
    """Loss of the scaling preconditioner and dL/do.

    o, a, c: [n,1,H,W]; per sample L_s = w_s sum_x (a e^{2o} - 2 c e^{o}) with
    w = loss_weights(a, c) unless given; L = mean_s L_s.
    """
    n = o.shape[0]
    w = loss_weights(a, c) if w is None else np.asarray(w, np.float64)
    s = np.exp(o)
    ww = w[:, None, None, None]
    L = float(np.mean((ww * (a * s * s - 2.0 * c * s)).reshape(n, -1).sum(axis=1)))
    go = ww * (2.0 * a * s * s - 2.0 * c * s) / n
    return L, go


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, clip=0.0):
    """One Adam update (Kingma & Ba 2015) of flat float64 arrays; t counts from
    1.  With clip > 0 the gradient is first scaled to norm at most clip."""
    if clip > 0:
        nrm = np.sqrt(np.sum(g * g))
        if nrm > clip:
            g = g * (clip / nrm)
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def precond_inputs(r, v, w2):
    """Network input of one shot: [log(1 + rms_t r / mean_x(rms_t r)), v / 3000, log(B) / 4].

    r: [nt, nz, nx] residual; v: [nz, nx] m/s; w2 = B^2 on the physical grid.
    Also returns a = sum_t r^2, the per-cell energy of r.
    """
    a = np.sum(np.asarray(r, np.float64) ** 2, axis=0)
    rms = np.sqrt(a / r.shape[0])
    mu = rms.mean()
    ch0 = np.log1p(rms / mu if mu > 0 else rms)
    return np.stack([ch0, np.asarray(v, np.float64) / 3000.0, np.log(np.sqrt(w2)) / 4.0]), a
