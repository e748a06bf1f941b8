"""Training data and training loop of the learned preconditioner.

Every computation runs in the library's kernels (propagation, CG, flexible CG,
feature maps, network forward / backward, Adam); this module allocates device
buffers, indexes batches and loops.

Training pairs.  For a model and its shots, the normal equation is solved
accurately once (flexible CG with the analytic cell scale
1 / (beta B^2 + gamma), to a relative residual of `ref_rtol`) to give x_ref.
Then two runs record, per iteration k, the cell maps a = sum_t r_k^2 and
c = sum_t r_k (x_ref - x_k):
  * plain CG (k = 0 .. k_plain): the iterates the preconditioner first meets;
  * flexible CG with the analytic scale (every `fcg_every`-th k up to
    k_fcg): residuals of the preconditioned regime.
The network learns a correction on top of the analytic scale s0 = 1 / (beta
B^2 + gamma0): the preconditioner is z = s0 exp(o) r.  A sample is the
network input of (a, v, B) with the padded a s0^2 and c s0, so the loss
(esi_unet_loss_grad) is the squared error of s0 exp(o) r against e = x_ref -
x_k; o = 0 is the analytic preconditioner itself.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import esi, inputs


def pad8(n: int) -> int:
    return (n + 7) // 8 * 8


def analytic_scale(plan, gamma: float) -> torch.Tensor:
    """The library's analytic cell scale of every shot of `plan`
    (esi_precond_scale); float32 [nshots, nz, nx] on the device."""
    return plan.precond_scale(gamma)


def observed_data(cfg, device="cuda") -> torch.Tensor:
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(device))
    w = torch.from_numpy(np.tile(cfg.wavelet, (cfg.nshots, 1))).to(device)
    d = plan.forward(w, esi.SRC_POINT)
    plan.close()
    return d


GAMMA0 = 0.03


def tiles(X, A, C, Wt, th, tw):
    """Cut padded images larger than th x tw into tiles of that size (first
    and last offset along each axis); every tile keeps its image's loss
    weight Wt."""
    H, W = X.shape[2], X.shape[3]
    if (H, W) == (th, tw):
        return X, A, C, Wt
    ro = sorted({0, H - th}) if H > th else [0]
    co = sorted({0, W - tw}) if W > tw else [0]
    xs, as_, cs, ws = [], [], [], []
    for r in ro:
        for c in co:
            xs.append(X[:, :, r:r + th, c:c + tw])
            as_.append(A[:, r:r + th, c:c + tw])
            cs.append(C[:, r:r + th, c:c + tw])
            ws.append(Wt)
    return (torch.cat(xs).contiguous(), torch.cat(as_).contiguous(), torch.cat(cs).contiguous(),
            torch.cat(ws).contiguous())


def loss_weights(A, C) -> torch.Tensor:
    """Default loss weights of whole images (esi_unet_loss_weights)."""
    lib = esi.load_library()
    n = int(A.shape[0])
    w = torch.empty(n, dtype=torch.float32, device=A.device)
    esi._check(lib.esi_unet_loss_weights(esi._ptr(A.contiguous()), esi._ptr(C.contiguous()), n,
                                         int(A[0].numel()), esi._ptr(w),
                                         __import__("ctypes").c_void_p(torch.cuda.current_stream(A.device).cuda_stream)))
    return w


def model_pairs(cfg, k_plain=25, k_fcg=130, fcg_every=5, gamma=GAMMA0, ref_rtol=2e-4, ref_iters=600,
                device="cuda", log=None):
    """Samples (x_in [n, 3, Hp, Wp], a [n, Hp, Wp], c [n, Hp, Wp]) of one model."""
    d = observed_data(cfg, device)
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(device))
    S = analytic_scale(plan, gamma)
    ns = cfg.nshots
    work = torch.empty((3, *plan.vec_shape(ns)), dtype=torch.float32, device=device)
    xref, rep = plan.fpcg_solve(d, ref_iters, rtol=ref_rtol, scale=S, work=work)
    x = plan.new_vec(ns)
    Hp, Wp = pad8(cfg.nz), pad8(cfg.nx)
    X, A, C = [], [], []

    def collect(out, ks, reached):
        for k in ks:
            for s in range(ns):
                if k > reached[s]:
                    continue
                a = out[k, s:s + 1, 0].reshape(1, cfg.nz, cfg.nx)
                c = out[k, s:s + 1, 1].reshape(1, cfg.nz, cfg.nx)
                xin, ap, cp = plan.precond_features(a, Hp, Wp, cmap=c, base=S[s:s + 1].contiguous(), shot0=s,
                                                    nshots=1, pads=True)
                X.append(xin)
                A.append(ap)
                C.append(cp)

    out = torch.zeros((k_plain + 1, ns, 2, plan.nphys), dtype=torch.float32, device=device)
    _, r1 = plan.fpcg_solve(d, k_plain, x=x, work=work, stat_xref=xref, stat_out=out)
    collect(out, range(k_plain + 1), r1["shot_iters"])
    out = torch.zeros((k_fcg + 1, ns, 2, plan.nphys), dtype=torch.float32, device=device)
    _, r2 = plan.fpcg_solve(d, k_fcg, scale=S, x=x, work=work, stat_xref=xref, stat_out=out)
    collect(out, range(fcg_every, k_fcg + 1, fcg_every), r2["shot_iters"])
    plan.close()
    if log:
        log(f"{cfg.name}: reference {rep['shot_iters'].tolist()} iterations, "
            f"{len(X)} samples")
    return torch.cat(X), torch.cat(A), torch.cat(C)


def build_dataset(seeds, nx=401, nz=201, nshots=4, nt=1500, device="cuda", log=None, tile=(208, 408), **kw):
    """Samples (x_in, a, c, loss weight) of the models `seeds` at nx x nz,
    cut into tiles of `tile`; samples whose weight is 0 are dropped."""
    Xs, As, Cs, Ws = [], [], [], []
    for sd in seeds:
        cfg = inputs.cfg_precond(int(sd), nx=nx, nz=nz, nshots=nshots, nt=nt)
        X, A, C = model_pairs(cfg, device=device, log=log, **kw)
        Wt = loss_weights(A, C)
        keep = torch.nonzero(Wt > 0).flatten()
        X, A, C, Wt = tiles(X[keep], A[keep], C[keep], Wt[keep], *tile)
        Xs.append(X)
        As.append(A)
        Cs.append(C)
        Ws.append(Wt)
    return torch.cat(Xs), torch.cat(As), torch.cat(Cs), torch.cat(Ws)


def init_params(seed: int, A: torch.Tensor, C: torch.Tensor) -> torch.Tensor:
    """He-initialised parameters with a quiet output layer whose bias is the
    log of the best single scale sum c / sum a of the data."""
    from . import unet_layout
    theta = inputs.he_init(unet_layout.fan_segments(), seed)
    theta[-17:-1] *= 0.1
    s = float(C.double().sum() / A.double().sum())
    theta[-1] = np.log(max(s, 1e-6))
    return torch.from_numpy(theta).to(A.device)


def train(X, A, C, Wt, epochs=8, batch=16, lr=3e-4, clip=1.0, seed=0, val_frac=0.05, log=None):
    """Adam (gradient norm clipped to `clip`, cosine learning-rate decay) on
    the scaling loss; returns (theta, history)."""
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    nval = max(1, int(n * val_frac))
    val, tr = perm[:nval], perm[nval:]
    H, W = X.shape[2], X.shape[3]
    net = esi.Unet(H, W, batch, device=X.device)
    theta = init_params(seed, A, C)
    net.set_params(theta)
    grad = torch.empty(net.P, dtype=torch.float32, device=X.device)
    hist = []
    step = 0

    def evaluate():
        tot = 0.0
        for i in range(0, nval, batch):
            idx = torch.from_numpy(val[i:i + batch]).to(X.device)
            _, L = net.loss_grad(X[idx].contiguous(), A[idx].contiguous(), C[idx].contiguous(), grad,
                                 weight=Wt[idx].contiguous())
            tot += L * len(idx)
        return tot / nval

    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(tr)
        lr_ep = lr * (0.5 * (1.0 + np.cos(np.pi * ep / epochs)))
        tl, cnt = 0.0, 0
        for i in range(0, len(order) - batch + 1, batch):
            idx = torch.from_numpy(order[i:i + batch]).to(X.device)
            _, L = net.loss_grad(X[idx].contiguous(), A[idx].contiguous(), C[idx].contiguous(), grad,
                                 weight=Wt[idx].contiguous())
            step += 1
            net.adam(grad, lr_ep, step, clip=clip)
            tl += L
            cnt += 1
        v = evaluate()
        hist.append({"epoch": ep, "train_loss": tl / max(cnt, 1), "val_loss": v, "lr": lr_ep,
                     "seconds": time.time() - t0})
        if log:
            log(f"epoch {ep}: train {tl / max(cnt, 1):.4f} val {v:.4f} lr {lr_ep:.2e} "
                f"({time.time() - t0:.0f} s)")
    theta = net.get_params()
    net.close()
    return theta, hist


def cell_optimum_loss(A, C, Wt) -> float:
    """Mean loss of the per-cell optimum exp(o) = c / a (a bound no cell
    scaling beats; the best single scale of a whole image scores -1)."""
    a = A.double().flatten(1)
    c = C.double().flatten(1)
    q = torch.where(a > 0, c * c / a.clamp_min(1e-300), torch.zeros_like(a)).sum(1)
    return float((-q * Wt.double()).mean())


def true_residual(plan, b, x):
    """||b - N x|| / ||b|| per shot (float64 norms of device vectors)."""
    Nx, _ = plan.normal_apply(x, want_pAp=False)
    return [float(torch.linalg.norm((b[s] - Nx[s]).double()) / torch.linalg.norm(b[s].double()))
            for s in range(b.shape[0])]


NET_EVERY = 10


def compare_solvers(cfg, theta=None, rtol=1e-3, max_iter=600, gamma=GAMMA0, device="cuda", log=None,
                    methods=("plain", "analytic", "learned"), net_every=NET_EVERY, plain_max_iter=None):
    """Plain CG, flexible CG with the analytic scale s0, and flexible CG with
    the learned correction s0 exp(Net) ("learned": the network on r_0 and then
    on every net_every-th iteration's residual; "learned_fixed": once, on r_0)
    on one model, each to a relative residual `rtol`: iterations per shot, wall
    time, true residual.  plain_max_iter caps plain CG (default max_iter)."""
    d = observed_data(cfg, device)
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(device))
    ns = cfg.nshots
    work = torch.empty((3, *plan.vec_shape(ns)), dtype=torch.float32, device=device)
    x = plan.new_vec(ns)
    S0 = analytic_scale(plan, gamma)
    net = None
    if theta is not None and any(m.startswith("learned") for m in methods):
        net = esi.Unet(pad8(cfg.nz), pad8(cfg.nx), ns, device=device)
        net.set_params(theta)
    b = plan.adjoint(d)
    out = {}
    for m in methods:
        if m.startswith("learned") and net is None:
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if m == "plain":
            _, rep = plan.cg_solve(d, plain_max_iter or max_iter, rtol, x=x, work=work)
            rep["fallback"] = np.full(ns, -1)
        else:
            _, rep = plan.fpcg_solve(d, max_iter, rtol, net=net if m.startswith("learned") else None, scale=S0,
                                     x=x, work=work, net_every=0 if m == "learned_fixed" else net_every)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        its = rep["shot_iters"]
        reached = [float(rep["res_hist"][s][its[s]]) for s in range(ns)]
        out[m] = {"iters": its.tolist(), "seconds": el, "recursive_residual": reached,
                  "true_residual": true_residual(plan, b, x), "fallback": np.asarray(rep["fallback"]).tolist(),
                  "converged": bool(all(r < rtol for r in reached))}
        if log:
            log(f"{cfg.name} {m}: iterations {its.tolist()} in {el:.2f} s, true residual "
                f"{np.round(out[m]['true_residual'], 5).tolist()}")
    if net is not None:
        net.close()
    plan.close()
    return out
