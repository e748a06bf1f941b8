"""Benchmark of the ESI hot path on one MI355X.

One step = the whole hot path over one batch of synthetic input: for every
shot group, the right-hand side S^T d by adjoint modelling, K iterations of
CG on (S^T S + beta B^T B) q = S^T d (two propagations each) and the PENALTY
gradient (one propagation).  Default workload: 801 x 401 grid, dx 12.5 m,
layered model with 3 anomalies, 32 shots of an 8 Hz Ricker, 401 receivers,
2000 steps of 1 ms, 20 CG iterations in the smoothed start model, full
wavefield storage of the CG vectors, shots in groups of 16.

Prints one JSON line.  value = padded grid-point updates per second over the
whole timed region (GPts/s).  The roofline object covers the dominant time-step
kernel, timed live with hipEvents around its time loops inside the timed
region; cpu_baseline is the FP64 oracle on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "stencil GPts/s + %HBM peak; ESI CG solve time to 1e-3 residual, plain vs learned PCG"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# algorithmic bytes of one time-step launch, per shot: 16 B per padded point
# (read u^n, u^{n-1}, c; write u^{n+1}) plus the dense streams of its variant
# per physical point: SRC_DENSE reads q (4), CG_FUSE reads r, p, x and writes
# p, x (20), OUT writes mu (4), NORMAL reads p and writes N p (8), STORE
# writes (dA/dm)u (4), CORR reads it back (4).  The gradient images the
# correlations add into (PENALTY, CORR) are accumulators, not streams of the
# method: they count 0 (PENALTY's q read is SRC_DENSE's).
DENSE_BYTES = {2: 4, 4: 20, 32: 4, 64: 8, 128: 0, 256: 4, 512: 4}


TWO_STEP = 1 << 15
RUPD = 1 << 14
CORR = 1 << 9
VARIANT_MASK = (1 << 15) - 1
TILE_2D = {2: "56x32", 3: "56x24", 4: "56x40"}


def launch_label(flags: int, ndim: int = 2) -> str:
    """Counter-summary label of a profiled loop's launches: '1step', the 2D
    two-step tile ('56x32', '56x24', '56x40') or '2step' (3D)."""
    if not flags & TWO_STEP:
        return "1step"
    return TILE_2D.get((flags >> 16) & 7, "56x32") if ndim == 2 else "2step"

# HBM counter summaries of the time-step kernels (two rocprofv3 --pmc passes,
# FETCH_SIZE and WRITE_SIZE, calibrated on a copy of known size), one per
# workload, each tied to a hash of the kernel sources it was measured on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step2d_t2_single-solve-801x401_traffic.md")
TRAFFIC_FILE_BATCHING = os.path.join(ROOT, "profiles", "k_step2d_t2_batching-1601x601-128shots_traffic.md")
TRAFFIC_FILE_3D = os.path.join(ROOT, "profiles", "k_step3d_diff3d-256x256x256-8shots_traffic.md")
KERNEL_SOURCES = ["paper_2211_06300_amd/csrc/step2d.hip", "paper_2211_06300_amd/csrc/esi_internal.h"]
KERNEL_SOURCES_3D = ["paper_2211_06300_amd/csrc/step3d.hip", "paper_2211_06300_amd/csrc/step3d_t2.hip",
                     "paper_2211_06300_amd/csrc/esi_internal.h"]


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(flags: int, shots_per_launch: float, path: str = TRAFFIC_FILE,
                     sources=KERNEL_SOURCES, ndim: int = 2):
    """HBM bytes per launch of the profiled loop `flags` from a committed
    counter summary, or None when the kernel sources changed since the counters
    were taken or the launch shape differs.  Rows name the variant's flag
    number and its launch label ("16404 56x32", "520 1step", "520 2step")."""
    try:
        with open(path) as fh:
            text = fh.read()
    except OSError:
        return None
    meta = {}
    for line in text.splitlines():
        for key in ("kernel-sources-sha256-16:", "calibration:", "shots-per-launch:"):
            if line.startswith(key):
                meta[key] = line[len(key):].split()
    if meta.get("kernel-sources-sha256-16:", [None])[0] != kernel_source_hash(sources):
        return None
    if float(meta["shots-per-launch:"][0]) != shots_per_launch:
        return None
    key = f"{flags & VARIANT_MASK} {launch_label(flags, ndim)}"
    cf, cw = float(meta["calibration:"][1]), float(meta["calibration:"][3])
    fi = wi = None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if "FETCH_SIZE KiB" in cells and "WRITE_SIZE KiB" in cells:   # the table's header
            fi, wi = cells.index("FETCH_SIZE KiB"), cells.index("WRITE_SIZE KiB")
        elif fi is not None and len(cells) > max(fi, wi) and cells[0] == key:
            return int((cf * float(cells[fi]) + cw * float(cells[wi])) * 1024)
    return None


def copy_bandwidth(torch, dev, mib: int = 2048, reps: int = 10) -> float:
    """Measured HBM bandwidth of a plain streaming kernel on this GPU: an
    elementwise multiply by 1 of `mib` MiB (read and written once), GB/s."""
    a = torch.ones(mib * 262144, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        torch.mul(a, 1.0, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * mib * 1048576 / (ms * 1e-3) / 1e9


def tune_report(esi, tuned, table, names=None):
    """The autotuner's choice and candidate table (milliseconds of the timed
    forward-type and adjoint-type loops per launch shape)."""
    names = esi.LAUNCH_NAMES if names is None else names
    return {"forward": names.get(tuned[0], str(tuned[0])), "adjoint": names.get(tuned[1], str(tuned[1])),
            "chosen_by": "autotuner",
            "candidates_ms": {names.get(sh, str(sh)): {"forward": round(f, 3), "adjoint": round(a, 3)}
                              for sh, f, a in table}}


def roofline(kernel: str, alg_bytes: float, launch_us: float, traffic, peak_measured):
    """Roofline object of one kernel: algorithmic bytes per launch over the
    average launch time against the 8 TB/s HBM peak, plus the counted HBM rate
    when counters for this kernel and launch shape are committed."""
    achieved = alg_bytes / launch_us / 1e3
    out = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "alg_bytes_per_launch": int(alg_bytes), "avg_launch_us": round(launch_us, 2),
           "hbm_frac_counted": None if traffic is None else round(traffic / launch_us / 1e3 / HBM_PEAK_GBS, 4)}
    if peak_measured:
        out["peak_measured"] = round(peak_measured, 1)
        out["frac_of_measured"] = round(achieved / peak_measured, 4)
        if traffic is not None:
            out["hbm_frac_counted_of_measured"] = round(traffic / launch_us / 1e3 / peak_measured, 4)
    return out


def bytes_per_shot_launch(flags: int, npad: int, nphys: int) -> int:
    """Algorithmic bytes of one launch for one shot (a two-step launch counts
    both steps)."""
    b = 16 * npad
    for bit, per in DENSE_BYTES.items():
        if flags & bit:
            b += per * nphys
    if flags & RUPD and flags & 64:   # the fused residual update: r read and written, no N p written
        b += 4 * nphys
    return b * (2 if flags & TWO_STEP else 1)


def bench_dense_bytes(flags: int) -> int:
    """Algorithmic dense-stream bytes per physical cell of one step of a variant."""
    return bytes_per_shot_launch(flags & VARIANT_MASK & ~TWO_STEP, 0, 1)


def cpu_baseline(cfg, nt_sample: int, iters: int = 3):
    """FP64 oracle (plain C loops, OpenMP over rows) on a bounded sample of the
    same solve: one shot, the first nt_sample steps of the time axis, the
    right-hand side S^T d plus `iters` CG iterations (1 + 2 iters propagations)."""
    from oracle import core
    g = core.Grid(2, cfg.nz, cfg.nx, nb=cfg.nb, nt=nt_sample, dx=cfg.dx, dt=cfg.dt)
    m_true = core.make_model(g, cfg.v_true)
    m0 = core.make_model(g, cfg.v_start)
    rec = cfg.shot_rec(0)
    d_obs = core.forward(m_true, cfg.wavelet[:nt_sample].astype(np.float64), rec,
                         src_pos=cfg.src[0])
    t0 = time.perf_counter()
    core.esi_cg(m0, cfg.src[0], rec, d_obs, cfg.beta, iters)
    t = time.perf_counter() - t0
    npad = (cfg.nz + 2 * cfg.nb) * (cfg.nx + 2 * cfg.nb)
    pts = (1 + 2 * iters) * npad * nt_sample
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": pts / t / 1e9, "unit": "GPts/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"1 shot of {cfg.nshots}, steps 0..{nt_sample - 1} of {cfg.nt}: right-hand "
                      f"side + {iters} CG iterations ({1 + 2 * iters} propagations) on the "
                      f"{cfg.nx}x{cfg.nz} grid in {t:.1f} s"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def unet_flops(H: int, W: int) -> int:
    """Multiply-adds x 2 of one network forward pass on an H x W image (real
    channel counts; the 3 input channels count as 3)."""
    from paper_2211_06300_amd import unet_layout
    lvl = {"c1a": 0, "c1b": 0, "c2a": 1, "c2b": 1, "c3a": 2, "c3b": 2, "c4a": 3, "c4b": 3, "u3": 3,
           "d3a": 2, "d3b": 2, "u2": 2, "d2a": 1, "d2b": 1, "u1": 1, "d1a": 0, "d1b": 0, "out": 0}
    macs = 0
    for name, kind, ci, co in unet_layout.LAYERS:
        px = (H >> lvl[name]) * (W >> lvl[name])
        macs += px * ci * co * {"c3": 9, "t2": 4, "c1": 1}[kind]
    return 2 * macs


def unet_roofline_us(H: int, W: int, nb: int, peak_tflops: float = 2500.0, peak_gbs: float = 8000.0) -> float:
    """The network's own ceiling for one forward pass on nb H x W images, in
    microseconds: the sum over its kernels of the larger of the FLOPs at the
    bf16 MFMA peak and the minimum HBM bytes at the HBM peak.  Minimum bytes:
    each input read once and each output written once, bf16 activations (the
    first layer's 3 channels stored as 16), float32 network input and output;
    the input conversion and the three poolings included."""
    from paper_2211_06300_amd import unet_layout
    lvl = {"c1a": 0, "c1b": 0, "c2a": 1, "c2b": 1, "c3a": 2, "c3b": 2, "c4a": 3, "c4b": 3, "u3": 3,
           "d3a": 2, "d3b": 2, "u2": 2, "d2a": 1, "d2b": 1, "u1": 1, "d1a": 0, "d1b": 0, "out": 0}

    def px(level):
        return nb * (H >> level) * (W >> level)

    items = [(0.0, (3 * 4 + 16 * 2) * px(0))]                       # input conversion
    items += [(0.0, c * 2 * px(l) + c * 2 * px(l + 1)) for l, c in ((0, 16), (1, 32), (2, 64))]   # pooling
    for name, kind, ci, co in unet_layout.LAYERS:
        l = lvl[name]
        if kind == "c3":
            items.append((2.0 * 9 * ci * co * px(l), ((16 if ci < 16 else ci) + co) * 2 * px(l)))
        elif kind == "t2":
            items.append((2.0 * 4 * ci * co * px(l), ci * 2 * px(l) + co * 2 * px(l - 1)))
        else:
            items.append((2.0 * ci * co * px(l), (ci * 2 + 4) * px(l)))
    return sum(max(f / (peak_tflops * 1e6), b / (peak_gbs * 1e3)) for f, b in items)


def solver_comparison(args, torch, dev):
    """Plain CG vs flexible CG (analytic scale, learned correction) to a
    relative residual of 1e-3 on held-out models, and the network's forward
    throughput on the MFMA units."""
    from paper_2211_06300_amd import esi, inputs, precond
    wpath = os.path.join(ROOT, "paper_2211_06300_amd", "weights", "precond_unet.npy")
    theta = torch.from_numpy(np.load(wpath)).to(dev)
    seeds = [int(x) for x in args.solve_seeds.split(",")]
    out = {"models": {}, "shots_per_model": args.solve_shots, "nt": args.nt, "rtol": 1e-3,
           "max_iter": args.solve_iters, "plain_max_iter": args.plain_iters, "net_every": precond.NET_EVERY}
    ratios = []
    for i, sd in enumerate(seeds):
        cfg = inputs.cfg_precond(sd, nx=801, nz=401, nshots=args.solve_shots, nt=args.nt)
        # plain CG (capped: in float32 it stalls far above 1e-3) on the first model only
        methods = ("plain", "analytic", "learned") if i == 0 else ("analytic", "learned")
        log(f"solver comparison on {cfg.name}: {cfg.nshots} shots, nt {cfg.nt}, to 1e-3 ({', '.join(methods)})")
        res = precond.compare_solvers(cfg, theta, rtol=1e-3, max_iter=args.solve_iters, log=log, methods=methods,
                                      plain_max_iter=args.plain_iters)
        m = {}
        for k, v in res.items():
            m[k] = {"iterations": v["iters"], "seconds": round(v["seconds"], 3), "reached_rtol": v["converged"],
                    "true_residual_max": round(max(v["true_residual"]), 6), "fallback": v["fallback"]}
        an, lr = res.get("analytic"), res.get("learned")
        if an and lr and an["converged"] and lr["converged"]:
            m["learned_speedup_vs_analytic_wall"] = round(an["seconds"] / lr["seconds"], 3)
            m["learned_iteration_ratio_vs_analytic"] = round(sum(lr["iters"]) / sum(an["iters"]), 3)
            ratios.append(an["seconds"] / lr["seconds"])
        if "plain" in res:
            pl = res["plain"]
            m["plain_time_to_rtol"] = (round(pl["seconds"], 3) if pl["converged"] else
                                       f"> {pl['seconds']:.1f} s (not reached in {args.plain_iters} iterations, "
                                       f"true residual {max(pl['true_residual']):.3g})")
        out["models"][cfg.name] = m
        torch.cuda.empty_cache()
    if ratios:
        out["learned_speedup_vs_analytic_wall"] = {"min": round(min(ratios), 3), "median": round(float(np.median(ratios)), 3),
                                                   "max": round(max(ratios), 3), "models": len(ratios)}
    out["network_forward"] = network_forward_run(args, torch, dev, theta)
    return out


def network_forward_run(args, torch, dev, theta=None):
    """The preconditioner network's forward throughput on the MFMA units:
    8 images of 408 x 808 (the padded 801 x 401 grid), 3 warm-up and 20 timed
    passes with the trained parameters."""
    from paper_2211_06300_amd import esi, precond
    if theta is None:
        wpath = os.path.join(ROOT, "paper_2211_06300_amd", "weights", "precond_unet.npy")
        theta = torch.from_numpy(np.load(wpath)).to(dev)
    H, W, nb = precond.pad8(401), precond.pad8(801), 8
    net = esi.Unet(H, W, nb, device=dev)
    net.set_params(theta)
    x = torch.rand((nb, 3, H, W), dtype=torch.float32, device=dev)
    for _ in range(3):
        net.forward(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        net.forward(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    net.close()
    flops = unet_flops(H, W) * nb
    tfs = flops / (ms * 1e-3) / 1e12
    own = unet_roofline_us(H, W, nb)
    return {"images": nb, "image": f"{W}x{H}", "ms": round(ms, 3),
            "tflops": round(tfs, 2), "bound": "mfma", "peak_tflops": 2500.0,
            "frac": round(tfs / 2500.0, 4), "dtype": "bf16 (fp32 accumulate)",
            "own_roofline_ms": round(own / 1e3, 4),
            "frac_of_own_roofline": round(own / 1e3 / ms, 4)}


def batching_run(args, torch, dev, peak_measured=None):
    """The uneven-aperture batching workload: one FWI-type gradient of all
    shots (forward keeping checkpoints every 50 steps, then the adjoint with
    segment recompute and the imaging correlation), every time step one launch
    over the (shot, tile) work list of all shots' windows."""
    from paper_2211_06300_amd import esi, inputs
    cfg = inputs.cfg_batching(nshots=args.batch_shots, nt=args.batch_nt)
    log(f"batching workload {cfg.name}: nt {cfg.nt}, mean window "
        f"{float(np.mean(cfg.window[:, 1] - cfg.window[:, 0])):.0f} columns")
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(dev))
    w = torch.from_numpy(np.tile(cfg.wavelet, (cfg.nshots, 1))).to(dev)
    seed = plan.forward(w, esi.SRC_POINT)          # adjoint seed with the observed data's shape
    grad = torch.zeros(plan.phys_shape, dtype=torch.float32, device=dev)
    # launch shapes: propagation-only timing run of every candidate over all
    # 128 shots' windows (the wavefield-sized vectors of a normal-operator run
    # would not fit)
    tuned = plan.autotune(probe=True) if not args.all_shapes else (2, 2)
    table = plan.tune_table()
    log(f"batching autotuner: forward {esi.LAUNCH_NAMES[tuned[0]]}, adjoint {esi.LAUNCH_NAMES[tuned[1]]}")

    def one():
        grad.zero_()
        plan.forward_ckpt(w, 50, kind=esi.SRC_POINT)
        plan.gradient(esi.GRAD_SEED_REUSE, w, seed, kind=esi.SRC_POINT, grad_m=grad, ckpt_every=50)

    if args.all_shapes:   # counter runs: one pass with every launch shape
        for sh in (1, 3, 2, 4):
            plan.set_launch_shape(sh, sh)
            one()
        plan.set_launch_shape(*tuned)
    one()
    torch.cuda.synchronize()
    plan.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    one()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    prof = plan.profile_read()
    plan.profile(False)
    plan.close()
    padded_cols = (cfg.window[:, 1] - cfg.window[:, 0] + 2 * cfg.nb).astype(np.int64)
    cells = int(np.sum(padded_cols) * (cfg.nz + 2 * cfg.nb))
    full = cfg.nshots * (cfg.nx + 2 * cfg.nb) * (cfg.nz + 2 * cfg.nb)
    pts = 3 * cells * cfg.nt                         # forward, recompute, adjoint
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    # algorithmic bytes of one launch of the dominant loop over all shots' windows:
    # 16 B per padded window cell plus the variant's dense streams per physical cell
    phys = int(np.sum(cfg.window[:, 1] - cfg.window[:, 0]) * cfg.nz)
    alg = (16 * cells + bench_dense_bytes(rec["flags"]) * phys) * (2 if rec["flags"] & TWO_STEP else 1)
    per_launch_us = rec["ms"] / rec["launches"] * 1e3
    traffic = measured_traffic(rec["flags"], rec["shot_launches"] / rec["launches"], TRAFFIC_FILE_BATCHING)
    kern = ("k_step2d_t2" if rec["flags"] & TWO_STEP else "k_step2d") + f"<{name}>"
    return {"workload": cfg.name, "shots": cfg.nshots, "nt": cfg.nt, "dt": cfg.dt,
            "mean_window_columns": round(float(np.mean(cfg.window[:, 1] - cfg.window[:, 0])), 1),
            "seconds": round(wall, 3), "gpts_per_s": round(pts / wall / 1e9, 2),
            "padded_cells_all_windows": cells, "padded_cells_whole_grid_all_shots": full,
            "propagations": 3, "checkpoint_every": 50,
            "launch_shape": tune_report(esi, tuned, table),
            "gpu_event_ms": round(gpu_ms, 1),
            "dominant_loop": {"variant": name, "launches": rec["launches"], "ms": round(rec["ms"], 1)},
            "roofline": roofline(kern, alg, per_launch_us, traffic, peak_measured),
            "kernel_loops": {k: {"launches": v["launches"], "ms": round(v["ms"], 1)} for k, v in prof.items()}}


def wri_run(args, torch, dev):
    """The WRI variant on the single-solve workload: per group of shots the data
    residual d - S f, the right-hand side S^T (d - S f), CG on
    (S^T S + beta I) q and the PENALTY gradient with u = A^{-1}(f + q)
    (2 + 2 * cg_iters + 1 propagations per shot)."""
    from paper_2211_06300_amd import esi, inputs
    cfg = inputs.cfg_single_solve(nshots=args.shots, nt=args.nt)
    npad = (cfg.nz + 2 * cfg.nb) * (cfg.nx + 2 * cfg.nb)
    G = min(args.group, cfg.nshots)
    groups = [(s, min(G, cfg.nshots - s)) for s in range(0, cfg.nshots, G)]
    plan_true = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(dev))
    wav = torch.from_numpy(np.tile(cfg.wavelet, (cfg.nshots, 1))).to(dev)
    d_obs = plan_true.forward(wav, esi.SRC_POINT)
    plan_true.close()
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(dev))
    plan.set_weight(esi.WEIGHT_IDENTITY)
    x = plan.new_vec(G)
    work = torch.empty((3, *plan.vec_shape(G)), dtype=torch.float32, device=dev)
    grad = torch.zeros(plan.phys_shape, dtype=torch.float32, device=dev)
    offs = [int(cfg.nt * cfg.rec_ptr[s]) for s in range(cfg.nshots + 1)]
    plan.autotune(nshots=G, p=work[0], Ap=work[1])
    hists = {}

    def one(iters):
        grad.zero_()
        for s0, ns in groups:
            d_res = plan.data_residual(wav[s0:s0 + ns], d_obs[offs[s0]:offs[s0 + ns]], shot0=s0, nshots=ns)
            xs, ws = x[:ns], work[:, :ns]
            _, rep = plan.cg_solve(d_res, iters, 0.0, shot0=s0, nshots=ns, x=xs, work=ws)
            plan.wri_gradient(esi.GRAD_PENALTY, wav[s0:s0 + ns], xs, shot0=s0, nshots=ns, grad_m=grad)
            hists[s0] = rep["res_hist"]

    one(2)                                            # warm-up: every kernel once
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    one(args.cg_iters)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    plan.close()
    props = 2 + 2 * args.cg_iters + 1
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    hist = np.concatenate(list(hists.values()))
    return {"workload": "wri-" + cfg.name, "shots": cfg.nshots, "shot_group": G, "nt": cfg.nt,
            "cg_iters": args.cg_iters, "beta": cfg.beta, "propagations_per_shot": props,
            "seconds": round(wall, 3), "gpts_per_s": round(cfg.nshots * props * npad * cfg.nt / wall / 1e9, 2),
            "cg_final_rel_residual_max": float(np.max(hist[:, -1])),
            "dominant_loop": {"variant": name, "launches": rec["launches"], "ms": round(rec["ms"], 1)}}


def invert_run(args, torch, dev):
    """The outer loop of Algorithm 2 on one group of shots of the single-solve
    workload: per evaluation the inner solve (flexible CG with the analytic
    cell scale, invert_cg iterations) and one fused pass for the PENALTY
    gradient, the data and the penalty; L-BFGS with an Armijo line search."""
    from paper_2211_06300_amd import esi, inputs
    cfg = inputs.cfg_single_solve(nshots=args.shots, nt=args.nt)
    ns = min(args.group, cfg.nshots)
    npad = (cfg.nz + 2 * cfg.nb) * (cfg.nx + 2 * cfg.nb)
    plan_true = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(dev))
    wav = torch.from_numpy(np.tile(cfg.wavelet, (ns, 1))).to(dev)
    d_obs = plan_true.forward(wav, esi.SRC_POINT, shot0=0, nshots=ns)
    plan_true.close()
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(dev))
    plan.set_beta(args.invert_beta)
    vel = torch.from_numpy(cfg.v_start.copy()).to(dev)
    mask = torch.ones(plan.phys_shape, dtype=torch.float32, device=dev)
    mask[:5] = 0.0                                    # source and receiver rows keep their model
    x = plan.new_vec(ns)
    work = torch.empty((3, *plan.vec_shape(ns)), dtype=torch.float32, device=dev)
    plan.autotune(nshots=ns, p=work[0], Ap=work[1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inner = {"fcg": esi.INNER_FCG_SCALE, "ds": esi.INNER_DATASPACE, "cg": esi.INNER_CG}[args.invert_inner]
    rep = plan.invert(d_obs, vel, mask=mask, nshots=ns, x=x, work=work, outer_iters=args.invert_iters,
                      cg_iters=args.invert_cg, first_step=0.02, v_min=1400.0, v_max=5000.0, inner=inner)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.close()
    props = 2 * args.invert_cg + (4 if args.invert_inner == "ds" else 2)   # per shot and evaluation
    return {"workload": "invert-" + cfg.name, "shots": ns, "nt": cfg.nt, "beta": args.invert_beta,
            "outer_iters": rep["outer_done"], "inner": {"fcg": "fcg-analytic-scale", "ds": "data-space-cg",
                                                         "cg": "cg"}[args.invert_inner],
            "inner_iters": args.invert_cg,
            "evals": rep["evals"], "line_search_trials": rep["trials"], "J": [round(j, 6) for j in rep["J"]],
            "data_misfit": [round(e, 6) for e in rep["misfit"]], "status": rep["status"],
            "seconds": round(wall, 3), "seconds_per_eval": round(wall / max(rep["evals"], 1), 3),
            "gpts_per_s": round(rep["evals"] * ns * props * npad * cfg.nt / wall / 1e9, 2)}


def dtft_run(args, torch, dev):
    """The DTFT variant on one group of shots of the single-solve workload:
    CG on the frequency vectors at nf frequencies (the inverse DTFT feeds the
    forward pass, the DTFT of the adjoint field accumulates in the adjoint
    pass), then the PENALTY gradient of G x."""
    from paper_2211_06300_amd import esi, inputs
    cfg = inputs.cfg_single_solve(nshots=args.shots, nt=args.nt)
    ns = min(args.group, cfg.nshots)
    npad = (cfg.nz + 2 * cfg.nb) * (cfg.nx + 2 * cfg.nb)
    freqs = np.arange(1, args.dtft_nf + 1) * 2.0            # 2, 4, ... Hz
    plan_true = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(dev))
    wav = torch.from_numpy(np.tile(cfg.wavelet, (ns, 1))).to(dev)
    d_obs = plan_true.forward(wav, esi.SRC_POINT, shot0=0, nshots=ns)
    plan_true.close()
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(dev))
    plan.dtft_set_freqs(freqs)
    if args.dtft_block >= 0:
        plan.set_dtft_block(args.dtft_block)
    block = min(args.dtft_block if args.dtft_block >= 0 else 64, cfg.nt)
    sh = plan.dtft_shape(ns)
    x = torch.empty(sh, dtype=torch.float32, device=dev)
    work = torch.empty((3, *sh), dtype=torch.float32, device=dev)
    grad = torch.zeros(plan.phys_shape, dtype=torch.float32, device=dev)
    plan.autotune(nshots=ns)
    plan.dtft_cg_solve(d_obs, 1, nshots=ns, x=x, work=work)       # warm-up: every kernel once
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    _, rep = plan.dtft_cg_solve(d_obs, args.cg_iters, nshots=ns, x=x, work=work)
    plan.dtft_gradient(x, nshots=ns, grad_m=grad)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    plan.close()
    props = 2 * args.cg_iters + 2
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    vec_gb = 4 * ns * len(freqs) * cfg.nz * cfg.nx * 8 / 1e9
    return {"workload": "dtft-" + cfg.name, "shots": ns, "nt": cfg.nt, "freqs_hz": freqs.tolist(),
            "cg_iters": args.cg_iters, "propagations_per_shot": props, "seconds": round(wall, 3),
            "gpts_per_s": round(ns * props * npad * cfg.nt / wall / 1e9, 2),
            "cg_final_rel_residual_max": float(np.max(rep["res_hist"][:, -1])),
            "cg_vectors_gb": round(vec_gb, 2),
            "block_steps": block, "block_buffer_gb": round(4 * ns * block * cfg.nz * cfg.nx / 1e9, 2),
            "time_domain_cg_vectors_gb": round(4 * ns * cfg.nt * cfg.nz * cfg.nx * 4 / 1e9, 1),
            "dominant_loop": {"variant": name, "launches": rec["launches"], "ms": round(rec["ms"], 1)}}


def dataspace_run(args, torch, dev):
    """The data-space solver on one group of shots of the single-solve
    workload: CG on (beta I + S W^-1 S^T) w = v (cg_iters iterations) and the
    extended source q = (beta W)^-1 S^T (d - w)."""
    from paper_2211_06300_amd import esi, inputs
    cfg = inputs.cfg_single_solve(nshots=args.shots, nt=args.nt)
    ns = min(args.group, cfg.nshots)
    npad = (cfg.nz + 2 * cfg.nb) * (cfg.nx + 2 * cfg.nb)
    plan_true = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(dev))
    wav = torch.from_numpy(np.tile(cfg.wavelet, (ns, 1))).to(dev)
    d_obs = plan_true.forward(wav, esi.SRC_POINT, shot0=0, nshots=ns)
    plan_true.close()
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(dev))
    plan.set_ds_ckpt(args.ds_ckpt)
    plan.autotune(nshots=ns)
    q = plan.new_vec(ns)
    plan.ds_cg_solve(d_obs, 1, nshots=ns, q=q)                 # warm-up: every kernel once
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    w, q, rep = plan.ds_cg_solve(d_obs, args.cg_iters, nshots=ns, q=q)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    # how well the extended source explains the data: ||S q - d|| / ||d|| (untimed)
    d_q = plan.forward(q, esi.SRC_DENSE, nshots=ns)
    q_misfit = float(torch.linalg.vector_norm((d_q - d_obs).double()) / torch.linalg.vector_norm(d_obs.double()))
    w_misfit = float(torch.linalg.vector_norm((w - d_obs).double()) / torch.linalg.vector_norm(d_obs.double()))
    plan.close()
    K = min(args.ds_ckpt, cfg.nt)
    # an operator application: adjoint + forward, plus the recompute of the
    # adjoint field when it is checkpointed (the first pass skips the last segment)
    per_apply = 2 + ((cfg.nt - K) / cfg.nt if K > 0 else 0)
    props = per_apply * (args.cg_iters + 1) + 1
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    dl = int(d_obs.numel())
    if K > 0:
        nseg = -(-cfg.nt // K)
        field = {"adjoint_field": f"checkpointed every {K} steps",
                 "segment_buffer_gb": round(ns * K * cfg.nz * cfg.nx * 4 / 1e9, 2),
                 "checkpoints_gb": round(ns * nseg * 2 * npad * 4 / 1e9, 2)}
    else:
        field = {"adjoint_field": "resident",
                 "adjoint_field_buffer_gb": round(ns * cfg.nt * cfg.nz * cfg.nx * 4 / 1e9, 1)}
    return {"workload": "dataspace-" + cfg.name, "shots": ns, "nt": cfg.nt, "beta": cfg.beta,
            "cg_iters": args.cg_iters, "propagations_per_shot": round(props, 2), "seconds": round(wall, 3),
            "gpts_per_s": round(ns * props * npad * cfg.nt / wall / 1e9, 2),
            "cg_final_rel_residual_max": float(np.max(rep["res_hist"][:, -1])),
            "data_misfit_w": round(w_misfit, 6), "data_misfit_Sq": round(q_misfit, 6),
            "cg_vectors_gb": round(4 * dl * 4 / 1e9, 3), **field,
            "time_domain_cg_vectors_gb": round(4 * ns * cfg.nt * cfg.nz * cfg.nx * 4 / 1e9, 1),
            "dominant_loop": {"variant": name, "launches": rec["launches"], "ms": round(rec["ms"], 1)}}


def diff3d_run(args, torch, dev, peak_measured=None):
    """The 3D differentiation workload: 256^3 cells, 8 shots at once, point
    sources, 128 x 128 receivers, nt steps.  One forward pass keeping
    checkpoints every 50 steps (esi_forward_ckpt), then the backward pass that
    recomputes each 50-step segment and runs the adjoint with the imaging
    correlation (esi_gradient, SEED_REUSE): the two calls behind the autograd
    Function's forward and backward."""
    from paper_2211_06300_amd import esi, inputs
    cfg = inputs.cfg_diff3d(n=256, nt=args.nt3d)
    log(f"3D differentiation workload {cfg.name}: {cfg.nshots} shots, nt {cfg.nt}")
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(dev))
    w = torch.from_numpy(np.stack([cfg.wavelet] * cfg.nshots)).to(dev)
    seed = plan.forward(w, esi.SRC_POINT)                           # adjoint seed of the data's shape
    grad = torch.zeros(plan.phys_shape, dtype=torch.float32, device=dev)
    K = 50
    # launch shape (one or two steps per launch): propagation-only timing run
    tuned = plan.autotune(probe=True) if not args.all_shapes else (1, 1)
    table = plan.tune_table()
    log(f"3D autotuner: forward {esi.LAUNCH_NAMES_3D[tuned[0]]}, adjoint {esi.LAUNCH_NAMES_3D[tuned[1]]}")
    if args.all_shapes:   # counter runs: one pass with every launch shape
        for sh in (1, 2):
            plan.set_launch_shape(sh, sh)
            grad.zero_()
            plan.forward_ckpt(w, K, kind=esi.SRC_POINT)
            plan.gradient(esi.GRAD_SEED_REUSE, w, seed, kind=esi.SRC_POINT, grad_m=grad, ckpt_every=K)
        plan.set_launch_shape(*tuned)

    def one():
        grad.zero_()
        plan.forward_ckpt(w, K, kind=esi.SRC_POINT)
        plan.gradient(esi.GRAD_SEED_REUSE, w, seed, kind=esi.SRC_POINT, grad_m=grad, ckpt_every=K)

    one()                                                           # warm-up
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    one()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    plan.close()
    npad = (cfg.nz + 2 * cfg.nb) * (cfg.ny + 2 * cfg.nb) * (cfg.nx + 2 * cfg.nb)
    nphys = cfg.nz * cfg.ny * cfg.nx
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    per_us = rec["ms"] / rec["launches"] * 1e3
    spl = rec["shot_launches"] / rec["launches"]
    alg = bytes_per_shot_launch(rec["flags"], npad, nphys) * spl
    two = bool(rec["flags"] & TWO_STEP)
    traffic = measured_traffic(rec["flags"], spl, TRAFFIC_FILE_3D, KERNEL_SOURCES_3D, ndim=3)
    kern = ("k_step3d_t2" if two else "k_step3d") + f"<{name}>"
    if not two and rec["flags"] & CORR:   # one-step correlating launches run in pairs
        kern += " paired with k_step3d<INJ>"
    return {"workload": f"diff3d-{cfg.nx}x{cfg.ny}x{cfg.nz}-{cfg.nshots}shots", "nt": cfg.nt,
            "checkpoint_every": K, "propagations": 3, "seconds": round(wall, 3),
            "launch_shape": tune_report(esi, tuned, table, esi.LAUNCH_NAMES_3D),
            "gpts_per_s": round(3 * cfg.nshots * npad * cfg.nt / wall / 1e9, 1),
            "dominant_loop": {"variant": name, "launches": rec["launches"], "ms": round(rec["ms"], 1)},
            "roofline": roofline(kern, alg, per_us, traffic, peak_measured),
            "kernel_loops": {k: {"launches": v["launches"], "ms": round(v["ms"], 1)} for k, v in prof.items()}}


def forward3d_run(args, torch, dev):
    """The 3D forward modelling of the differentiation workload (256^3, 8
    shots at once, point sources, 128 x 128 receivers) over its first
    args.nt3d steps: wall time of the pass, and the step kernel's average
    launch time from the live profile against its algorithmic bytes."""
    from paper_2211_06300_amd import esi, inputs
    cfg = inputs.cfg_diff3d(n=256, nt=args.nt3d)
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(dev))
    w = torch.from_numpy(np.stack([cfg.wavelet] * cfg.nshots)).to(dev)
    plan.forward(w, esi.SRC_POINT)                                  # warm-up
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    plan.forward(w, esi.SRC_POINT)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    plan.close()
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    per_us = rec["ms"] / rec["launches"] * 1e3
    npad = (cfg.nz + 2 * cfg.nb) * (cfg.ny + 2 * cfg.nb) * (cfg.nx + 2 * cfg.nb)
    alg = bytes_per_shot_launch(rec["flags"], npad, cfg.nz * cfg.ny * cfg.nx) * cfg.nshots
    return {"workload": f"forward-3d-{cfg.nx}x{cfg.ny}x{cfg.nz}-{cfg.nshots}shots", "nt": cfg.nt,
            "seconds": round(wall, 4), "gpts_per_s": round(cfg.nshots * npad * cfg.nt / wall / 1e9, 1),
            "kernel": f"k_step3d<{name}>", "avg_launch_us": round(per_us, 1),
            "alg_bytes_per_launch": int(alg), "alg_gbs": round(alg / per_us / 1e3, 1),
            "frac": round(alg / per_us / 1e3 / HBM_PEAK_GBS, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shots", type=int, default=32)
    ap.add_argument("--group", type=int, default=16)
    ap.add_argument("--cg-iters", type=int, default=20)
    ap.add_argument("--nt", type=int, default=2000)
    ap.add_argument("--cpu-nt", type=int, default=1000, help="steps in the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-rfuse", action="store_true",
                    help="CG with the residual update as a separate pass (default: fused into the adjoint)")
    ap.add_argument("--no-solve", action="store_true", help="skip the plain vs learned CG comparison")
    ap.add_argument("--solve-seeds", default="6000,6001,6002,6003,6004",
                    help="held-out 801 x 401 models of the solver comparison")
    ap.add_argument("--solve-shots", type=int, default=4)
    ap.add_argument("--solve-iters", type=int, default=500)
    ap.add_argument("--plain-iters", type=int, default=200, help="iteration cap of plain CG in the comparison")
    ap.add_argument("--no-batching", action="store_true", help="skip the uneven-aperture batching run")
    ap.add_argument("--batch-shots", type=int, default=128)
    ap.add_argument("--batch-nt", type=int, default=4000)
    ap.add_argument("--no-wri", action="store_true", help="skip the WRI run on the single-solve workload")
    ap.add_argument("--no-invert", action="store_true", help="skip the outer-loop (Algorithm 2) run")
    ap.add_argument("--no-dtft", action="store_true", help="skip the DTFT-variant run")
    ap.add_argument("--no-dataspace", action="store_true", help="skip the data-space solver run")
    ap.add_argument("--dtft-nf", type=int, default=8)
    ap.add_argument("--ds-ckpt", type=int, default=0,
                    help="data-space leg: checkpoint the adjoint field every K steps (0: resident)")
    ap.add_argument("--dtft-block", type=int, default=-1,
                    help="DTFT steps per block (0: slices met at every step; default: the library's 64)")
    ap.add_argument("--invert-iters", type=int, default=2)
    ap.add_argument("--invert-cg", type=int, default=30)
    ap.add_argument("--invert-beta", type=float, default=100.0)
    ap.add_argument("--invert-inner", choices=["fcg", "ds", "cg"], default="fcg")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="also run one elementwise copy of this many MiB (counter calibration)")
    ap.add_argument("--all-shapes", action="store_true",
                    help="counter runs: run the legs with every launch shape (main leg: step i with shape i % 4) "
                         "instead of the autotuner's choice")
    ap.add_argument("--nt3d", type=int, default=1500, help="steps of the 3D differentiation leg")
    ap.add_argument("--no-diff3d", action="store_true", help="skip the 3D differentiation run")
    ap.add_argument("--only-3d", action="store_true",
                    help="run the 3D forward modelling alone (--nt3d steps) and print its JSON object")
    ap.add_argument("--only", default="", metavar="LEGS",
                    help="comma list of legs to run alone (batching, diff3d, solve, network, wri, invert, "
                         "dtft, dataspace); prints one JSON object of them, not the contract line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1 "
                                   "(a multi-GPU run would give each GPU its own group of shots)"}))
        sys.exit(2)

    import torch
    from paper_2211_06300_amd import esi, inputs

    dev = torch.device("cuda:0")
    if args.copy_calib:
        # reference kernel of known traffic: reads and writes copy_calib MiB each
        a = torch.ones(args.copy_calib * 262144, dtype=torch.float32, device=dev)
        b = torch.mul(a, 1.0)
        torch.cuda.synchronize()
        del a, b
    if args.only_3d:
        print(json.dumps({"forward3d": forward3d_run(args, torch, dev)}), flush=True)
        return
    # (a counter-calibration run keeps its copy kernel the only one of its kind)
    peak_measured = None if args.copy_calib else copy_bandwidth(torch, dev)
    if peak_measured:
        log(f"measured copy bandwidth: {peak_measured:.0f} GB/s")
    legs = {"batching": lambda: batching_run(args, torch, dev, peak_measured),
            "diff3d": lambda: diff3d_run(args, torch, dev, peak_measured),
            "solve": lambda: solver_comparison(args, torch, dev),
            "network": lambda: network_forward_run(args, torch, dev),
            "wri": lambda: wri_run(args, torch, dev),
            "invert": lambda: invert_run(args, torch, dev),
            "dtft": lambda: dtft_run(args, torch, dev),
            "dataspace": lambda: dataspace_run(args, torch, dev)}
    if args.only:
        res = {"peak_measured_gbs": peak_measured and round(peak_measured, 1)}
        for leg in args.only.split(","):
            res[leg] = legs[leg]()
            torch.cuda.empty_cache()
        print(json.dumps(res), flush=True)
        return
    cfg = inputs.cfg_single_solve(nshots=args.shots, nt=args.nt)
    npad = (cfg.nz + 2 * cfg.nb) * (cfg.nx + 2 * cfg.nb)
    nphys = cfg.nz * cfg.nx
    G = min(args.group, cfg.nshots)
    groups = [(s, min(G, cfg.nshots - s)) for s in range(0, cfg.nshots, G)]
    log(f"workload {cfg.name}: {cfg.nshots} shots, groups of {G}, nt {cfg.nt}, "
        f"{args.cg_iters} CG iterations")

    # observed data from the true model (setup, untimed)
    plan_true = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_true).to(dev))
    wav = torch.from_numpy(np.tile(cfg.wavelet, (cfg.nshots, 1))).to(dev)
    d_obs = plan_true.forward(wav, esi.SRC_POINT)
    torch.cuda.synchronize()
    plan_true.close()
    del plan_true, wav
    plan = esi.Plan.from_config(cfg, vel=torch.from_numpy(cfg.v_start).to(dev))
    plan.set_cg_rfuse(not args.no_rfuse)
    x = plan.new_vec(G)
    work = torch.empty((3, *plan.vec_shape(G)), dtype=torch.float32, device=dev)
    grad = torch.zeros(plan.phys_shape, dtype=torch.float32, device=dev)
    offs = [int(cfg.nt * cfg.rec_ptr[s]) for s in range(cfg.nshots + 1)]
    tuned = plan.autotune(nshots=G, p=work[0], Ap=work[1]) if not args.all_shapes else (2, 2)
    tune_table = plan.tune_table()
    log(f"autotuned launch shapes: forward {esi.LAUNCH_NAMES[tuned[0]]}, adjoint {esi.LAUNCH_NAMES[tuned[1]]}")
    log("setup done")

    last_hist = {}

    def step():
        grad.zero_()
        for s0, ns in groups:
            d = d_obs[offs[s0]:offs[s0 + ns]]
            xs = x[:ns]
            ws = work[:, :ns] if ns == G else torch.empty((3, *plan.vec_shape(ns)),
                                                          dtype=torch.float32, device=dev)
            _, rep = plan.cg_solve(d, args.cg_iters, 0.0, shot0=s0, nshots=ns, x=xs, work=ws)
            plan.gradient(esi.GRAD_PENALTY, xs, shot0=s0, nshots=ns, grad_m=grad)
            last_hist[s0] = rep["res_hist"]

    for i in range(args.warmup):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t0:.2f} s")

    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        if args.all_shapes:   # counter runs: step i with launch shape i % 4
            plan.set_launch_shape((1, 3, 2, 4)[i % 4], (1, 3, 2, 4)[i % 4])
        step()
        log(f"step {i} queued/done")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    prof = plan.profile_read()
    plan.profile(False)

    props_per_shot = 1 + 2 * args.cg_iters + 1
    pts = args.steps * cfg.nshots * props_per_shot * npad * cfg.nt
    value = pts / wall / 1e9

    # dominant time-step kernel variant: largest share of the timed loops
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    per_launch_ms = rec["ms"] / rec["launches"]
    shots_per_launch = rec["shot_launches"] / rec["launches"]
    alg_bytes = bytes_per_shot_launch(rec["flags"], npad, nphys) * shots_per_launch
    traffic = measured_traffic(rec["flags"], shots_per_launch)
    hist = np.concatenate([h for h in last_hist.values()])
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "grid": f"{cfg.nx}x{cfg.nz}", "nb": cfg.nb,
                   "nt": cfg.nt, "shots": cfg.nshots, "shot_group": G,
                   "cg_iters": args.cg_iters, "beta": cfg.beta,
                   "cg_residual_update": "separate pass" if args.no_rfuse else "fused into the adjoint",
                   "propagations_per_shot": props_per_shot,
                   "launch_shape": tune_report(esi, tuned, tune_table)},
        "roofline": roofline(("k_step2d_t2" if rec["flags"] & TWO_STEP else "k_step2d") + f"<{name}>",
                             alg_bytes, per_launch_ms * 1e3, traffic, peak_measured),
        "gpu_event_ms": round(gpu_ms, 1),
        "cg_final_rel_residual_max": float(np.max(hist[:, -1])),
        "kernel_loops": {k: {"launches": v["launches"], "ms": round(v["ms"], 1)} for k, v in prof.items()},
    }
    plan.close()
    del plan, x, work, d_obs
    torch.cuda.empty_cache()
    if not args.no_solve:
        out["solve_to_1e-3"] = solver_comparison(args, torch, dev)
        torch.cuda.empty_cache()
    if not args.no_batching:
        out["batching"] = batching_run(args, torch, dev, peak_measured)
        torch.cuda.empty_cache()
    if not args.no_diff3d:
        out["diff3d"] = diff3d_run(args, torch, dev, peak_measured)
        torch.cuda.empty_cache()
    if not args.no_wri:
        out["wri"] = wri_run(args, torch, dev)
        torch.cuda.empty_cache()
    if not args.no_invert:
        out["invert"] = invert_run(args, torch, dev)
        torch.cuda.empty_cache()
    if not args.no_dtft:
        out["dtft"] = dtft_run(args, torch, dev)
        torch.cuda.empty_cache()
    if not args.no_dataspace:
        out["dataspace"] = dataspace_run(args, torch, dev)
        torch.cuda.empty_cache()
    if not args.no_cpu:
        log("timing the oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_nt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
