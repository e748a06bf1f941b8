"""Train the preconditioner network on the GPU and write its parameters.

    python -m paper_2211_06300_amd.train_precond --models 40 --epochs 8 --out DIR

Training models: seeds 5000, 5001, ... of inputs.cfg_precond at 401 x 201
(4 shots, 1500 steps) and, with --large-models, seeds 5100, 5101, ... at
801 x 401 (4 shots, 2000 steps) cut into 208 x 408 tiles.  Writes
DIR/precond_unet.npy (float32 parameters) and DIR/precond_unet.json
(settings and loss history).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--models", type=int, default=40)
    ap.add_argument("--first-seed", type=int, default=5000)
    ap.add_argument("--large-models", type=int, default=0)
    ap.add_argument("--first-large-seed", type=int, default=5100)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--clip", type=float, default=1.0)
    ap.add_argument("--nt", type=int, default=1500)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-seeds", type=str, default="6000",
                    help="held-out 401 x 201 models compared after training (comma list, empty: none)")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    import torch
    from . import precond

    def log(msg):
        print(f"[train {time.strftime('%H:%M:%S')}] {msg}", flush=True)

    t0 = time.time()
    seeds = list(range(a.first_seed, a.first_seed + a.models))
    X, A, C, Wt = precond.build_dataset(seeds, nt=a.nt, log=log)
    large = list(range(a.first_large_seed, a.first_large_seed + a.large_models))
    if large:
        XL, AL, CL, WL = precond.build_dataset(large, nx=801, nz=401, nt=2000, log=log)
        X, A, C, Wt = torch.cat([X, XL]), torch.cat([A, AL]), torch.cat([C, CL]), torch.cat([Wt, WL])
        del XL, AL, CL, WL
    log(f"dataset: {X.shape[0]} samples of {X.shape[2]} x {X.shape[3]} in {time.time() - t0:.0f} s; "
        f"per-cell optimum loss {precond.cell_optimum_loss(A, C, Wt):.3f} (best single scale: -1)")
    theta, hist = precond.train(X, A, C, Wt, epochs=a.epochs, batch=a.batch, lr=a.lr, clip=a.clip, seed=a.seed,
                                log=log)
    os.makedirs(a.out, exist_ok=True)
    np.save(os.path.join(a.out, "precond_unet.npy"), theta.cpu().numpy().astype(np.float32))
    meta = {"models": seeds, "nt": a.nt, "grid": "401x201", "shots_per_model": 4,
            "large_models": large, "large_grid": "801x401", "large_nt": 2000, "tile": "408x208",
            "samples": int(X.shape[0]), "epochs": a.epochs, "batch": a.batch, "lr": a.lr, "clip": a.clip,
            "seed": a.seed, "history": hist, "cell_optimum_loss": precond.cell_optimum_loss(A, C, Wt),
            "seconds": time.time() - t0,
            "command": "python -m paper_2211_06300_amd.train_precond " + " ".join(argv or sys.argv[1:])}
    with open(os.path.join(a.out, "precond_unet.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    evals = {}
    for sd in [int(x) for x in a.eval_seeds.split(",") if x]:
        cfg = precond.inputs.cfg_precond(sd, nt=a.nt)
        evals[sd] = precond.compare_solvers(cfg, theta, log=log)
    meta["eval"] = evals
    with open(os.path.join(a.out, "precond_unet.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    log(f"done in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
