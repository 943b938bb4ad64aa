"""Train the learned cost model on the current GPU and save it.

    python -m paper_1907_06487_amd.train_cost_model [--out DIR] [--matrices 200]

Training set: the uneven-batch family (2D 5-point, 3D 27-point and
irregular banded matrices of 10^4 to 5*10^5 rows, seeds 1000 upwards) plus
a few larger members of the same families (seeds 1200 upwards) so that
unit counts of multi-million-row matrices are covered.  Every matrix is
scheduled under two configurations drawn from a grid of N_t, eps, recursion
depth and right-hand-side count, and every unit of a traced product is one
sample.  Held-out evaluation is left to the caller (the 160^3 stencil is
never part of this set).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def training_matrices(count, first_seed=1000):
    import matgen
    mats = [matgen.batch_family(i, first_seed + i) for i in range(count)]
    large = [matgen.stencil3d_27pt(100, seed=first_seed + 200), matgen.stencil3d_27pt(128, seed=first_seed + 201),
             matgen.stencil2d_5pt(1024, seed=first_seed + 202), matgen.stencil2d_5pt(1448, seed=first_seed + 203),
             matgen.banded_irregular(1 << 20, seed=first_seed + 204, band=1 << 16),
             matgen.stencil3d_27pt(112, seed=first_seed + 205)]
    return mats + large


def configurations(m, seed):
    """Two schedule configurations for one matrix, drawn from the grid."""
    from . import autotune
    rng = np.random.default_rng(seed)
    n = m.n
    nts = sorted({int(min(4096, max(4, n // r))) for r in (8000, 4000, 2000, 1000)})
    if n > 10 ** 6:
        nts = [128, 256, 512, 1024]
    out = []
    for _ in range(2):
        k = int(rng.choice([1, 1, 1, 4, 16]))
        kw = dict(n_workers=int(rng.choice(nts)), eps=[(0.8, 0.8), (0.6, 0.6), (0.9, 0.9)][rng.integers(3)],
                  max_stages=int(rng.choice([2, 3, 4])), block_threads=512, window_max=autotune.max_window(k))
        out.append((k, kw))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="directory for cost_model.npy/.json (default: the package)")
    ap.add_argument("--matrices", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=80)
    ap.add_argument("--save-data", default=None, help="also write the samples (npz) here")
    args = ap.parse_args()

    import torch

    from . import costmodel as CM
    torch.cuda.set_device(0)
    t0 = time.time()
    mats = training_matrices(args.matrices)
    log(f"generated {len(mats)} matrices in {time.time() - t0:.1f}s")
    cfgs = [configurations(m, 7000 + i) for i, m in enumerate(mats)]
    t0 = time.time()
    data = CM.collect(mats, cfgs, log=log)
    log(f"collected {data['t'].size} unit samples in {time.time() - t0:.1f}s")
    if args.save_data:
        os.makedirs(os.path.dirname(os.path.abspath(args.save_data)), exist_ok=True)
        np.savez(args.save_data, X=data["X"], t=data["t"], flush_frac=data["flush_frac"], group=data["group"])
    t0 = time.time()
    theta, hist = CM.train(data["X"], data["t"], data["group"], epochs=args.epochs, log=log)
    log(f"trained in {time.time() - t0:.1f}s")
    # held-out schedules: error of the ln-cost prediction in the raw feature space
    pred = np.log(CM.predict_costs(theta, data["X"]))
    resid = pred - data["t"]
    meta = {
        "inputs": "12 unit features (race_schedule_features)", "target": "ln(compute + flush microseconds) of a unit",
        "flush_frac": float(np.median(data["flush_frac"])), "samples": int(data["t"].size),
        "matrices": len(mats), "first_seed": 1000, "epochs": args.epochs,
        "train_mse": hist["train"][-1], "best_validation_mse": hist["best_val_mse"],
        "n_train": hist["n_train"], "n_validation": hist["n_val"],
        "rms_ln_error_all": float(np.sqrt(np.mean(resid ** 2))),
        "device": torch.cuda.get_device_name(0),
    }
    out = args.out or os.path.dirname(CM.MODEL_PATH)
    os.makedirs(out, exist_ok=True)
    CM.save(theta, meta, os.path.join(out, "cost_model.npy"), os.path.join(out, "cost_model.json"))
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
