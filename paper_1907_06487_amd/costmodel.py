"""Learned cost model: traces, training on the device, schedule choice.

The engine measures itself: a traced product (race_symm_spmm_traced) stamps
every unit with the device wall clock when it was taken, computed, released
by its conflict edges and flushed.  A unit's cost is compute + flush time;
the network (12 -> 64 -> 64 -> 1, ReLU, float32; race_mlp_* kernels) learns
ln(cost in microseconds) from the unit's 12 features.

The trained network then
  * supplies the loads of the tree builder (balance="model": learned cost
    instead of the nonzero count of Sections 4.3-4.4), and
  * picks the efficiency parameters eps_0, eps_1, the recursion depth and
    N_t (Section 5 tunes these by hand) by the predicted makespan of each
    candidate schedule (race_schedule_simulate).
The nonzero heuristic is the fallback and the yardstick: the same candidates
scored with unit cost = stored entries give the choice the method makes
without the network.

Everything numeric runs in the library: features, makespan and learned
loads on the host (C++), inference and training in the gfx950 kernels.
Torch only holds device memory and shuffles minibatch indices.
"""
from __future__ import annotations

import json
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import Schedule, _lib

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "cost_model.npy")
META_PATH = os.path.join(HERE, "cost_model.json")
N_IN, N_HID, N_PARAMS = _lib.MLP_INPUTS, _lib.MLP_HIDDEN, _lib.MLP_PARAMS


# --- measurements -------------------------------------------------------------

def traced_unit_costs(s, k=1, reps=3, device="cuda:0", seed=0):
    """Median over `reps` traced products of each unit's compute and flush
    time (microseconds), units in execution order."""
    st = s.stats()
    nu, hz = st["n_units"], st["wall_clock_hz"]
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    shape = (st["n"], k) if k > 1 else (st["n"],)
    x = torch.rand(shape, dtype=torch.float64, device=device, generator=g) * 2 - 1
    y = torch.empty_like(x)
    tr = torch.zeros(4 * nu, dtype=torch.int64, device=device)
    (s.spmm if k > 1 else s.spmv)(x, y)  # warm caches and code
    comp, flush = [], []
    for _ in range(reps):
        s.traced(x, y, tr)
        torch.cuda.synchronize()
        t = tr.cpu().numpy().reshape(nu, 4).astype(np.float64)
        comp.append((t[:, 1] - t[:, 0]) * 1e6 / hz)
        flush.append((t[:, 3] - t[:, 2]) * 1e6 / hz)
    s.check()
    return np.median(comp, axis=0), np.median(flush, axis=0)


def collect(mats, configs, log=None, device="cuda:0"):
    """Traced unit costs for every (matrix, configuration).  configs[i] is a
    list of (k, Schedule keyword dict) for mats[i].  Returns features X,
    targets t = ln(compute + flush), the flush fractions and a group id per
    sample (the schedule it came from)."""
    X, t, frac, group = [], [], [], []
    gid = 0
    for i, (m, cfgs) in enumerate(zip(mats, configs)):
        for k, kw in cfgs:
            s = Schedule(m.n, m.row_ptr, m.col, m.val, **kw)
            try:
                c, f = traced_unit_costs(s, k, device=device, seed=i)
                X.append(s.features(k))
            finally:
                s.close()
            tot = np.maximum(c + f, 1e-3)
            t.append(np.log(tot))
            frac.append(f / tot)
            group.append(np.full(tot.size, gid))
            gid += 1
        if log and (i % 20 == 19 or i == len(mats) - 1):
            log(f"traced {i + 1}/{len(mats)} matrices, {sum(a.size for a in t)} units")
    return {"X": np.concatenate(X).astype(np.float32), "t": np.concatenate(t).astype(np.float32),
            "flush_frac": np.concatenate(frac), "group": np.concatenate(group)}


# --- training -----------------------------------------------------------------

def init_params(seed):
    """He initialisation, flat in the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, math.sqrt(2.0 / N_IN), N_HID * N_IN), np.zeros(N_HID),
             rng.normal(0, math.sqrt(2.0 / N_HID), N_HID * N_HID), np.zeros(N_HID),
             rng.normal(0, math.sqrt(1.0 / N_HID), N_HID), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def fold_normalisation(theta, mu, sd):
    """Network on standardised inputs -> the same network on raw inputs:
    W1' = W1 / sd (per input), b1' = b1 - W1' mu."""
    th = theta.astype(np.float64).copy()
    W1 = th[:N_HID * N_IN].reshape(N_HID, N_IN) / sd
    b1 = th[N_HID * N_IN:N_HID * N_IN + N_HID] - W1 @ mu
    th[:N_HID * N_IN] = W1.ravel()
    th[N_HID * N_IN:N_HID * N_IN + N_HID] = b1
    return th.astype(np.float32)


def train(X, t, group, epochs=80, batch=1024, lr=2e-3, val_frac=0.15, seed=0, device="cuda:0", log=None):
    """Adam on the mean squared error of ln(cost), on the device kernels.
    Validation holds out whole schedules (groups).  Returns (theta on raw
    features, history)."""
    rng = np.random.default_rng(seed)
    groups = np.unique(group)
    val_groups = set(rng.choice(groups, size=max(1, int(round(val_frac * groups.size))), replace=False).tolist())
    is_val = np.array([g in val_groups for g in group])
    mu = X[~is_val].astype(np.float64).mean(axis=0)
    sd = X[~is_val].astype(np.float64).std(axis=0)
    sd[sd < 1e-6] = 1.0
    Xn = ((X - mu) / sd).astype(np.float32)
    Xtr = torch.as_tensor(Xn[~is_val], device=device)
    ttr = torch.as_tensor(t[~is_val], device=device)
    Xva = torch.as_tensor(Xn[is_val], device=device)
    tva = torch.as_tensor(t[is_val], device=device)
    n = Xtr.shape[0]
    th = torch.as_tensor(init_params(seed), device=device)
    m = torch.zeros(N_PARAMS, dtype=torch.float32, device=device)
    v = torch.zeros_like(m)
    g = torch.empty_like(m)
    loss = torch.empty(1, dtype=torch.float32, device=device)
    ws = torch.empty(_lib.race_mlp_workspace(max(batch, n, Xva.shape[0])), dtype=torch.float32, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)

    def full_loss(Xs, ts):
        _lib.race_mlp_loss_grad(th, Xs, ts, ws, g, loss)
        torch.cuda.synchronize()
        return float(loss.item())

    hist = {"train": [], "val": []}
    step = 0
    best = (float("inf"), None)
    for ep in range(epochs):
        order = torch.randperm(n, device=device, generator=gen)
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / epochs))  # cosine decay
        for b in range(0, n, batch):
            idx = order[b:b + batch]
            step += 1
            _lib.race_mlp_loss_grad(th, Xtr[idx].contiguous(), ttr[idx].contiguous(), ws, g, loss)
            _lib.race_mlp_adam(th, g, m, v, step, lr_ep)
        tr_l, va_l = full_loss(Xtr, ttr), full_loss(Xva, tva)
        hist["train"].append(tr_l)
        hist["val"].append(va_l)
        if va_l < best[0]:
            best = (va_l, th.cpu().numpy().copy())
        if log and (ep % 10 == 9 or ep == epochs - 1):
            log(f"epoch {ep + 1}: train mse {tr_l:.4f}, validation mse {va_l:.4f} (ln-cost units)")
    theta = fold_normalisation(best[1], mu, sd)
    hist.update({"best_val_mse": best[0], "n_train": int(n), "n_val": int(Xva.shape[0]), "steps": step})
    return theta, hist


def save(theta, meta, path=MODEL_PATH, meta_path=META_PATH):
    np.save(path, np.asarray(theta, dtype=np.float32), allow_pickle=False)
    with open(meta_path, "w") as fh:
        json.dump(meta, fh, indent=1, sort_keys=True)


def load(path=MODEL_PATH, meta_path=META_PATH):
    theta = np.load(path, allow_pickle=False).astype(np.float32)
    if theta.size != N_PARAMS:
        raise ValueError(f"{path}: {theta.size} parameters, expected {N_PARAMS}")
    with open(meta_path) as fh:
        meta = json.load(fh)
    return theta, meta


# --- inference and choice -------------------------------------------------------

def predict_costs(theta, feats, device="cuda:0"):
    """Predicted unit costs in microseconds (device inference kernel)."""
    th = torch.as_tensor(np.ascontiguousarray(theta, dtype=np.float32), device=device)
    X = torch.as_tensor(np.ascontiguousarray(feats, dtype=np.float32), device=device)
    y = torch.empty(X.shape[0], dtype=torch.float32, device=device)
    _lib.race_mlp_forward(th, X, y)
    torch.cuda.synchronize()
    return np.exp(np.minimum(y.cpu().numpy().astype(np.float64), 30.0))


def candidate_grid(n_workers=(128, 256, 512, 1024), eps=((0.8, 0.8), (0.6, 0.6)), stages=(2, 4)):
    return [dict(n_workers=nt, eps=e, max_stages=d) for nt in n_workers for e in eps for d in stages]


def choose(m, theta, meta, grid=None, k=1, block=512, window=3840, threads=8, device="cuda:0", log=None):
    """Score every candidate (nonzero loads and learned loads) by predicted
    makespan.  Returns the candidates with both predictions and the two
    choices: 'heuristic' (nonzero loads, scored by stored entries) and
    'learned' (any loads, scored by the network's unit costs in the
    dataflow simulation).  The simulation has no model of bandwidth shared
    between concurrent units: the network learns each unit's cost as it
    was measured among its neighbours, and the predicted makespans read
    30-40% below the measured times on large matrices."""
    grid = grid or candidate_grid()
    cands = []
    for c in grid:
        for bal in ("nnz", "model"):
            kw = dict(c, block_threads=block, window_max=window, balance=bal)
            if bal == "model":
                kw["cost_model"] = theta
            cands.append(kw)

    def build(kw):
        return Schedule(m.n, m.row_ptr, m.col, None, upload=False, **kw)

    frac = float(meta["flush_frac"])
    out = []
    # builds in parallel, a chunk at a time (large schedules hold GBs of host memory)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for c0 in range(0, len(cands), threads):
            chunk = cands[c0:c0 + threads]
            for kw, s in zip(chunk, ex.map(build, chunk)):
                try:
                    f = s.features(k)
                    workers = s.flow_grid(k)
                    learned = predict_costs(theta, f, device)
                    nnz = np.exp2(f[:, 1].astype(np.float64)) - 1.0
                    st = s.stats()
                    out.append({"params": {key: val for key, val in kw.items() if key != "cost_model"},
                                "pred_us": s.simulate(learned, frac, workers),
                                "pred_nnz": s.simulate(nnz, frac, workers),
                                "units": st["n_units"], "eta": st["eta"], "workers": workers})
                finally:
                    s.close()
    heur = min((c for c in out if c["params"]["balance"] == "nnz"), key=lambda c: c["pred_nnz"])
    lrn = min(out, key=lambda c: c["pred_us"])
    if log:
        log(f"choice: heuristic {heur['params']} (pred {heur['pred_us']:.1f} us); "
            f"learned {lrn['params']} (pred {lrn['pred_us']:.1f} us)")
    return {"candidates": out, "heuristic": heur, "learned": lrn}
