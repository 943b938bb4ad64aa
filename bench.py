"""RACE SymmSpMV benchmark on one MI355X.

One step = one product y = A x of the whole RACE path (every phase launch)
on the 3D 27-point stencil with a 128^3 grid (N = 2,097,152, 28,920,060
stored upper entries, float64), inputs resident in HBM.  Vectors rotate
through two ring buffers larger than the last-level caches (the paper's
measurement protocol: two rings, one vector pair per product, mean time).

Also timed the same way on the same GPU: full-matrix CRS SpMV (the
yardstick) and SymmSpMV with global float64 atomics.  The CPU baseline is
the plain serial oracle on one host core over a bounded sample.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SymmSpMV GFLOP/s + % peak HBM GB/s vs CRS SpMV, same GPU, FP64 rel err ≤1e-12"
PEAK_HBM_GBS = 8000.0
RING_BYTES = 576 << 20  # each ring >= 2 x (256 MB last-level cache + L2s)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    import matgen
    if name == "3d27pt_128":
        return matgen.config_3d_128(), "3D 27-point stencil 128^3, lexicographic, FP64, seed 2"
    if name == "2d5pt_100":
        return matgen.config_2d_small(), "2D 5-point Laplacian 100x100, FP64, seed 1"
    if name == "banded_4m":
        return matgen.config_banded_4m(), "irregular banded 2^22 rows, bandwidth 2^16, FP64, seed 3"
    if name == "3d27pt_160":
        return matgen.config_3d_160(), "3D 27-point stencil 160^3, FP64, seed 2000"
    if name == "3d27pt_128_relabel":
        return matgen.config_3d_128_relabel(), "3D 27-point stencil 128^3 under a random symmetric relabelling (seed 7)"
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash(product_path=0):
    """Hash of the sources that decide what the product kernel moves: the
    RACE kernels (path 0) or the expanded CRS kernels (path 1)."""
    import hashlib
    h = hashlib.sha256()
    kern = "race_kernels.hip" if product_path == 0 else "csr_kernels.hip"
    for f in [kern, "unit_device.hpp", "kernels.hpp", "layout.cpp", "layout.hpp", "schedule.cpp"]:
        with open(os.path.join(ROOT, "paper_1907_06487_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_ring(fn, xs, ys, steps, warmup, torch):
    """Mean milliseconds per call over `steps` calls after `warmup`, HIP
    events on the current stream (the stream the library launches on)."""
    nr = len(xs)
    for i in range(warmup):
        fn(xs[i % nr], ys[i % nr])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        fn(xs[i % nr], ys[(i + 1) % nr])
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_ring_median(fn, xs, ys, steps, torch):
    """Median milliseconds per call: an event between consecutive calls
    (a separate pass, so the mean above has no events inside it)."""
    import numpy as np
    nr = len(xs)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        fn(xs[i % nr], ys[(i + 1) % nr])
        ev[i + 1].record()
    torch.cuda.synchronize()
    return float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]))


def attainable_bandwidth(torch, gib=4, reps=10):
    """Read-only and copy bandwidth of the library's 16-byte stream kernels
    over 4 GiB arrays (larger than every cache), the best over a few grid
    sizes: what a kernel can reach on this device, the input of the paper's
    roofline bound (Table 1, Eq. upper_performance)."""
    import paper_1907_06487_amd as R
    dev = torch.device("cuda:0")
    nbytes = gib << 30
    src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).uniform_()
    dst = torch.empty_like(src)
    sink = torch.zeros(4, dtype=torch.int32, device=dev)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    res = {"bytes": nbytes, "grids": {}}
    best_r = best_c = (0.0, 0)
    for mult in (8, 16, 32, 64, 128):
        grid = cus * mult
        tr = time_ring(lambda x, y: R.race_stream_read(src, sink, grid), [0], [0], reps, 2, torch)
        tc = time_ring(lambda x, y: R.race_stream_copy(src, dst, grid), [0], [0], reps, 2, torch)
        rg, cg = nbytes / (tr * 1e-3) / 1e9, 2 * nbytes / (tc * 1e-3) / 1e9
        res["grids"][grid] = {"read_GBs": round(rg, 1), "copy_GBs": round(cg, 1)}
        best_r = max(best_r, (rg, grid))
        best_c = max(best_c, (cg, grid))
    assert torch.equal(src, dst)
    res.update(read_GBs=round(best_r[0], 1), read_grid=best_r[1], copy_GBs=round(best_c[0], 1), copy_grid=best_c[1])
    log(f"attainable bandwidth over {gib} GiB: read {best_r[0]:.0f} GB/s (grid {best_r[1]}), "
        f"copy {best_c[0]:.0f} GB/s (grid {best_c[1]})")
    del src, dst
    torch.cuda.empty_cache()
    return res


def host_cpu():
    """Model name of the host CPU and the threads this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0)), os.cpu_count()


def yardsticks(m, perm, flops, nnz_full, xs, ys, args, torch):
    """Same-GPU baselines, each in input order and in the RACE order, the
    best setting reported: CRS SpMV on the full matrix with 1..64 lanes per
    row and over row blocks of 4, 8 or 16 entries per thread (Algorithm
    "SpMV"), rocSPARSE's SpMV with each of its CSR
    algorithms on the full matrix and as its own symmetric product on the
    upper triangle, and SymmSpMV with global atomics with 1..32 lanes per
    row.  Inputs come from matgen's format conversions."""
    import matgen
    import paper_1907_06487_amd as R
    orders = {"input": m, "race": matgen.permuted(m, perm)}
    bytes_spmv = 12 * nnz_full + 20 * m.n + 4
    t_all = {"crs_spmv": [], "vendor_general": [], "vendor_symmetric": [], "atomic_symmspmv": []}
    T = lambda fn: time_ring(lambda x, y: fn(x, y), xs, ys, args.steps, args.warmup, torch)
    for oname, mo in orders.items():
        rp, c, v = matgen.full_crs(mo)
        for lpr in (1, 2, 4, 8, 16, 32, 64, -4, -8, -16):
            h = R.race_csr_create(m.n, rp, c, v, lpr)
            cfg = {"order": oname, "lanes_per_row": lpr} if lpr > 0 else {"order": oname, "row_blocks_per_thread": -lpr}
            t_all["crs_spmv"].append((T(lambda x, y: R.race_csr_spmv(h, x, y)), cfg))
            R.race_csr_destroy(h)
        for sym in (False, True):
            for alg in ("adaptive", "rowsplit", "lrb"):
                try:
                    h = (R.race_vendor_create(m.n, mo.row_ptr, mo.col, mo.val, True, alg) if sym
                         else R.race_vendor_create(m.n, rp, c, v, False, alg))
                except R.RaceError as e:
                    log(f"rocSPARSE {alg} symmetric={sym}: {e}")
                    continue
                key = "vendor_symmetric" if sym else "vendor_general"
                t_all[key].append((T(lambda x, y: R.race_vendor_spmv(h, x, y)), {"order": oname, "alg": alg}))
                R.race_vendor_destroy(h)
        del rp, c, v
        for lpr in (1, 2, 4, 8, 16, 32):
            h = R.race_atomic_create(m.n, mo.row_ptr, mo.col, mo.val, lpr)
            t_all["atomic_symmspmv"].append((T(lambda x, y: R.race_symm_spmv_atomic(h, x, y)),
                                             {"order": oname, "lanes_per_row": lpr}))
            R.race_csr_destroy(h)
    out = {}
    for key, runs in t_all.items():
        for t, cfg in runs:
            log(f"{key} {cfg}: {t * 1e3:.2f} us")
        if not runs:
            continue
        t, cfg = min(runs, key=lambda r: r[0])
        b = bytes_spmv if key in ("crs_spmv", "vendor_general") else 12 * m.nnz + 20 * m.n + 4
        out[key] = {"us": t * 1e3, **cfg, "gflops": flops / (t * 1e-3) / 1e9,
                    "algorithmic_GBs": b / (t * 1e-3) / 1e9, "settings_timed": len(runs)}
    return out


def unit_trace(s, st, xs, ys, reps, torch):
    """Per-unit device timestamps of `reps` traced products (race_symm_spmm_traced:
    start, end of the arithmetic, end of the conflict-edge waits, end of the
    flush, on the device's wall clock) summarised: the span of a product,
    what an average unit spends in each part, how many workgroups hold a
    unit over time, and the drain after the last unit starts."""
    import numpy as np
    nu = st["n_units"]
    tr = torch.zeros(4 * nu, dtype=torch.int64, device=xs[0].device)
    spans, parts, timelines, drains, idle = [], [], [], [], []
    grid = s.flow_grid(1)
    for rep in range(reps):
        s.traced(xs[rep % len(xs)], ys[rep % len(ys)], tr)
        torch.cuda.synchronize()
        t = tr.cpu().numpy().reshape(nu, 4).astype(np.float64) * 1e6 / float(st["wall_clock_hz"])
        t -= t[:, 0].min()
        span = float(t[:, 3].max())
        spans.append(span)
        parts.append([float(np.mean(t[:, 1] - t[:, 0])), float(np.mean(t[:, 2] - t[:, 1])),
                      float(np.mean(t[:, 3] - t[:, 2]))])
        drains.append(span - float(t[:, 0].max()))
        idle.append(1.0 - float(np.sum(t[:, 3] - t[:, 0])) / (grid * span))
        edges = np.arange(0.0, span + 5.0, 5.0)
        timelines.append([int(np.sum((t[:, 0] <= b) & (t[:, 3] > b))) for b in edges])
    s.check()
    k = int(np.argsort(spans)[len(spans) // 2])  # the median product
    out = {"reps": reps, "workgroups": grid, "units": nu, "span_us_median": round(float(np.median(spans)), 2),
           "unit_us_mean": {"compute": round(parts[k][0], 2), "wait": round(parts[k][1], 2),
                            "flush": round(parts[k][2], 2)},
           "drain_after_last_start_us": round(drains[k], 2), "idle_workgroup_time": round(idle[k], 3),
           "units_in_flight_every_5us": timelines[k]}
    log(f"unit trace ({reps} traced products, median span {out['span_us_median']} us on {grid} workgroups): "
        f"a unit computes {parts[k][0]:.1f} us, waits {parts[k][1]:.1f} us, flushes {parts[k][2]:.1f} us; "
        f"drain after the last start {drains[k]:.1f} us; workgroups idle {idle[k] * 100:.1f}% of the span; "
        f"units in flight every 5 us: {timelines[k]}")
    return out


def cpu_baseline(m, budget_s):
    """The serial C oracle on one host core, the process pinned to that
    core while it runs: mean and median seconds per product."""
    import numpy as np

    import matgen
    from oracle import build as ob
    from oracle import symmspmv as O
    ob.build(force=False)
    x = matgen.rhs(m.n, 99)
    y = np.empty(m.n)
    allowed = os.sched_getaffinity(0)
    core = min(allowed)
    os.sched_setaffinity(0, {core})
    try:
        O.symm_spmv_c(m.n, m.row_ptr, m.col, m.val, x, y)  # warm
        times = []
        t0 = time.perf_counter()
        while True:
            t1 = time.perf_counter()
            O.symm_spmv_c(m.n, m.row_ptr, m.col, m.val, x, y)
            times.append(time.perf_counter() - t1)
            if time.perf_counter() - t0 >= budget_s:
                break
    finally:
        os.sched_setaffinity(0, allowed)
    return float(np.mean(times)), float(np.median(times)), len(times), core


def run_batch(args, k, torch):
    """64 seeded matrices of uneven size (2D 5-pt / 3D 27-pt / irregular
    banded, 1e4..5e5 rows) with k right-hand sides: one hipGraph replay of the
    persistent batch launch with autotuned shapes, against 64 separate
    product launches with the library's default shapes."""
    import numpy as np

    import matgen
    import paper_1907_06487_amd as R
    from paper_1907_06487_amd import autotune
    from oracle import symmspmv as O

    t0 = time.perf_counter()
    mats = matgen.config_batch(64, 100)
    log(f"batch64 k={k}: generated {len(mats)} matrices, {sum(m.n for m in mats)} rows, "
        f"{sum(m.nnz for m in mats)} stored entries in {time.perf_counter() - t0:.1f}s")
    dev = "cuda:0"
    shape = lambda m: (m.n, k) if k > 1 else (m.n,)
    xs = [torch.rand(shape(m), dtype=torch.float64, device=dev) * 2 - 1 for m in mats]
    ys = [torch.empty_like(x) for x in xs]
    # plain: library defaults (column tiles as the default window needs), one call per matrix
    plain = [R.Schedule(m.n, m.row_ptr, m.col, m.val) for m in mats]
    stats = [s.stats() for s in plain]
    flops = sum(2 * st["nnz_full"] * k for st in stats)
    bytes_min = sum(12 * m.nnz + 4 * (m.n + 1) + 16 * m.n * k for m in mats)

    def run_plain():
        for s, x, y in zip(plain, xs, ys):
            if k > 1:
                s.spmm(x, y)
            else:
                s.spmv(x, y)

    ms_plain = time_ring(lambda x, y: run_plain(), [0], [0], args.steps, args.warmup, torch)
    t0 = time.perf_counter()
    scheds, batch, chosen = autotune.tune_batch(mats, k, log=log, low_locality=args.low_locality)
    t_tune = time.perf_counter() - t0
    batch.bind(xs, ys)
    ms_graph = time_ring(lambda x, y: batch.run(use_graph=True), [0], [0], args.steps, args.warmup, torch)
    ms_direct = time_ring(lambda x, y: batch.run(use_graph=False), [0], [0], args.steps, args.warmup, torch)
    batch.check()
    n_expanded = sum(1 for sc in scheds if sc.stats()["product_path"] == 1)

    def run_tuned():
        for sc, x, y in zip(scheds, xs, ys):
            if k > 1:
                sc.spmm(x, y)
            else:
                sc.spmv(x, y)

    ms_tuned = time_ring(lambda x, y: run_tuned(), [0], [0], args.steps, args.warmup, torch)
    # error of every matrix against the oracle (permuted order)
    batch.run(use_graph=True)
    torch.cuda.synchronize()
    worst = 0.0
    for m, s, x, y in zip(mats, scheds, xs, ys):
        perm = s.perm()
        xh = x.cpu().numpy()
        xo = np.empty_like(xh)
        xo[perm] = xh
        y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, xo)[perm]
        worst = max(worst, O.errors(y.cpu().numpy(), y_ref)[0])
    log(f"batch64 k={k}: graph {ms_graph * 1e3:.1f} us, direct {ms_direct * 1e3:.1f} us, 64 separate {ms_plain * 1e3:.1f} us "
        f"(library defaults), 64 separate calls of the tuned schedules {ms_tuned * 1e3:.1f} us, {n_expanded} matrices "
        f"on the expanded CRS product, tuning {t_tune:.1f}s, worst error {worst:.2e}")
    out = {
        "metric": "batched SymmSpMM GFLOP/s, 64 matrices in one hipGraph replay", "value": round(flops / (ms_graph * 1e-3) / 1e9, 3),
        "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_graph,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch64_k{k}", "matrices": 64, "rows": sum(m.n for m in mats), "k": k,
                   "block_threads": chosen["block_threads"],
                   "n_workers": [p["n_workers"] for p in chosen["params"]],
                   "window_max": [p["window_max"] for p in chosen["params"]]},
        "roofline": {"bound": "hbm", "achieved": round(bytes_min / (ms_graph * 1e-3) / 1e9, 3), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(bytes_min / (ms_graph * 1e-3) / 1e9 / PEAK_HBM_GBS, 4), "traffic": None},
        "separate_launches": {"ms": ms_plain, "gflops": flops / (ms_plain * 1e-3) / 1e9,
                              "shapes": "library defaults, RACE kernels"},
        "separate_launches_tuned": {"ms": ms_tuned, "gflops": flops / (ms_tuned * 1e-3) / 1e9,
                                    "shapes": "the batch's own schedules"},
        "expanded_members": n_expanded, "low_locality": args.low_locality,
        "batch_direct_launch": {"ms": ms_direct},
        "speedup_vs_separate": ms_plain / ms_graph,
        "error": {"norm_worst": worst},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    batch.close()
    for s in scheds + plain:
        s.close()


def run_spmm(args, k, torch, m=None, one_pass=False):
    """SymmSpMM Y = A X with k right-hand sides (row-major n x k) on the
    workload's matrix: one JSON line per k.  Default: the bench window, in
    passes of the widest column tile that fits; one_pass: a window small
    enough for all k columns at once."""
    import numpy as np

    import paper_1907_06487_amd as R
    from paper_1907_06487_amd import autotune
    from oracle import symmspmv as O

    if m is None:
        m, desc = workload(args.workload)
    win = min(args.window, autotune.max_window(k)) if one_pass else args.window
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=args.n_workers, max_stages=args.max_stages,
                   block_threads=args.block, window_max=win, value_type=args.value_type, exec_mode=args.exec_mode,
                   shared_atomics=bool(args.shared_atomics), low_locality=args.low_locality)
    st = s.stats()
    dev = "cuda:0"
    nring = max(2, -(-RING_BYTES // (8 * m.n * k)))
    gen = torch.Generator(device=dev)
    gen.manual_seed(54321 + k)
    xs = [torch.rand((m.n, k), dtype=torch.float64, device=dev, generator=gen) * 2 - 1 for _ in range(nring)]
    ys = [torch.empty((m.n, k), dtype=torch.float64, device=dev) for _ in range(nring)]
    perm = s.perm()
    X0 = np.empty((m.n, k))
    X0[perm] = xs[0].cpu().numpy()
    s.spmm(xs[0], ys[0])
    torch.cuda.synchronize()
    Y = ys[0].cpu().numpy()
    Y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, X0)[perm]
    absax = O.abs_product(m.n, m.row_ptr, m.col, m.val, np.abs(X0))[perm]
    err = max(O.errors(Y[:, j], Y_ref[:, j], absax[:, j])[0] for j in range(k))
    ms = time_ring(lambda x, y: s.spmm(x, y), xs, ys, args.steps, args.warmup, torch)
    s.check()
    flops = 2 * st["nnz_full"] * k
    bytes_min = (8 if args.value_type == "f32" else 12) * st["nnz_upper"] + 16 * k * m.n + 4 * (m.n + 1)
    achieved = bytes_min / (ms * 1e-3) / 1e9
    tile = k
    while tile > 1 and st["max_window"] * (16 * tile + 4) > 159 * 1024:
        tile -= 1
    path = "expanded CRS SpMM" if st["product_path"] == 1 else "RACE kernels"
    log(f"SpMM k={k} ({path}): {ms * 1e3:.2f} us/product, {flops / (ms * 1e-3) / 1e9:.1f} GFLOP/s, {achieved:.1f} GB/s "
        f"algorithmic, window {win}, passes of {tile} columns, worst column error {err:.2e}")
    out = {
        "metric": f"SymmSpMM GFLOP/s, {k} right-hand sides", "value": round(flops / (ms * 1e-3) / 1e9, 3),
        "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "k": k, "n_workers": args.n_workers, "block_threads": args.block,
                   "window_max": win, "rhs_tile": tile, "units": st["n_units"], "product_path": path,
                   "low_locality": args.low_locality},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "bytes_per_step": bytes_min},
        "error": {"norm_worst_column": err}, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    s.close()


def run_learned_ab(args, torch):
    """Held-out A/B of the learned cost model on the 3D 27-point 160^3
    stencil: the schedule the nonzero heuristic picks against the one the
    network picks (same candidate grid, same makespan simulation, different
    unit costs), plus the default parameters; each timed over several rounds
    of ring-buffered products."""
    import numpy as np

    import matgen
    import paper_1907_06487_amd as R
    from paper_1907_06487_amd import costmodel as CM
    from oracle import symmspmv as O

    mdir = args.model_dir or os.path.dirname(CM.MODEL_PATH)
    theta, meta = CM.load(os.path.join(mdir, "cost_model.npy"), os.path.join(mdir, "cost_model.json"))
    t0 = time.perf_counter()
    m = matgen.config_3d_160()
    log(f"learned A/B: 3d27pt_160 n={m.n} nnz_upper={m.nnz} generated in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    res = CM.choose(m, theta, meta, log=log)
    t_choose = time.perf_counter() - t0
    log(f"scored {len(res['candidates'])} candidate schedules in {t_choose:.1f}s")
    dev = "cuda:0"
    nring = max(2, -(-RING_BYTES // (8 * m.n)))
    gen = torch.Generator(device=dev)
    gen.manual_seed(4242)
    xs = [torch.rand(m.n, dtype=torch.float64, device=dev, generator=gen) * 2 - 1 for _ in range(nring)]
    ys = [torch.empty(m.n, dtype=torch.float64, device=dev) for _ in range(nring)]
    x0 = xs[0].cpu().numpy()
    # the network's best schedule with learned loads, reported on its own
    learned_loads = min((c for c in res["candidates"] if c["params"]["balance"] == "model"),
                        key=lambda c: c["pred_us"])
    arms = {"heuristic": res["heuristic"], "learned": res["learned"], "learned_loads": learned_loads,
            "default": {"params": dict(n_workers=args.n_workers, block_threads=args.block, window_max=args.window,
                                       balance="nnz"), "pred_us": None, "pred_nnz": None}}
    out_arms = {}
    for name, arm in arms.items():
        kw = dict(arm["params"])
        if kw.get("balance") == "model":
            kw["cost_model"] = theta
        t0 = time.perf_counter()
        s = R.Schedule(m.n, m.row_ptr, m.col, m.val, **kw)
        t_build = time.perf_counter() - t0
        st = s.stats()
        if arm["pred_us"] is None:
            arm["pred_us"] = s.simulate(CM.predict_costs(theta, s.features(1)), meta["flush_frac"], s.flow_grid(1))
        rounds = [time_ring(lambda x, y: s.spmv(x, y), xs, ys, args.steps, args.warmup, torch) * 1e3
                  for _ in range(args.rounds)]
        s.check()
        perm = s.perm()
        xo = np.empty(m.n)
        xo[perm] = x0
        s.spmv(xs[0], ys[0])
        torch.cuda.synchronize()
        err = O.errors(ys[0].cpu().numpy(), O.symm_spmv(m.n, m.row_ptr, m.col, m.val, xo)[perm])[0]
        out_arms[name] = {"params": {k: (list(v) if isinstance(v, tuple) else v) for k, v in arm["params"].items()},
                          "us_median": float(np.median(rounds)), "us_min": float(min(rounds)),
                          "us_max": float(max(rounds)), "pred_us": arm["pred_us"], "units": st["n_units"],
                          "eta": st["eta"], "build_s": t_build, "err_norm": err,
                          "gbs": st["bytes_min"] / (np.median(rounds) * 1e-6) / 1e9}
        log(f"{name}: {out_arms[name]['us_median']:.2f} us (min {min(rounds):.2f}, max {max(rounds):.2f}), "
            f"predicted {arm['pred_us']:.2f} us, params {arm['params']}, err {err:.2e}")
        s.close()
    h, l, d = out_arms["heuristic"], out_arms["learned"], out_arms["default"]
    flops = 2 * (2 * m.nnz - m.n)
    spread = max((a["us_max"] - a["us_min"]) / a["us_median"] for a in out_arms.values())
    without = min(h["us_median"], d["us_median"])
    log(f"learned vs the best arm without the network: {without / l['us_median']:.4f}x "
        f"(round-to-round spread up to {spread * 100:.1f}%)")
    out = {
        "metric": "learned cost model: time per SymmSpMV product, learned vs nonzero-heuristic schedule choice",
        "value": round(h["us_median"] / l["us_median"], 4), "unit": "speedup (heuristic time / learned time)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": l["us_median"] * 1e-3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3d27pt_160 (held out)", "n": m.n, "nnz_upper": m.nnz, "rounds": args.rounds,
                   "candidates": len(res["candidates"])},
        "arms": out_arms, "gflops_learned": flops / (l["us_median"] * 1e-6) / 1e9,
        "speedup_vs_default": d["us_median"] / l["us_median"],
        "speedup_vs_best_without_network": without / l["us_median"], "round_spread": spread,
        "candidates": res["candidates"], "model": meta, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_complex(args, torch):
    """Complex SymmSpMV (complex symmetric, or Hermitian with c128h) on the
    workload's pattern: values a*(1 + 0.5i) + i*N(0, 1) (seeded), one JSON
    line.  A complex multiply-add is 8 real flops; the CRS minimum moves
    20 B per stored upper entry (16 value + 4 column), 36 B per row (x read,
    y written, row pointer) and 4 more."""
    import numpy as np

    import paper_1907_06487_amd as R
    from oracle import symmspmv as O
    herm = args.value_type == "c128h"
    m, desc = workload(args.workload)
    rng = np.random.default_rng(21)
    vals = m.val * (1 + 0.5j) + 1j * rng.standard_normal(m.nnz)
    s = R.Schedule(m.n, m.row_ptr, m.col, vals, n_workers=args.n_workers, max_stages=args.max_stages,
                   block_threads=args.block, window_max=args.window, value_type=args.value_type, root=args.root,
                   level_order=args.level_order)
    st = s.stats()
    dev = torch.device("cuda:0")
    nring = max(2, -(-RING_BYTES // (16 * m.n)))
    gen = torch.Generator(device=dev)
    gen.manual_seed(4321)
    xs = [torch.complex(torch.rand(m.n, dtype=torch.float64, device=dev, generator=gen) * 2 - 1,
                        torch.rand(m.n, dtype=torch.float64, device=dev, generator=gen) * 2 - 1) for _ in range(nring)]
    ys = [torch.empty_like(xs[0]) for _ in range(nring)]
    # correctness in input order against the complex oracle
    x0 = xs[0].cpu().numpy()
    perm = s.perm()
    xo = np.empty(m.n, dtype=np.complex128)
    xo[perm] = x0
    s.spmv(xs[0], ys[0])
    torch.cuda.synchronize()
    s.check()
    ref = O.symm_spmv_complex(m.n, m.row_ptr, m.col, vals, xo, herm)[perm]
    got = ys[0].cpu().numpy()
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    ms = time_ring(lambda x, y: s.spmv(x, y), xs, ys, args.steps, args.warmup, torch)
    s.check()
    flops = 8 * st["nnz_full"]
    bytes_min = 20 * st["nnz_upper"] + 36 * m.n + 4
    achieved = bytes_min / (ms * 1e-3) / 1e9
    log(f"complex {'Hermitian' if herm else 'symmetric'} {args.workload}: {ms * 1e3:.2f} us/product, "
        f"{flops / (ms * 1e-3) / 1e9:.1f} GFLOP/s, {achieved:.1f} GB/s algorithmic, error {err:.2e}")
    out = {
        "metric": "complex SymmSpMV GFLOP/s (8 flop per complex multiply-add)",
        "value": round(flops / (ms * 1e-3) / 1e9, 3), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "hermitian": herm, "n": m.n,
                   "nnz_upper": m.nnz, "n_workers": args.n_workers, "block_threads": args.block,
                   "window_max": args.window, "units": st["n_units"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "bytes_per_step": bytes_min},
        "error": {"norm": err},
    }
    print(json.dumps(out), flush=True)
    s.close()


def run_gs(args, torch):
    """Symmetric Gauss-Seidel sweeps (forward then backward) over a
    distance-1 RACE schedule of the workload's matrix (diagonal made
    dominant): time per symmetric sweep, checked against the serial C
    oracle over the same row order.  One JSON line.  A sweep direction
    reads the off-diagonal entries of the full matrix (value + column),
    the diagonal, b and x, and writes x: 12 (nnz_full - N) + 4 (N + 1) + 32 N
    bytes in CRS."""
    import numpy as np

    import matgen
    import paper_1907_06487_amd as R
    from oracle import gauss_seidel as G
    from oracle import symmspmv as O
    m, desc = workload(args.workload)
    absrow = O.abs_product(m.n, m.row_ptr, m.col, m.val, np.ones(m.n))
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    d = rows == m.col
    v = m.val.copy()
    v[d] = 1.0 + absrow[rows[d]] - np.abs(m.val[d])
    m = matgen.UpperCSR(m.n, m.row_ptr, m.col, v, m.name + "_dominant")
    t0 = time.perf_counter()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, dist_k=1, n_workers=args.gs_workers, max_stages=args.gs_stages,
                   root=args.root, level_order=args.level_order)
    st = s.stats()
    s.set_gs_exec(args.gs_exec)
    log(f"Gauss-Seidel schedule built in {time.perf_counter() - t0:.2f}s: leaves {st['n_leaves']}, phases "
        f"{st['n_phases_used']}, largest window {st['max_window']}, execution {args.gs_exec}")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    b = rng.uniform(-1, 1, m.n)
    bd = torch.as_tensor(b, device=dev)
    bp = torch.empty_like(bd)
    s.permute(bd, bp, True)
    xp = torch.zeros_like(bp)
    s.gauss_seidel(bp, xp)
    x = torch.empty_like(xp)
    s.permute(xp, x, False)
    torch.cuda.synchronize()
    s.check()
    tr = s.tree()
    node, phase = s.leaves()
    order = G.race_order(s.perm(), np.asarray(tr["lo"])[node], np.asarray(tr["hi"])[node], phase)
    ref = G.symmetric_sweep_c(m.n, m.row_ptr, m.col, m.val, b, np.zeros(m.n), order)
    err = float(np.max(np.abs(x.cpu().numpy() - ref)) / np.max(np.abs(ref)))
    ms = time_ring(lambda x_, y_: s.gauss_seidel(bp, xp), [0], [0], args.steps, args.warmup, torch)
    s.check()
    nnz_full = st["nnz_full"]
    flops = 2 * 2 * nnz_full  # both directions: a multiply-add per off-diagonal, the diagonal division
    bytes_min = 2 * (12 * (nnz_full - m.n) + 4 * (m.n + 1) + 32 * m.n)
    achieved = bytes_min / (ms * 1e-3) / 1e9
    log(f"Gauss-Seidel {args.workload}: {ms * 1e3:.1f} us per symmetric sweep, {flops / (ms * 1e-3) / 1e9:.1f} GFLOP/s, "
        f"{achieved:.1f} GB/s algorithmic, error vs oracle {err:.2e}")
    out = {
        "metric": "symmetric Gauss-Seidel sweeps over a distance-1 RACE schedule, GFLOP/s",
        "value": round(flops / (ms * 1e-3) / 1e9, 3), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload + "_dominant", "description": desc + ", diagonal 1 + row abs-sum",
                   "n": m.n, "nnz_full": nnz_full, "n_workers": args.gs_workers, "max_stages": args.gs_stages,
                   "execution": args.gs_exec,
                   "leaves": st["n_leaves"],
                   "phases": st["n_phases_used"], "max_window": st["max_window"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "bytes_per_step": bytes_min},
        "error": {"norm": err}, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    s.close()


def run_kacz(args, torch):
    """Symmetric Kaczmarz sweeps (forward then backward, omega 1) over a
    distance-2 RACE schedule of the workload's matrix: time per symmetric
    sweep, checked against the serial C oracle over the same row order.
    One JSON line.  A sweep direction reads every entry of the full matrix
    (value + column, diagonal included), b and x, and writes x: at least
    12 nnz_full + 4 (N + 1) + 24 N bytes in CRS (squared row norms
    recomputed; the library keeps them, 8 N more)."""
    import numpy as np

    import paper_1907_06487_amd as R
    from oracle import gauss_seidel as G
    from oracle import kaczmarz as K
    m, desc = workload(args.workload)
    t0 = time.perf_counter()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=args.kacz_workers, max_stages=args.kacz_stages,
                   root=args.root, level_order=args.level_order, kaczmarz=True)
    s.set_gs_quad(args.kacz_quad)
    s.set_gs_exec(args.kacz_exec)
    st = s.stats()
    log(f"Kaczmarz schedule built in {time.perf_counter() - t0:.2f}s: leaves {st['n_leaves']}, phases "
        f"{st['n_phases_used']}, largest window {st['kacz_max_window']}, execution {args.kacz_exec}")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    b = rng.uniform(-1, 1, m.n)
    bd = torch.as_tensor(b, device=dev)
    bp = torch.empty_like(bd)
    s.permute(bd, bp, True)
    xp = torch.zeros_like(bp)
    s.kaczmarz(bp, xp)
    x = torch.empty_like(xp)
    s.permute(xp, x, False)
    torch.cuda.synchronize()
    tr = s.tree()
    node, phase = s.leaves()
    order = G.race_order(s.perm(), np.asarray(tr["lo"])[node], np.asarray(tr["hi"])[node], phase)
    ref = K.symmetric_sweep_c(m.n, m.row_ptr, m.col, m.val, b, np.zeros(m.n), order)
    err = float(np.max(np.abs(x.cpu().numpy() - ref)) / np.max(np.abs(ref)))
    ms = time_ring(lambda x_, y_: s.kaczmarz(bp, xp), [0], [0], args.steps, args.warmup, torch)
    s.check()
    nnz_full = st["nnz_full"]
    flops = 2 * 4 * nnz_full  # both directions: a multiply-add per entry for the dot product and for the update
    bytes_min = 2 * (12 * nnz_full + 4 * (m.n + 1) + 24 * m.n)
    achieved = bytes_min / (ms * 1e-3) / 1e9
    log(f"Kaczmarz {args.workload}: {ms * 1e3:.1f} us per symmetric sweep, {flops / (ms * 1e-3) / 1e9:.1f} GFLOP/s, "
        f"{achieved:.1f} GB/s algorithmic, error vs oracle {err:.2e}")
    out = {
        "metric": "symmetric Kaczmarz sweeps over a distance-2 RACE schedule, GFLOP/s",
        "value": round(flops / (ms * 1e-3) / 1e9, 3), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": m.n, "nnz_full": nnz_full,
                   "n_workers": args.kacz_workers, "max_stages": args.kacz_stages, "omega": 1.0,
                   "quad_min_leaves": args.kacz_quad, "execution": args.kacz_exec,
                   "leaves": st["n_leaves"], "phases": st["n_phases_used"],
                   "max_window": st["kacz_max_window"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "bytes_per_step": bytes_min},
        "error": {"norm": err}, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    s.close()


def run_mpk(args, torch):
    """Matrix powers y_p = A^p x, p = 1..P, of the workload's matrix scaled
    by its largest absolute row sum: one race_symm_mpk launch against P
    separate race_symm_spmv products, each error against the oracle's
    power.  One JSON line; each power moves the product's algorithmic
    bytes."""
    import numpy as np

    import matgen
    import paper_1907_06487_amd as R
    from oracle import powers as OP
    from oracle import symmspmv as O
    P = args.mpk
    m, desc = workload(args.workload)
    scale = float(np.max(O.abs_product(m.n, m.row_ptr, m.col, m.val, np.ones(m.n))))
    m = matgen.UpperCSR(m.n, m.row_ptr, m.col, m.val / scale, m.name + "_scaled")
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=args.n_workers, max_stages=args.max_stages,
                   block_threads=args.block, window_max=args.window, value_type=args.value_type)
    st = s.stats()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(61)
    x = rng.uniform(-1, 1, m.n)
    xd = torch.as_tensor(x, device=dev)
    xp = torch.empty_like(xd)
    s.permute(xd, xp, True)
    nring = max(2, -(-RING_BYTES // (8 * m.n * P)))
    Ys = [torch.empty((P, m.n), dtype=torch.float64, device=dev) for _ in range(nring)]
    perm = s.perm()
    vals = m.val if args.value_type == "f64" else m.val.astype(np.float32).astype(np.float64)
    refs = OP.powers(m.n, m.row_ptr, m.col, vals, x, P)
    # ticket orders: lag_rows:cache_matrix pairs (lag < 0: power-major)
    orders = []
    for item in args.mpk_orders.split(","):
        lag, cache = (int(v) for v in item.split(":"))
        s.set_mpk_order(lag, bool(cache))
        Ys[0].fill_(float("nan"))
        s.mpk(xp, Ys[0])
        torch.cuda.synchronize()
        s.check()
        Yh = Ys[0].cpu().numpy()
        errs_o = [float(np.max(np.abs(Yh[p] - refs[p][perm])) / np.max(np.abs(refs[p]))) for p in range(P)]
        ms_o = time_ring(lambda a, y: s.mpk(xp, y), Ys, Ys, args.steps, args.warmup, torch)
        s.check()
        log(f"matrix powers P={P} order lag={lag} cache={cache}: {ms_o * 1e3:.1f} us, {ms_o * 1e3 / P:.1f} us per power, "
            f"worst power error {max(errs_o):.2e}")
        orders.append({"lag_rows": lag, "cache_matrix": cache, "ms": ms_o, "worst_error": max(errs_o), "errs": errs_o})
    best = min(orders, key=lambda o: o["ms"])
    ms, errs = best["ms"], best["errs"]

    def separate(a, Y):
        s.spmv(xp, Y[0])
        for p in range(1, P):
            s.spmv(Y[p - 1], Y[p])

    ms_sep = time_ring(separate, Ys, Ys, args.steps, args.warmup, torch)
    flops = 2 * st["nnz_full"] * P
    bytes_alg = (st["bytes_min"] - (4 * st["nnz_upper"] if args.value_type == "f32" else 0)) * P
    achieved = bytes_alg / (ms * 1e-3) / 1e9
    log(f"matrix powers P={P} {args.workload}: {ms * 1e3:.1f} us in one launch, {ms_sep * 1e3:.1f} us as {P} products "
        f"({ms_sep / ms:.3f}x), {flops / (ms * 1e-3) / 1e9:.1f} GFLOP/s, {achieved:.1f} GB/s algorithmic, "
        f"worst power error {max(errs):.2e}")
    out = {
        "metric": f"matrix powers A^p x, p = 1..{P}, GFLOP/s", "value": round(flops / (ms * 1e-3) / 1e9, 3),
        "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.value_type == "f64" else "f32-values/f64-accumulate", "data": "synthetic",
        "config": {"workload": args.workload + "_scaled", "description": desc + ", scaled by its largest row sum",
                   "powers": P, "n": m.n, "n_workers": args.n_workers, "block_threads": args.block,
                   "window_max": args.window, "units": st["n_units"],
                   "ticket_order": {"lag_rows": best["lag_rows"], "cache_matrix": best["cache_matrix"]}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "bytes_per_step": bytes_alg},
        "orders": [{k: v for k, v in o.items() if k != "errs"} for o in orders],
        "separate_products": {"ms": ms_sep, "speedup_of_one_launch": ms_sep / ms},
        "error": {"per_power_norm": errs}, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    s.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="3d27pt_128")
    ap.add_argument("--n-workers", type=int, default=256)
    ap.add_argument("--max-stages", type=int, default=2,
                    help="recursion stages (2 measured 1.5%% faster than the library default 4 on the 128^3 stencil)")
    ap.add_argument("--block", type=int, default=512)
    ap.add_argument("--window", type=int, default=4064,
                    help="largest unit window (4064: two 512-thread workgroups per CU still fit the LDS; 1.5%% "
                         "faster than the library default 3840 on the 128^3 stencil)")
    ap.add_argument("--value-type", default="f64", choices=["f64", "f32", "c128", "c128h"])
    ap.add_argument("--exec-mode", default="flow", choices=["flow", "phases"])
    ap.add_argument("--shared-atomics", type=int, default=1, choices=[0, 1],
                    help="units of one leaf run concurrently, combining shared y entries atomically (1) or in order (0)")
    ap.add_argument("--root", default="first", choices=["first", "peripheral"],
                    help="stage-0 BFS root of every island: its first vertex or a pseudo-peripheral one")
    ap.add_argument("--level-order", default="input", choices=["input", "cm"],
                    help="stage-0 order inside a level: input order or Cuthill-McKee numbering")
    ap.add_argument("--dist-k", type=int, default=2, help="distance of the coloring (2 for SymmSpMV; 3..8 wider)")
    ap.add_argument("--global-lb", type=int, default=0, choices=[0, 1],
                    help="also run Algorithm \"Load Balancing\" over all children of every refined node")
    ap.add_argument("--low-locality", default="auto", choices=["auto", "race", "expanded"],
                    help="single-vector products: the library's choice (auto: a CRS product of the expanded permuted "
                         "matrix when the schedule predicts no window reuse), the RACE kernels, or always expanded")
    ap.add_argument("--unit-trace", type=int, default=0,
                    help="also run this many traced products and summarise their per-unit timestamps")
    ap.add_argument("--mpk", type=int, default=0, help="matrix powers A^p x, p = 1..MPK, in one launch instead")
    ap.add_argument("--mpk-orders", default="-1:0",
                    help="matrix-power ticket orders to time, lag_rows:cache_matrix pairs (lag < 0: power-major), "
                         "e.g. -1:0,0:1,500000:1; the fastest is reported")
    ap.add_argument("--gs", action="store_true",
                    help="symmetric Gauss-Seidel sweeps over a distance-1 schedule of the workload instead")
    ap.add_argument("--gs-exec", default="flow", choices=["phases", "flow"],
                    help="--gs: one launch per phase, or one dataflow launch per sweep (128^3, N_t 16384: 527 us "
                         "against 712 us with phase launches)")
    ap.add_argument("--gs-stages", type=int, default=4, help="--gs: recursion stages of the distance-1 schedule")
    ap.add_argument("--gs-workers", type=int, default=16384,
                    help="--gs: n_workers of the distance-1 schedule (on the 128^3 stencil 16384 measured fastest with "
                         "the dataflow launch: 527 us against 585 us at 65536)")
    ap.add_argument("--kacz", action="store_true",
                    help="symmetric Kaczmarz sweeps over a distance-2 schedule of the workload instead")
    ap.add_argument("--kacz-workers", type=int, default=4096, help="--kacz: n_workers of the schedule")
    ap.add_argument("--kacz-stages", type=int, default=3, help="--kacz: recursion stages of the schedule")
    ap.add_argument("--kacz-exec", default="flow", choices=["phases", "flow"],
                    help="--kacz: one launch per phase, or one dataflow launch per sweep (128^3, N_t 4096: 930 us "
                         "against 1,398 us with phase launches)")
    ap.add_argument("--kacz-quad", type=int, default=-1,
                    help="--kacz: phases of at least this many leaves run four per wavefront (-1 library default, "
                         "-2 never, 0 always)")
    ap.add_argument("--order", default="default", choices=["default", "critical"],
                    help="dataflow ticket order: the layout's execution order, or the critical path of unit costs "
                         "measured by traced products on this device (part of the schedule's preparation)")
    ap.add_argument("--order-rounds", type=int, default=1,
                    help="critical order: trace-and-reorder rounds (each traces under the previous order)")
    ap.add_argument("--no-attainable", action="store_true", help="skip the attainable-bandwidth measurement")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-baselines", action="store_true")
    ap.add_argument("--k", default="1", help="batch64 workload: right-hand sides, e.g. 1,4,16")
    ap.add_argument("--model-dir", default=None, help="learned_ab workload: directory of cost_model.npy/.json")
    ap.add_argument("--rounds", type=int, default=5, help="learned_ab workload: timing rounds per arm")
    ap.add_argument("--spmm-k", default="", help="SymmSpMM on the workload's matrix instead, e.g. 4,16 (one line each)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run a device copy of this many MiB (reference for the traffic counters)")
    ap.add_argument("--calibrate-stream", type=int, default=0,
                    help="also run the library's read-only and copy stream kernels over this many MiB, three "
                         "times each (references for FETCH_SIZE and WRITE_SIZE larger than every cache)")
    ap.add_argument("--sweep", default="",
                    help="n_workers:block[:window[:mode[:shared]]] list, e.g. 256:256,512:512:2048:phases:0 (stderr)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding over several GPUs is described "
              "as a design, not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1907_06487_amd as R
    from oracle import symmspmv as O

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batch64":
        for k in (int(v) for v in args.k.split(",")):
            run_batch(args, k, torch)
        return
    if args.workload == "learned_ab":
        run_learned_ab(args, torch)
        return
    if args.value_type.startswith("c"):
        run_complex(args, torch)
        return
    if args.gs:
        run_gs(args, torch)
        return
    if args.kacz:
        run_kacz(args, torch)
        return
    if args.mpk:
        run_mpk(args, torch)
        return
    if args.spmm_k:
        m, _ = workload(args.workload)
        for k in (int(v) for v in args.spmm_k.split(",")):
            run_spmm(args, k, torch, m)
            if k > 2:
                run_spmm(args, k, torch, m, one_pass=True)
        return
    m, desc = workload(args.workload)
    log(f"workload {args.workload}: n={m.n} nnz_upper={m.nnz}")
    t0 = time.perf_counter()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=args.n_workers, max_stages=args.max_stages,
                   block_threads=args.block, window_max=args.window, value_type=args.value_type,
                   exec_mode=args.exec_mode, shared_atomics=bool(args.shared_atomics), root=args.root,
                   level_order=args.level_order, dist_k=args.dist_k, global_lb=bool(args.global_lb),
                   low_locality=args.low_locality)
    t_build = time.perf_counter() - t0
    st = s.stats()
    log(f"schedule built in {t_build:.2f}s: " + json.dumps({k: st[k] for k in (
        "n_levels0", "depth", "n_leaves", "n_phases_used", "n_units", "max_window", "eta", "halo_total",
        "sell_elems", "bytes_min", "bytes_kernel", "n_deps", "shared_touches", "n_zeroed", "product_path",
        "expanded_per_thread")}))

    nring = max(2, -(-RING_BYTES // (8 * m.n)))
    gen = torch.Generator(device=dev)
    gen.manual_seed(12345)
    xs = [torch.rand(m.n, dtype=torch.float64, device=dev, generator=gen) * 2 - 1 for _ in range(nring)]
    ys = [torch.empty(m.n, dtype=torch.float64, device=dev) for _ in range(nring)]

    order_info = {"order": args.order}
    if args.order == "critical":
        # preparation, outside the timed region: unit costs from traced
        # products, then the critical-path ticket order for them
        t0 = time.perf_counter()
        s.order_tickets(None)
        for rnd in range(args.order_rounds):
            cost, frac = s.unit_costs(xs[0], ys[0], reps=3)
            grid = s.flow_grid(1)
            pred_before = s.simulate(cost, frac, grid)
            s.order_tickets(cost)
            pred_after = s.simulate(cost, frac, grid)
            log(f"ticket order round {rnd}: measured unit costs sum {cost.sum():.0f} us, flush share {frac:.2f}; "
                f"predicted makespan {pred_before:.1f} -> {pred_after:.1f} us")
        order_info.update(rounds=args.order_rounds, predicted_us=round(pred_after, 2),
                          prep_s=round(time.perf_counter() - t0, 2))

    # correctness of the timed configuration against the oracle (input order)
    x0 = xs[0].cpu().numpy()
    perm = s.perm()
    x_orig = np.empty(m.n)
    x_orig[perm] = x0
    s.spmv(xs[0], ys[0])
    torch.cuda.synchronize()
    y_perm = ys[0].cpu().numpy()
    y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x_orig)
    err_norm, err_comp = O.errors(y_perm, y_ref[perm], O.abs_product(m.n, m.row_ptr, m.col, m.val, x_orig)[perm])
    log(f"error vs oracle: norm {err_norm:.3e} comp {err_comp:.3e}")

    ms = time_ring(lambda x, y: s.spmv(x, y), xs, ys, args.steps, args.warmup, torch)
    ms_median = time_ring_median(lambda x, y: s.spmv(x, y), xs, ys, args.steps, torch)
    s.check()
    flops = 2 * st["nnz_full"]
    gflops = flops / (ms * 1e-3) / 1e9
    # algorithmic bytes: upper CRS (value + column per stored entry), x, y, row pointers;
    # FP32 values store 4 bytes less per entry
    bytes_alg = st["bytes_min"] - (4 * st["nnz_upper"] if args.value_type == "f32" else 0)
    achieved = bytes_alg / (ms * 1e-3) / 1e9
    # the dataflow mode is one launch (it clears shared-first entries in its
    # first tickets); the phase mode launches once per phase plus the clearing
    launches = 1 if args.exec_mode == "flow" else st["n_phases_used"] + (1 if st["n_zeroed"] else 0)
    path_name = "expanded CRS product" if st["product_path"] == 1 else "RACE"
    # bytes in the format the running kernel reads: the RACE layout's, or for
    # the expanded product the full CRS matrix (value + column per entry, row
    # pointers), x and y
    if st["product_path"] == 1:
        vb = 4 if args.value_type == "f32" else 8
        bytes_fmt = (vb + 4) * st["nnz_full"] + 20 * m.n + 4
    else:
        bytes_fmt = st["bytes_kernel"]
    log(f"{path_name}: {ms * 1e3:.2f} us/product (median {ms_median * 1e3:.2f}), {gflops:.1f} GFLOP/s, {achieved:.1f} GB/s "
        f"algorithmic ({achieved / PEAK_HBM_GBS * 100:.1f}% of peak), kernel-format bytes "
        f"{bytes_fmt / (ms * 1e-3) / 1e9:.1f} GB/s")

    trace_info = unit_trace(s, st, xs, ys, args.unit_trace, torch) if args.unit_trace and st["product_path"] == 0 \
        and args.exec_mode == "flow" else None

    race_kernels = None
    if st["product_path"] == 1:
        # the schedule predicted no window reuse and runs the expanded CRS
        # product; the RACE kernels on the same schedule, for the record
        s3 = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=args.n_workers, max_stages=args.max_stages,
                        block_threads=args.block, window_max=args.window, value_type=args.value_type,
                        exec_mode=args.exec_mode, shared_atomics=bool(args.shared_atomics), root=args.root,
                        level_order=args.level_order, dist_k=args.dist_k, global_lb=bool(args.global_lb),
                        low_locality="race")
        s3.spmv(xs[0], ys[0])
        torch.cuda.synchronize()
        e3 = O.errors(ys[0].cpu().numpy(), y_ref[perm])[0]
        ms3 = time_ring(lambda x, y: s3.spmv(x, y), xs, ys, args.steps, args.warmup, torch)
        s3.check()
        share = st["shared_touches"] / (m.n + st["halo_total"])
        race_kernels = {"us": ms3 * 1e3, "gflops": flops / (ms3 * 1e-3) / 1e9, "err_norm": e3,
                        "shared_touch_share": share,
                        "note": "RACE kernels on this matrix: shared window entries combine through global float64 "
                                "atomics, so the library runs the expanded CRS product instead"}
        log(f"RACE kernels on the same schedule: {ms3 * 1e3:.2f} us ({share * 100:.1f}% of window touches shared), "
            f"error {e3:.2e}; expanded CRS product: {ms * 1e3:.2f} us")
        s3.close()

    for item in filter(None, args.sweep.split(",")):
        nt, blk = (int(v) for v in item.split(":")[:2])
        parts = item.split(":")
        win = int(parts[2]) if len(parts) > 2 else args.window
        mode = parts[3] if len(parts) > 3 else args.exec_mode
        shared = bool(int(parts[4])) if len(parts) > 4 else bool(args.shared_atomics)
        s2 = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=nt, max_stages=args.max_stages, block_threads=blk,
                        window_max=win, value_type=args.value_type, exec_mode=mode, shared_atomics=shared)
        st2 = s2.stats()
        ms2 = time_ring(lambda x, y: s2.spmv(x, y), xs, ys, args.steps, args.warmup, torch)
        s2.check()
        log(f"sweep n_workers={nt} block={blk} window={win} mode={mode} shared={int(shared)}: {ms2 * 1e3:.2f} us, "
            f"{st2['bytes_min'] / (ms2 * 1e-3) / 1e9 / PEAK_HBM_GBS * 100:.1f}% peak, phases={st2['n_phases_used']} "
            f"leaves={st2['n_leaves']} units={st2['n_units']} kernel bytes={st2['bytes_kernel']}")
        s2.close()

    if args.calibrate_copy:
        # a compute-kernel copy (elementwise multiply by one) of known size,
        # larger than every cache: the traffic counters' reference
        nbytes = args.calibrate_copy << 20
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).uniform_()
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"calibration: elementwise copy reading and writing {nbytes} bytes, 3 times")
    if args.calibrate_stream:
        nbytes = args.calibrate_stream << 20
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).uniform_()
        dst = torch.empty_like(src)
        sink = torch.zeros(4, dtype=torch.int32, device=dev)
        grid = torch.cuda.get_device_properties(dev).multi_processor_count * 32
        for _ in range(3):
            R.race_stream_read(src, sink, grid)
        for _ in range(3):
            R.race_stream_copy(src, dst, grid)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
        log(f"calibration: stream read of {nbytes} bytes (3 times), stream copy of {nbytes} bytes each way (3 times)")

    baselines = {}
    if not args.no_baselines:
        baselines = yardsticks(m, perm, flops, st["nnz_full"], xs, ys, args, torch)
        best = min((b["us"], k) for k, b in baselines.items() if k in ("crs_spmv", "vendor_general"))
        baselines["best_spmv"] = best[1]
        baselines["race_speedup_vs_best_spmv"] = best[0] / (ms * 1e3)
        baselines["race_speedup_vs_crs"] = baselines["crs_spmv"]["us"] / (ms * 1e3)
        if "vendor_symmetric" in baselines:
            baselines["race_speedup_vs_vendor_symmetric"] = baselines["vendor_symmetric"]["us"] / (ms * 1e3)
        baselines["race_speedup_vs_atomic"] = baselines["atomic_symmspmv"]["us"] / (ms * 1e3)
        log(f"RACE vs best full-matrix SpMV ({best[1]}, {best[0]:.2f} us): {baselines['race_speedup_vs_best_spmv']:.3f}x")

    attain = None
    if not args.no_attainable:
        attain = attainable_bandwidth(torch)

    cpu = None
    if not args.no_cpu:
        dt, dt_med, reps, core = cpu_baseline(m, args.cpu_seconds)
        model, threads, ncpu = host_cpu()
        cpu = {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full products of the same matrix with the serial C oracle (-O2), "
                         f"{dt * 1e3:.1f} ms each (median {dt_med * 1e3:.1f} ms), one thread pinned to core {core}",
               "median_value": flops / dt_med / 1e9, "host_cpu": model, "host_threads_allowed": threads,
               "host_nproc": ncpu}
        log(f"CPU oracle: {dt * 1e3:.1f} ms/product ({cpu['value']:.3f} GFLOP/s) on {model}")

    # HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    # runs, valid only while the kernel, layout and parameters are unchanged
    traffic = traffic_rw = None
    tpath = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")
    if os.path.exists(tpath):
        tr = json.load(open(tpath))
        same = (tr.get("source_hash") == kernel_source_hash(st["product_path"])
                and tr.get("bytes_kernel") == st["bytes_kernel"]
                and tr.get("n_workers") == args.n_workers and tr.get("block_threads") == args.block
                and tr.get("window_max") == args.window and tr.get("exec_mode") == args.exec_mode
                and tr.get("max_stages", 4) == args.max_stages
                and tr.get("shared_atomics", 0) == args.shared_atomics and tr.get("root", "first") == args.root
                and tr.get("level_order", "input") == args.level_order and args.dist_k == 2
                and tr.get("product_path", 0) == st["product_path"])
        if same and args.value_type == "f64":
            traffic = tr.get("bytes_per_launch")
            traffic_rw = {"read": tr.get("read_bytes_per_launch"), "write": tr.get("write_bytes_per_launch")}

    out = {
        "metric": METRIC, "value": round(gflops, 3), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.value_type == "f64" else "f32-values/f64-accumulate", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": m.n, "nnz_upper": m.nnz,
                   "nnz_full": st["nnz_full"], "n_workers": args.n_workers, "max_stages": args.max_stages,
                   "block_threads": args.block,
                   "window_max": args.window, "exec_mode": args.exec_mode, "shared_atomics": args.shared_atomics,
                   "root": args.root, "level_order": args.level_order, "dist_k": args.dist_k,
                   "levels0": st["n_levels0"], "ticket_order": order_info,
                   "phases": st["n_phases_used"], "leaves": st["n_leaves"], "eta": st["eta"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "traffic_read_write": traffic_rw, "launches_per_step": launches,
                     "bytes_per_step": bytes_alg, "kernel_format_bytes_per_step": bytes_fmt,
                     "attainable_read_GBs": attain["read_GBs"] if attain else None,
                     "attainable_copy_GBs": attain["copy_GBs"] if attain else None,
                     "frac_of_attainable_read": round(achieved / attain["read_GBs"], 4) if attain else None,
                     "ms_per_step_median": ms_median},
        "schedule": {"shared_touches": st["shared_touches"], "halo_total": st["halo_total"],
                     "units": st["n_units"], "global_lb": args.global_lb,
                     "product_path": "expanded CRS" if st["product_path"] == 1 else "RACE kernels",
                     "expanded_per_thread": st["expanded_per_thread"]},
        "race_kernels": race_kernels,
        "unit_trace": trace_info,
        "attainable": attain,
        "error": {"norm": err_norm, "componentwise": err_comp},
        "baselines": baselines,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    s.close()


if __name__ == "__main__":
    main()
