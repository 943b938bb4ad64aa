"""The committed learned cost model on held-out inputs (never traced for
training): prediction quality on unit timings the engine measures, and the
held-out A/B on the 3D 27-point 160^3 stencil -- the schedule chosen with
the network against the one the nonzero heuristic chooses.  The gain is
measured and reported; the test requires no loss beyond timing noise and
correct products from both schedules."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import matgen
import paper_1907_06487_amd as R
from paper_1907_06487_amd import costmodel as CM
from oracle import symmspmv as O

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_predictions_on_held_out_matrices():
    theta, meta = CM.load()
    mats = [matgen.batch_family(i, 3000 + i) for i in range(6)] + [matgen.stencil3d_27pt(72, seed=3100)]
    pred, meas = [], []
    for i, m in enumerate(mats):
        for k in (1, 4):
            s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=max(4, m.n // 4000), block_threads=512,
                           window_max=min(3840, (159 * 1024) // (16 * k + 4) - 16))
            c, f = CM.traced_unit_costs(s, k, seed=i)
            pred.append(np.log(CM.predict_costs(theta, s.features(k))))
            meas.append(np.log(np.maximum(c + f, 1e-3)))
            s.close()
    pred, meas = np.concatenate(pred), np.concatenate(meas)
    rms = float(np.sqrt(np.mean((pred - meas) ** 2)))
    rank = lambda a: np.argsort(np.argsort(a))
    rho = float(np.corrcoef(rank(pred), rank(meas))[0, 1])
    print(f"held-out units: {pred.size}, rms ln error {rms:.3f}, rank correlation {rho:.3f}", flush=True)
    assert rms <= 0.5 and rho >= 0.8


def _time(s, xs, ys, reps=50, rounds=3):
    out = []
    for _ in range(rounds):
        for i in range(3):
            s.spmv(xs[i % len(xs)], ys[i % len(ys)])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(reps):
            s.spmv(xs[i % len(xs)], ys[(i + 1) % len(ys)])
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / reps * 1e3)
    return float(np.median(out)), float((max(out) - min(out)) / np.median(out))


@pytest.mark.timeout(600)
def test_learned_choice_on_held_out_160():
    theta, meta = CM.load()
    m = matgen.config_3d_160()
    print(f"case learned A/B 3d27pt_160: n={m.n} nnz={m.nnz}", flush=True)
    res = CM.choose(m, theta, meta)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(5)
    xs = [torch.rand(m.n, dtype=torch.float64, device=DEV, generator=gen) * 2 - 1 for _ in range(18)]
    ys = [torch.empty_like(xs[0]) for _ in xs]
    times, spread = {}, {}
    res["default"] = {"params": dict(n_workers=256, block_threads=512, window_max=3840, balance="nnz"), "pred_us": float("nan")}
    for arm in ("heuristic", "learned", "default"):
        kw = dict(res[arm]["params"])
        if kw["balance"] == "model":
            kw["cost_model"] = theta
        s = R.Schedule(m.n, m.row_ptr, m.col, m.val, **kw)
        times[arm], spread[arm] = _time(s, xs, ys)
        s.check()
        x0 = xs[0].cpu().numpy()
        perm = s.perm()
        xo = np.empty(m.n)
        xo[perm] = x0
        yp = torch.full_like(xs[0], float("nan"))
        s.spmv(xs[0], yp)
        torch.cuda.synchronize()
        err = O.errors(yp.cpu().numpy(), O.symm_spmv(m.n, m.row_ptr, m.col, m.val, xo)[perm])[0]
        print(f"  {arm}: {times[arm]:.2f} us per product, predicted {res[arm]['pred_us']:.1f} us, "
              f"params {res[arm]['params']}, error {err:.2e}", flush=True)
        assert err <= 1e-12
        s.close()
    best_without = min(times["heuristic"], times["default"])
    gain = best_without / times["learned"]
    print(f"  learned / heuristic time: {times['learned'] / times['heuristic']:.3f}; gain over the best arm without "
          f"the network (heuristic choice or library defaults): {gain:.4f}x, round-to-round spread up to "
          f"{max(spread.values()) * 100:.1f}%", flush=True)
    # the network's choice must not lose to the method without it beyond
    # the 2% tolerance; on this stencil it does not win beyond the spread
    # either (the defaults are already near the best the candidates offer)
    assert times["learned"] <= 1.02 * best_without
