"""GPU parity of the matrix powers and polynomials (race_symm_mpk,
race_symm_poly) against the oracle (oracle/powers.py: one product after
the other, float64).  Every power vector is compared normwise; the
powers grow as the matrix norm to the p, so the bound is relative to each
power's own magnitude:  ||y_p - y_p,ref||_inf / ||y_p,ref||_inf <= 1e-12.
Cases cover shared-atomic units with clearing tasks, chained units, a
schedule built for the phase mode, FP32 values (oracle on the same
rounded values), workgroups forced to join late (static tickets taken
over), a critical-path ticket order, the diagonal ticket order with and
without cacheable matrix loads, and repeated calls."""
import numpy as np
import pytest

import matgen
import paper_1907_06487_amd as R
from oracle import powers as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _err(y, ref):
    return float(np.max(np.abs(y - ref)) / max(np.max(np.abs(ref)), 1e-300))


CASES = [
    ("2d5pt_100", matgen.config_2d_small, dict(n_workers=64)),
    ("3d27pt_24_w128", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=64, window_max=128)),
    ("3d27pt_24_w128_chain", lambda: matgen.stencil3d_27pt(24, seed=5),
     dict(n_workers=64, window_max=128, shared_atomics=False)),
    ("banded_40k_w96", lambda: matgen.banded_irregular(40000, seed=6, band=4000), dict(n_workers=16, window_max=96)),
    ("3d27pt_40_b512", lambda: matgen.stencil3d_27pt(40, seed=71), dict(n_workers=256, block_threads=512)),
    ("3d27pt_24_phases", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256, exec_mode="phases")),
    ("rand_islands", lambda: matgen.random_symmetric(500, 0.003, seed=8), dict(n_workers=16)),
]


def _scaled(m):
    """The matrix divided by its largest absolute row sum, so that the
    powers neither overflow nor vanish."""
    from oracle import symmspmv as O
    s = float(np.max(O.abs_product(m.n, m.row_ptr, m.col, m.val, np.ones(m.n))))
    return matgen.UpperCSR(m.n, m.row_ptr, m.col, m.val / s, m.name + "_scaled")


@pytest.mark.parametrize("powers", [1, 3, 6])
@pytest.mark.parametrize("name,make,params", CASES, ids=[c[0] for c in CASES])
def test_mpk_parity(name, make, params, powers):
    m = _scaled(make())
    x = matgen.rhs(m.n, 51)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, **params)
    try:
        print(f"case mpk {name} powers={powers}: n={m.n} units={s.stats()['n_units']}", flush=True)
        perm = s.perm()
        refs = P.powers(m.n, m.row_ptr, m.col, m.val, x, powers)
        xd = torch.as_tensor(x, device=DEV)
        xp = torch.empty_like(xd)
        s.permute(xd, xp, True)
        for rep in range(2):  # a second call reuses the launch state
            Y = torch.full((powers, m.n), float("nan"), dtype=torch.float64, device=DEV)
            s.mpk(xp, Y)
            torch.cuda.synchronize()
            s.check()
            Yh = Y.cpu().numpy()
            errs = [_err(Yh[p], refs[p][perm]) for p in range(powers)]
            print(f"  rep {rep}: errors {['%.2e' % e for e in errs]}", flush=True)
            assert max(errs) <= 1e-12
    finally:
        s.close()


@pytest.mark.parametrize("lag,cache", [(0, True), (500, False), (4000, True)])
@pytest.mark.parametrize("name,make,params", [CASES[0], CASES[1], CASES[3], CASES[4], CASES[6]],
                         ids=[CASES[i][0] for i in (0, 1, 3, 4, 6)])
def test_mpk_diagonal_order(name, make, params, lag, cache):
    """The diagonal ticket order (race_schedule_set_mpk_order) with several
    lags, cacheable or non-temporal matrix loads, 5 powers, two calls, and
    a change of the number of powers in between (the order is rebuilt)."""
    m = _scaled(make())
    x = matgen.rhs(m.n, 53)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, **params)
    try:
        s.set_mpk_order(lag, cache)
        perm = s.perm()
        refs = P.powers(m.n, m.row_ptr, m.col, m.val, x, 5)
        xd = torch.as_tensor(x, device=DEV)
        xp = torch.empty_like(xd)
        s.permute(xd, xp, True)
        for powers in (5, 2, 5):
            print(f"case mpk diagonal {name} lag={lag} cache={cache} powers={powers}: n={m.n}", flush=True)
            Y = torch.full((powers, m.n), float("nan"), dtype=torch.float64, device=DEV)
            s.mpk(xp, Y)
            torch.cuda.synchronize()
            s.check()
            Yh = Y.cpu().numpy()
            errs = [_err(Yh[p], refs[p][perm]) for p in range(powers)]
            print(f"  errors {['%.2e' % e for e in errs]}", flush=True)
            assert max(errs) <= 1e-12
    finally:
        s.close()


def test_mpk_float32_values_late_workgroups_and_ticket_order():
    m = _scaled(matgen.stencil3d_27pt(40, seed=72))
    vals32 = m.val.astype(np.float32).astype(np.float64)
    x = matgen.rhs(m.n, 52)
    refs = P.powers(m.n, m.row_ptr, m.col, vals32, x, 4)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=64, window_max=512, value_type="f32")
    try:
        perm = s.perm()
        xd = torch.as_tensor(x, device=DEV)
        xp = torch.empty_like(xd)
        s.permute(xd, xp, True)
        nu = s.stats()["n_units"]
        for tag, setup in (("late", lambda: s.test_late(3)),
                           ("late_diagonal", lambda: s.set_mpk_order(300, True)),
                           ("critical_order", lambda: (s.test_late(0), s.set_mpk_order(-1, False),
                                                       s.order_tickets(np.random.default_rng(3).uniform(1, 5, nu).astype(np.float32)))),
                           ("critical_order_diagonal", lambda: s.set_mpk_order(0, False))):
            setup()
            before = s.takeovers()
            Y = torch.full((4, m.n), float("nan"), dtype=torch.float64, device=DEV)
            s.mpk(xp, Y)
            torch.cuda.synchronize()
            s.check()
            errs = [_err(Y[p].cpu().numpy(), refs[p][perm]) for p in range(4)]
            print(f"[mpk f32 {tag}] errors {['%.2e' % e for e in errs]} takeovers {s.takeovers() - before}", flush=True)
            assert max(errs) <= 1e-12
            if tag in ("late", "late_diagonal"):
                assert s.takeovers() - before > 0
    finally:
        s.close()


@pytest.mark.parametrize("coeffs", [[0.5], [1.0, 2.0, 1.0], [0.3, -1.0, 0.25, 2.0, -0.5]])
def test_poly_parity(coeffs):
    m = _scaled(matgen.stencil3d_27pt(24, seed=5))
    x = matgen.rhs(m.n, 53)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=64, window_max=256)
    try:
        perm = s.perm()
        ref = P.poly(m.n, m.row_ptr, m.col, m.val, coeffs, x)[perm]
        xd = torch.as_tensor(x, device=DEV)
        xp = torch.empty_like(xd)
        s.permute(xd, xp, True)
        work = torch.empty((max(1, len(coeffs) - 1), m.n), dtype=torch.float64, device=DEV)
        z = torch.full_like(xp, float("nan"))
        s.poly(coeffs, xp, work, z)
        torch.cuda.synchronize()
        s.check()
        e = _err(z.cpu().numpy(), ref)
        print(f"[poly {coeffs}] error {e:.2e}", flush=True)
        assert e <= 1e-12
    finally:
        s.close()


def test_mpk_errors():
    m = matgen.config_2d_small()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=64)
    g = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=64, dist_k=1)
    try:
        x = torch.zeros(m.n, dtype=torch.float64, device=DEV)
        for bad in (0, 65):
            with pytest.raises(R.RaceError) as e:
                R.race_symm_mpk(s.handle, bad, x, torch.zeros((1, m.n), dtype=torch.float64, device=DEV))
            assert e.value.code == -1
        with pytest.raises(R.RaceError) as e:
            g.mpk(x, torch.zeros((2, m.n), dtype=torch.float64, device=DEV))
        assert e.value.code == -4
        with pytest.raises(R.RaceError) as e:
            s.poly(list(range(34)), x, torch.zeros((33, m.n), dtype=torch.float64, device=DEV), torch.zeros_like(x))
        assert e.value.code == -1
    finally:
        s.close()
        g.close()
