"""RACE-scheduled symmetric SpMV for AMD MI355X (gfx950).

The work happens in librace.so (C ABI, include/race.h): the host builds the
recursive distance-2 coloring of the matrix graph (Section 4 of Alappat et
al.) and the kernels' data layout; gfx950 kernels run the product one
phase at a time.  This package only marshals arguments (``_lib``) and adds
a small owning wrapper (``Schedule``).  PyTorch supplies device memory and
streams.
"""
from __future__ import annotations

from . import _lib
from ._lib import (RaceError, race_atomic_create, race_batch_bind, race_batch_check, race_batch_create,
                   race_batch_destroy, race_batch_info, race_batch_run, race_build_schedule, race_csr_create, race_csr_destroy,
                   race_csr_spmv, race_last_error, race_params_default, race_permute, race_schedule_check, race_schedule_destroy,
                   race_schedule_flow_takeovers, race_schedule_flow_test_late, race_schedule_order_tickets,
                   race_schedule_set_ticket_order, race_schedule_ticket_order, race_symm_mpk, race_symm_poly,
                   race_schedule_read_deps,
                   race_schedule_leaves, race_schedule_perm, race_schedule_stats, race_schedule_tree,
                   race_schedule_units, race_schedule_upload, race_schedule_zero_list, race_symm_spmm, race_symm_spmm_traced, race_symm_spmv,
                   race_symm_gs, race_symm_kacz, race_symm_spmv_atomic, race_symm_spmv_noalloc, race_stream_copy, race_stream_read,
                   race_vendor_create, race_vendor_destroy, race_vendor_spmv)

BALANCE = {"nnz": 0, "rows": 1, "model": 2}


def make_params(n_workers=1024, max_stages=4, balance="nnz", global_lb=False, value_type="f64", window_max=3840,
                block_threads=256, eps=(0.8, 0.8, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5), exec_mode="flow",
                shared_atomics=True, cost_model=None, rhs_tile=0, root="first", level_order="input", dist_k=2,
                low_locality="race", kaczmarz=False):
    """race_params from keywords.  balance="model" needs cost_model: the
    network's MLP_PARAMS float32 weights (kept alive on the returned struct).
    root: "first" (stage-0 islands start at their first vertex in the input
    order) or "peripheral" (at a pseudo-peripheral vertex).  level_order:
    "input" or "cm" (Cuthill-McKee discovery order inside stage-0 levels).
    low_locality: "race" (always the RACE kernels), "auto" (single-vector
    products switch to a full-matrix CRS product of the permuted matrix when
    the layout predicts no window reuse) or "expanded" (always that).
    kaczmarz: also build the Kaczmarz sweep layout (distance >= 2)."""
    p = race_params_default()
    p.dist_k = int(dist_k)
    p.n_workers = int(n_workers)
    p.max_stages = int(max_stages)
    p.balance_by = BALANCE[balance]
    p.global_lb = int(bool(global_lb))
    p.value_type = {"f64": 0, "f32": 1, "c128": 2, "c128h": 3}[value_type]
    p.window_max = int(window_max)
    p.block_threads = int(block_threads)
    p.exec_mode = {"phases": 0, "flow": 1}[exec_mode]
    p.shared_atomics = int(bool(shared_atomics))
    p.rhs_tile = int(rhs_tile)
    p.root_mode = {"first": 0, "peripheral": 1}[root]
    p.level_order = {"input": 0, "cm": 1}[level_order]
    p.low_locality = {"race": 0, "auto": 1, "expanded": 2}[low_locality]
    p.kaczmarz = int(bool(kaczmarz))
    if cost_model is not None:
        import ctypes

        import numpy as np
        w = np.ascontiguousarray(cost_model, dtype=np.float32)
        p._cost_model_ref = w
        p.cost_model = w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        p.cost_model_len = int(w.size)
    eps = list(eps) + [eps[-1]] * (8 - len(eps))
    for i in range(8):
        p.eps[i] = float(eps[i])
    return p


class Schedule:
    """Owning wrapper around a race_schedule_t."""

    def __init__(self, n, row_ptr, col, val, upload=True, **params):
        self.n = int(n)
        self.params = make_params(**params)
        self.handle = race_build_schedule(self.n, row_ptr, col, val, self.params)
        if upload:
            race_schedule_upload(self.handle)

    def upload(self):
        race_schedule_upload(self.handle)

    def check(self):
        race_schedule_check(self.handle)

    def takeovers(self):
        """Static dataflow tickets run by a workgroup other than their own (cumulative)."""
        return race_schedule_flow_takeovers(self.handle)

    def test_late(self, stride):
        """Tests only: every stride-th workgroup of later dataflow launches joins late."""
        race_schedule_flow_test_late(self.handle, stride)

    def stats(self):
        return race_schedule_stats(self.handle)

    def perm(self):
        return race_schedule_perm(self.handle, self.n)

    def tree(self):
        return race_schedule_tree(self.handle)

    def leaves(self):
        return race_schedule_leaves(self.handle)

    def units(self):
        return race_schedule_units(self.handle, self.n)

    def zero_list(self):
        return race_schedule_zero_list(self.handle)

    def features(self, k=1):
        """Cost-model features of every unit (n_units x 12, float32)."""
        return _lib.race_schedule_features(self.handle, self.stats()["n_units"], k)

    def simulate(self, cost, flush_frac, workers):
        """Predicted dataflow makespan for per-unit costs."""
        return _lib.race_schedule_simulate(self.handle, cost, flush_frac, workers)

    def flow_grid(self, k=1):
        return _lib.race_schedule_flow_grid(self.handle, k)

    def ticket_order(self):
        """Units by dataflow ticket."""
        return race_schedule_ticket_order(self.handle, self.stats()["n_units"])

    def set_ticket_order(self, ticket_unit):
        race_schedule_set_ticket_order(self.handle, ticket_unit)

    def order_tickets(self, cost):
        """Critical-path ticket order for per-unit costs (None: the default order)."""
        race_schedule_order_tickets(self.handle, cost)

    def unit_costs(self, x, y, reps=3, stream=None):
        """Measured per-unit costs (microseconds: arithmetic plus flush,
        waits excluded; the median over `reps` traced products) and the
        flush's mean share of them."""
        import numpy as np
        import torch
        nu = self.stats()["n_units"]
        hz = self.stats()["wall_clock_hz"]
        tr = torch.empty(4 * nu, dtype=torch.int64, device=x.device)
        costs, flush = [], []
        for _ in range(reps):
            self.traced(x, y, tr, stream)
            torch.cuda.synchronize()
            t = tr.cpu().numpy().reshape(nu, 4).astype(np.float64) * (1e6 / hz)
            comp, fl = t[:, 1] - t[:, 0], t[:, 3] - t[:, 2]
            costs.append(comp + fl)
            flush.append(fl.sum() / max((comp + fl).sum(), 1e-30))
        self.check()
        return np.median(np.stack(costs), axis=0).astype(np.float32), float(np.median(flush))

    def tune_order(self, x, y, reps=3, stream=None):
        """Critical-path ticket order from this device's measured unit costs
        (one traced product per rep, default order first)."""
        self.order_tickets(None)
        cost, flush_frac = self.unit_costs(x, y, reps, stream)
        self.order_tickets(cost)
        return cost, flush_frac

    def spmv(self, x, y, stream=None):
        race_symm_spmv(self.handle, x, y, stream)

    def gauss_seidel(self, b, x, direction="symmetric", stream=None):
        """Gauss-Seidel sweep(s) on A x = b in place (distance-1 schedules)."""
        race_symm_gs(self.handle, b, x, direction, stream)

    def kaczmarz(self, b, x, direction="symmetric", omega=1.0, stream=None):
        """Kaczmarz sweep(s) on A x = b in place (schedules built with
        kaczmarz=True); omega in (0, 2)."""
        race_symm_kacz(self.handle, b, x, direction, omega, stream)

    def mpk(self, x, Y, stream=None):
        """Y[p] = A^(p+1) x for p < Y.shape[0] (Y: powers x n) in one launch."""
        race_symm_mpk(self.handle, Y.shape[0], x, Y, stream)

    def poly(self, coeffs, x, work, z, stream=None):
        """z = sum_p coeffs[p] A^p x; work holds (len(coeffs) - 1) x n doubles."""
        race_symm_poly(self.handle, coeffs, x, work, z, stream)

    def read_deps(self):
        return race_schedule_read_deps(self.handle, self.stats()["n_units"])

    def set_mpk_order(self, lag_rows=-1, cache_matrix=False):
        """Ticket order of mpk(): lag_rows < 0 power-major, else the
        diagonal order with that lag; cache_matrix: cacheable matrix loads."""
        _lib.race_schedule_set_mpk_order(self.handle, lag_rows, int(bool(cache_matrix)))

    def set_gs_exec(self, mode="phases"):
        """Gauss-Seidel sweeps as one launch per phase ("phases") or one
        dataflow launch per sweep ("flow")."""
        _lib.race_schedule_set_gs_exec(self.handle, {"phases": 0, "flow": 1}[mode])

    def gs_flow_plan(self, direction=2):
        """Tickets and waits of the dataflow sweep (0 forward, 1 backward, 2 both)."""
        return _lib.race_schedule_gs_flow_plan(self.handle, direction)

    def set_gs_quad(self, min_leaves=-1):
        """Gauss-Seidel phases with at least min_leaves leaves run four leaves
        per wavefront (-1: the default threshold, -2: never, 0: always)."""
        _lib.race_schedule_set_gs_quad(self.handle, min_leaves)

    def mpk_order(self, powers, n_static):
        """The matrix-power ticket order (power-major indices by ticket)."""
        st = self.stats()
        return _lib.race_schedule_mpk_order(self.handle, powers, n_static, st["n_units"] + st["n_zero_tasks"])

    def spmv_noalloc(self, x, y, stream=None):
        """The product through the entry point that allocates nothing."""
        race_symm_spmv_noalloc(self.handle, x, y, stream)

    def spmm(self, X, Y, stream=None):
        race_symm_spmm(self.handle, X.shape[1] if X.dim() == 2 else 1, X, Y, stream)

    def traced(self, X, Y, trace, stream=None):
        race_symm_spmm_traced(self.handle, X.shape[1] if X.dim() == 2 else 1, X, Y, trace, stream)

    def permute(self, inp, out, to_permuted=True, stream=None):
        k = inp.shape[1] if inp.dim() == 2 else 1
        if inp.is_complex():  # (re, im) pairs move as two columns
            k *= 2
        race_permute(self.handle, k, inp, out, to_permuted, stream)

    def close(self):
        if self.handle is not None:
            race_schedule_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owning wrapper around a race_batch_t (the schedules must outlive it)."""

    def __init__(self, schedules, k, threads=0):
        self.schedules = list(schedules)
        self.k = int(k)
        self.handle = race_batch_create([s.handle for s in self.schedules], self.k, threads)

    def bind(self, xs, ys):
        race_batch_bind(self.handle, xs, ys)

    def run(self, use_graph=True, stream=None):
        race_batch_run(self.handle, use_graph, stream)

    def check(self):
        race_batch_check(self.handle)

    def info(self):
        return race_batch_info(self.handle)

    def close(self):
        if self.handle is not None:
            race_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
