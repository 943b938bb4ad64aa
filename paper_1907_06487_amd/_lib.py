"""ctypes binding of librace.so (argument marshalling only).

Every function here forwards to the C entry point of the same name declared
in include/race.h.  Device arrays are passed as torch CUDA tensors (their
data pointers), streams as torch streams or raw hipStream_t integers.  The
library must have been built (paper_1907_06487_amd/build.py); importing it
fails loudly otherwise -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librace.so")

RACE_OK = 0
ERRORS = {-1: "RACE_EINVAL", -2: "RACE_ENOMEM", -3: "RACE_EHIP", -4: "RACE_EUNSUPPORTED", -5: "RACE_ESTATE",
          -6: "RACE_EINTERNAL"}

# every symbol the header declares
EXPORTS = [
    "race_params_default", "race_build_schedule", "race_schedule_upload", "race_schedule_destroy",
    "race_schedule_stats", "race_schedule_perm", "race_schedule_tree", "race_schedule_leaves",
    "race_schedule_units", "race_schedule_zero_list", "race_schedule_check", "race_schedule_flow_takeovers", "race_schedule_flow_test_late", "race_symm_spmv", "race_symm_spmm", "race_symm_spmm_traced", "race_permute", "race_csr_create",
    "race_csr_spmv", "race_atomic_create", "race_symm_spmv_atomic", "race_csr_destroy", "race_last_error",
    "race_batch_create", "race_batch_bind", "race_batch_run", "race_batch_check", "race_batch_info",
    "race_batch_destroy", "race_schedule_features", "race_schedule_simulate", "race_schedule_flow_grid",
    "race_mlp_forward_host", "race_mlp_forward", "race_mlp_workspace", "race_mlp_loss_grad", "race_mlp_adam",
    "race_symm_spmv_noalloc", "race_vendor_create", "race_vendor_spmv", "race_vendor_destroy", "race_stream_read",
    "race_stream_copy", "race_symm_gs", "race_schedule_set_ticket_order", "race_schedule_order_tickets",
    "race_schedule_ticket_order", "race_symm_mpk", "race_symm_poly", "race_schedule_read_deps",
    "race_schedule_set_mpk_order", "race_schedule_mpk_order", "race_schedule_set_gs_quad", "race_schedule_set_gs_exec",
    "race_schedule_gs_flow_plan", "race_symm_kacz",
]

MLP_INPUTS = 12
MLP_HIDDEN = 64
MLP_PARAMS = 5057


class RaceError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class race_params(ctypes.Structure):
    _fields_ = [
        ("dist_k", ctypes.c_int32), ("n_workers", ctypes.c_int32), ("max_stages", ctypes.c_int32),
        ("balance_by", ctypes.c_int32), ("global_lb", ctypes.c_int32), ("value_type", ctypes.c_int32),
        ("window_max", ctypes.c_int32), ("block_threads", ctypes.c_int32), ("eps", ctypes.c_double * 8),
        ("cost_model", ctypes.POINTER(ctypes.c_float)), ("cost_model_len", ctypes.c_int32),
        ("exec_mode", ctypes.c_int32), ("shared_atomics", ctypes.c_int32), ("rhs_tile", ctypes.c_int32),
        ("root_mode", ctypes.c_int32), ("level_order", ctypes.c_int32), ("low_locality", ctypes.c_int32),
        ("kaczmarz", ctypes.c_int32),
    ]


class race_stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_levels0", ctypes.c_int32), ("depth", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
        ("n_leaves", ctypes.c_int32), ("n_phases", ctypes.c_int32), ("n_phases_used", ctypes.c_int32),
        ("n_units", ctypes.c_int32), ("max_window", ctypes.c_int32), ("n_chunks", ctypes.c_int32),
        ("n_eff_root", ctypes.c_int32), ("n_workers", ctypes.c_int32), ("eta", ctypes.c_double),
        ("nnz_upper", ctypes.c_int64), ("nnz_full", ctypes.c_int64), ("n_diag", ctypes.c_int64),
        ("sell_elems", ctypes.c_int64), ("halo_total", ctypes.c_int64), ("rows_rmw", ctypes.c_int64),
        ("halo_rmw", ctypes.c_int64), ("bytes_min", ctypes.c_int64), ("bytes_kernel", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64), ("n_deps", ctypes.c_int64), ("flow_grid", ctypes.c_int32),
        ("exec_mode", ctypes.c_int32), ("wall_clock_hz", ctypes.c_int64), ("shared_touches", ctypes.c_int64),
        ("n_zeroed", ctypes.c_int64), ("product_path", ctypes.c_int32), ("expanded_per_thread", ctypes.c_int32),
        ("n_zero_tasks", ctypes.c_int32), ("kacz_max_window", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)
_U8P = ctypes.POINTER(ctypes.c_uint8)
_DP = ctypes.POINTER(ctypes.c_double)
_FP = ctypes.POINTER(ctypes.c_float)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"librace.so is not built ({LIB_PATH}); run paper_1907_06487_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "race_params_default": ([ctypes.POINTER(race_params)], ctypes.c_int),
        "race_build_schedule": ([ctypes.c_int32, _I32P, _I32P, _DP, ctypes.POINTER(race_params), ctypes.POINTER(_P)],
                                ctypes.c_int),
        "race_schedule_upload": ([_P], ctypes.c_int),
        "race_schedule_destroy": ([_P], None),
        "race_schedule_stats": ([_P, ctypes.POINTER(race_stats)], ctypes.c_int),
        "race_schedule_perm": ([_P, _I32P], ctypes.c_int),
        "race_schedule_tree": ([_P, _I32P, _I32P, _I32P, _I32P, _I32P, _I32P, _I32P], ctypes.c_int),
        "race_schedule_leaves": ([_P, _I32P, _I32P, _I32P], ctypes.c_int),
        "race_schedule_units": ([_P, _I32P, _I64P, _I32P, _I32P, _I32P, _I64P, _I32P, _U8P, _U8P], ctypes.c_int),
        "race_schedule_zero_list": ([_P, _I64P, _I32P], ctypes.c_int),
        "race_schedule_check": ([_P], ctypes.c_int),
        "race_schedule_flow_takeovers": ([_P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "race_schedule_flow_test_late": ([_P, ctypes.c_int32], ctypes.c_int),
        "race_schedule_set_ticket_order": ([_P, _I32P], ctypes.c_int),
        "race_schedule_order_tickets": ([_P, _FP], ctypes.c_int),
        "race_schedule_ticket_order": ([_P, _I32P], ctypes.c_int),
        "race_symm_mpk": ([_P, ctypes.c_int32, _P, _P, _P], ctypes.c_int),
        "race_symm_poly": ([_P, ctypes.c_int32, _DP, _P, _P, _P, _P], ctypes.c_int),
        "race_schedule_read_deps": ([_P, _I64P, _I32P, _I32P], ctypes.c_int),
        "race_schedule_set_mpk_order": ([_P, ctypes.c_int64, ctypes.c_int32], ctypes.c_int),
        "race_schedule_mpk_order": ([_P, ctypes.c_int32, ctypes.c_int32, _I32P], ctypes.c_int),
        "race_schedule_set_gs_quad": ([_P, ctypes.c_int32], ctypes.c_int),
        "race_schedule_set_gs_exec": ([_P, ctypes.c_int32], ctypes.c_int),
        "race_schedule_gs_flow_plan": ([_P, ctypes.c_int32, _I32P, _I64P, _I32P, _I32P, _I32P, _I32P, _I32P],
                                       ctypes.c_int),
        "race_symm_spmv": ([_P, _P, _P, _P], ctypes.c_int),
        "race_symm_spmm": ([_P, ctypes.c_int32, _P, _P, _P], ctypes.c_int),
        "race_symm_spmm_traced": ([_P, ctypes.c_int32, _P, _P, _P, _P], ctypes.c_int),
        "race_permute": ([_P, ctypes.c_int32, _P, _P, ctypes.c_int32, _P], ctypes.c_int),
        "race_csr_create": ([ctypes.c_int32, _I32P, _I32P, _DP, ctypes.c_int32, ctypes.POINTER(_P)], ctypes.c_int),
        "race_csr_spmv": ([_P, _P, _P, _P], ctypes.c_int),
        "race_atomic_create": ([ctypes.c_int32, _I32P, _I32P, _DP, ctypes.c_int32, ctypes.POINTER(_P)],
                               ctypes.c_int),
        "race_symm_spmv_noalloc": ([_P, _P, _P, _P], ctypes.c_int),
        "race_symm_gs": ([_P, _P, _P, ctypes.c_int32, _P], ctypes.c_int),
        "race_symm_kacz": ([_P, _P, _P, ctypes.c_int32, ctypes.c_double, _P], ctypes.c_int),
        "race_vendor_create": ([ctypes.c_int32, _I32P, _I32P, _DP, ctypes.c_int32, ctypes.c_int32,
                                ctypes.POINTER(_P)], ctypes.c_int),
        "race_vendor_spmv": ([_P, _P, _P, _P], ctypes.c_int),
        "race_vendor_destroy": ([_P], None),
        "race_stream_read": ([_P, ctypes.c_int64, _P, ctypes.c_int32, _P], ctypes.c_int),
        "race_stream_copy": ([_P, _P, ctypes.c_int64, ctypes.c_int32, _P], ctypes.c_int),
        "race_symm_spmv_atomic": ([_P, _P, _P, _P], ctypes.c_int),
        "race_csr_destroy": ([_P], None),
        "race_last_error": ([], ctypes.c_char_p),
        "race_batch_create": ([ctypes.c_int32, ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)],
                              ctypes.c_int),
        "race_batch_bind": ([_P, ctypes.POINTER(_P), ctypes.POINTER(_P)], ctypes.c_int),
        "race_batch_run": ([_P, ctypes.c_int32, _P], ctypes.c_int),
        "race_batch_check": ([_P], ctypes.c_int),
        "race_batch_info": ([_P, _I32P, _I32P, _I32P], ctypes.c_int),
        "race_batch_destroy": ([_P], None),
        "race_schedule_features": ([_P, ctypes.c_int32, _FP], ctypes.c_int),
        "race_schedule_simulate": ([_P, _FP, ctypes.c_double, ctypes.c_int32, _DP], ctypes.c_int),
        "race_schedule_flow_grid": ([_P, ctypes.c_int32, _I32P], ctypes.c_int),
        "race_mlp_forward_host": ([_FP, _FP, ctypes.c_int64, _FP], ctypes.c_int),
        "race_mlp_forward": ([_P, _P, ctypes.c_int64, _P, _P], ctypes.c_int),
        "race_mlp_workspace": ([ctypes.c_int64, _I64P], ctypes.c_int),
        "race_mlp_loss_grad": ([_P, _P, _P, ctypes.c_int64, _P, _P, _P, _P], ctypes.c_int),
        "race_mlp_adam": ([_P, _P, _P, _P, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, _P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(rc):
    if rc != RACE_OK:
        raise RaceError(rc, lib().race_last_error().decode())
    return rc


def _np_ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _dev_ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------------------
# same names as the C ABI

def race_params_default():
    p = race_params()
    check(lib().race_params_default(ctypes.byref(p)))
    return p


def race_build_schedule(n, row_ptr, col, val, params=None):
    """Host CRS arrays (upper triangle); returns an opaque handle (c_void_p)."""
    rp, c = _i32(row_ptr), _i32(col)
    if val is None:
        v = None
    elif np.iscomplexobj(val):  # complex values go over as interleaved (re, im) pairs
        v = np.ascontiguousarray(val, dtype=np.complex128).view(np.float64)
    else:
        v = np.ascontiguousarray(val, dtype=np.float64)
    h = _P()
    p = params if params is not None else race_params_default()
    check(lib().race_build_schedule(int(n), _np_ptr(rp, ctypes.c_int32), _np_ptr(c, ctypes.c_int32),
                                    None if v is None else _np_ptr(v, ctypes.c_double), ctypes.byref(p),
                                    ctypes.byref(h)))
    return h


def race_schedule_upload(h):
    check(lib().race_schedule_upload(h))


def race_schedule_destroy(h):
    lib().race_schedule_destroy(h)


def race_schedule_stats(h):
    st = race_stats()
    check(lib().race_schedule_stats(h, ctypes.byref(st)))
    return st.as_dict()


def race_schedule_perm(h, n):
    out = np.empty(n, dtype=np.int32)
    check(lib().race_schedule_perm(h, _np_ptr(out, ctypes.c_int32)))
    return out


def race_schedule_tree(h):
    cnt = ctypes.c_int32()
    check(lib().race_schedule_tree(h, ctypes.byref(cnt), None, None, None, None, None, None))
    k = cnt.value
    arrs = [np.empty(k, dtype=np.int32) for _ in range(6)]
    check(lib().race_schedule_tree(h, ctypes.byref(cnt), *[_np_ptr(a, ctypes.c_int32) for a in arrs]))
    return dict(zip(["stage", "color", "parent", "lo", "hi", "workers"], arrs))


def race_schedule_leaves(h):
    cnt = ctypes.c_int32()
    check(lib().race_schedule_leaves(h, ctypes.byref(cnt), None, None))
    node = np.empty(cnt.value, dtype=np.int32)
    phase = np.empty(cnt.value, dtype=np.int32)
    check(lib().race_schedule_leaves(h, ctypes.byref(cnt), _np_ptr(node, ctypes.c_int32),
                                     _np_ptr(phase, ctypes.c_int32)))
    return node, phase


def race_schedule_units(h, n):
    nu = ctypes.c_int32()
    nh = ctypes.c_int64()
    check(lib().race_schedule_units(h, ctypes.byref(nu), ctypes.byref(nh), *([None] * 7)))
    u, hcount = nu.value, nh.value
    unit_leaf = np.empty(u, dtype=np.int32)
    lo = np.empty(u, dtype=np.int32)
    hi = np.empty(u, dtype=np.int32)
    hptr = np.empty(u + 1, dtype=np.int64)
    halo = np.empty(hcount, dtype=np.int32)
    hflags = np.empty(hcount, dtype=np.uint8)
    rflags = np.empty(n, dtype=np.uint8)
    check(lib().race_schedule_units(h, ctypes.byref(nu), ctypes.byref(nh), _np_ptr(unit_leaf, ctypes.c_int32),
                                    _np_ptr(lo, ctypes.c_int32), _np_ptr(hi, ctypes.c_int32),
                                    _np_ptr(hptr, ctypes.c_int64), _np_ptr(halo, ctypes.c_int32),
                                    _np_ptr(hflags, ctypes.c_uint8), _np_ptr(rflags, ctypes.c_uint8)))
    return {"unit_leaf": unit_leaf, "lo": lo, "hi": hi, "halo_ptr": hptr, "halo": halo, "halo_flags": hflags,
            "row_flags": rflags}


def race_schedule_zero_list(h):
    cnt = ctypes.c_int64()
    check(lib().race_schedule_zero_list(h, ctypes.byref(cnt), None))
    out = np.empty(cnt.value, dtype=np.int32)
    check(lib().race_schedule_zero_list(h, ctypes.byref(cnt), _np_ptr(out, ctypes.c_int32)))
    return out


def race_schedule_check(h):
    check(lib().race_schedule_check(h))


def race_schedule_flow_takeovers(h):
    v = ctypes.c_int64(0)
    check(lib().race_schedule_flow_takeovers(h, ctypes.byref(v)))
    return int(v.value)


def race_schedule_flow_test_late(h, stride):
    check(lib().race_schedule_flow_test_late(h, int(stride)))


def race_schedule_set_ticket_order(h, ticket_unit):
    """ticket_unit: int32 array of n_units (units by ticket), or None for the default order."""
    if ticket_unit is None:
        check(lib().race_schedule_set_ticket_order(h, None))
        return
    t = np.ascontiguousarray(ticket_unit, dtype=np.int32)
    check(lib().race_schedule_set_ticket_order(h, _np_ptr(t, ctypes.c_int32)))


def race_schedule_order_tickets(h, cost):
    """cost: float32 array of n_units (critical-path order), or None for the default order."""
    if cost is None:
        check(lib().race_schedule_order_tickets(h, None))
        return
    c = np.ascontiguousarray(cost, dtype=np.float32)
    check(lib().race_schedule_order_tickets(h, _np_ptr(c, ctypes.c_float)))


def race_schedule_ticket_order(h, n_units):
    out = np.empty(n_units, dtype=np.int32)
    check(lib().race_schedule_ticket_order(h, _np_ptr(out, ctypes.c_int32)))
    return out


def race_symm_mpk(h, powers, x, Y, stream=None):
    """Y: device tensor of powers * n (power-major)."""
    check(lib().race_symm_mpk(h, int(powers), _dev_ptr(x), _dev_ptr(Y), _stream_ptr(stream)))


def race_symm_poly(h, coeffs, x, work, z, stream=None):
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    check(lib().race_symm_poly(h, int(c.size - 1), _np_ptr(c, ctypes.c_double), _dev_ptr(x),
                               _dev_ptr(work) if work is not None else None, _dev_ptr(z), _stream_ptr(stream)))


def race_schedule_read_deps(h, n_units):
    cnt = ctypes.c_int64()
    check(lib().race_schedule_read_deps(h, ctypes.byref(cnt), None, None))
    ptr = np.empty(n_units + 1, dtype=np.int32)
    idx = np.empty(cnt.value, dtype=np.int32)
    check(lib().race_schedule_read_deps(h, ctypes.byref(cnt), _np_ptr(ptr, ctypes.c_int32), _np_ptr(idx, ctypes.c_int32)))
    return ptr, idx


def race_schedule_set_mpk_order(h, lag_rows, cache_matrix):
    check(lib().race_schedule_set_mpk_order(h, int(lag_rows), int(cache_matrix)))


def race_schedule_mpk_order(h, powers, n_static, per_power):
    out = np.empty(int(powers) * int(per_power), dtype=np.int32)
    check(lib().race_schedule_mpk_order(h, int(powers), int(n_static), _np_ptr(out, ctypes.c_int32)))
    return out


def race_schedule_set_gs_exec(h, mode):
    check(lib().race_schedule_set_gs_exec(h, int(mode)))


def race_schedule_gs_flow_plan(h, direction):
    nt, nd = ctypes.c_int32(), ctypes.c_int64()
    check(lib().race_schedule_gs_flow_plan(h, int(direction), ctypes.byref(nt), ctypes.byref(nd), *([None] * 5)))
    arrs = [np.empty(nt.value, dtype=np.int32) for _ in range(3)]
    ptr = np.empty(nt.value + 1, dtype=np.int32)
    idx = np.empty(nd.value, dtype=np.int32)
    check(lib().race_schedule_gs_flow_plan(h, int(direction), ctypes.byref(nt), ctypes.byref(nd),
                                           *[_np_ptr(a, ctypes.c_int32) for a in arrs + [ptr, idx]]))
    return {"leaf0": arrs[0], "count": arrs[1], "back": arrs[2], "dep_ptr": ptr, "dep_idx": idx}


def race_schedule_set_gs_quad(h, min_leaves):
    check(lib().race_schedule_set_gs_quad(h, int(min_leaves)))


def race_symm_spmv(h, x, y, stream=None):
    check(lib().race_symm_spmv(h, _dev_ptr(x), _dev_ptr(y), _stream_ptr(stream)))


def race_symm_spmm(h, k, X, Y, stream=None):
    check(lib().race_symm_spmm(h, int(k), _dev_ptr(X), _dev_ptr(Y), _stream_ptr(stream)))


def race_symm_spmm_traced(h, k, X, Y, trace, stream=None):
    """trace: device int64 tensor of 4 * n_units (stamps are unsigned ticks)."""
    check(lib().race_symm_spmm_traced(h, int(k), _dev_ptr(X), _dev_ptr(Y), _dev_ptr(trace), _stream_ptr(stream)))


def race_permute(h, k, inp, out, to_permuted, stream=None):
    check(lib().race_permute(h, int(k), _dev_ptr(inp), _dev_ptr(out), int(bool(to_permuted)), _stream_ptr(stream)))


def race_csr_create(n, row_ptr, col, val, lanes_per_row=0):
    rp, c = _i32(row_ptr), _i32(col)
    v = np.ascontiguousarray(val, dtype=np.float64)
    h = _P()
    check(lib().race_csr_create(int(n), _np_ptr(rp, ctypes.c_int32), _np_ptr(c, ctypes.c_int32),
                                _np_ptr(v, ctypes.c_double), int(lanes_per_row), ctypes.byref(h)))
    return h


def race_csr_spmv(h, x, y, stream=None):
    check(lib().race_csr_spmv(h, _dev_ptr(x), _dev_ptr(y), _stream_ptr(stream)))


def race_atomic_create(n, row_ptr, col, val, lanes_per_row=0):
    rp, c = _i32(row_ptr), _i32(col)
    v = np.ascontiguousarray(val, dtype=np.float64)
    h = _P()
    check(lib().race_atomic_create(int(n), _np_ptr(rp, ctypes.c_int32), _np_ptr(c, ctypes.c_int32),
                                   _np_ptr(v, ctypes.c_double), int(lanes_per_row), ctypes.byref(h)))
    return h


GS_DIRECTIONS = {"forward": 0, "backward": 1, "symmetric": 2}


def race_symm_gs(h, b, x, direction="symmetric", stream=None):
    check(lib().race_symm_gs(h, _dev_ptr(b), _dev_ptr(x), GS_DIRECTIONS.get(direction, direction),
                             _stream_ptr(stream)))


def race_symm_kacz(h, b, x, direction="symmetric", omega=1.0, stream=None):
    check(lib().race_symm_kacz(h, _dev_ptr(b), _dev_ptr(x), GS_DIRECTIONS.get(direction, direction), float(omega),
                               _stream_ptr(stream)))


def race_symm_spmv_noalloc(h, x, y, stream=None):
    check(lib().race_symm_spmv_noalloc(h, _dev_ptr(x), _dev_ptr(y), _stream_ptr(stream)))


VENDOR_ALGS = {"adaptive": 0, "rowsplit": 1, "lrb": 2}


def race_vendor_create(n, row_ptr, col, val, symmetric_upper, alg):
    rp, c = _i32(row_ptr), _i32(col)
    v = np.ascontiguousarray(val, dtype=np.float64)
    h = _P()
    check(lib().race_vendor_create(int(n), _np_ptr(rp, ctypes.c_int32), _np_ptr(c, ctypes.c_int32),
                                   _np_ptr(v, ctypes.c_double), int(bool(symmetric_upper)),
                                   VENDOR_ALGS.get(alg, alg), ctypes.byref(h)))
    return h


def race_vendor_spmv(h, x, y, stream=None):
    check(lib().race_vendor_spmv(h, _dev_ptr(x), _dev_ptr(y), _stream_ptr(stream)))


def race_vendor_destroy(h):
    lib().race_vendor_destroy(h)


def race_stream_read(src, sink, grid, stream=None):
    """src: device tensor (its bytes are read); sink: device int32 tensor of >= 1 element."""
    check(lib().race_stream_read(_dev_ptr(src), src.numel() * src.element_size(), _dev_ptr(sink), int(grid),
                                 _stream_ptr(stream)))


def race_stream_copy(src, dst, grid, stream=None):
    if dst.numel() * dst.element_size() != src.numel() * src.element_size():
        raise ValueError("src and dst must hold the same number of bytes")
    check(lib().race_stream_copy(_dev_ptr(src), _dev_ptr(dst), src.numel() * src.element_size(), int(grid),
                                 _stream_ptr(stream)))


def race_symm_spmv_atomic(h, x, y, stream=None):
    check(lib().race_symm_spmv_atomic(h, _dev_ptr(x), _dev_ptr(y), _stream_ptr(stream)))


def race_csr_destroy(h):
    lib().race_csr_destroy(h)


def race_last_error():
    return lib().race_last_error().decode()


def race_batch_create(handles, k, threads=0):
    arr = (_P * len(handles))(*[h.value if isinstance(h, _P) else h for h in handles])
    b = _P()
    check(lib().race_batch_create(len(handles), arr, int(k), int(threads), ctypes.byref(b)))
    return b


def race_batch_bind(b, xs, ys):
    X = (_P * len(xs))(*[_dev_ptr(t).value for t in xs])
    Y = (_P * len(ys))(*[_dev_ptr(t).value for t in ys])
    check(lib().race_batch_bind(b, X, Y))


def race_batch_run(b, use_graph=True, stream=None):
    check(lib().race_batch_run(b, int(bool(use_graph)), _stream_ptr(stream)))


def race_batch_check(b):
    check(lib().race_batch_check(b))


def race_batch_info(b):
    t, g, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().race_batch_info(b, ctypes.byref(t), ctypes.byref(g), ctypes.byref(w)))
    return {"n_tickets": t.value, "grid": g.value, "wmax": w.value}


def race_batch_destroy(b):
    lib().race_batch_destroy(b)


def race_schedule_features(h, n_units, k=1):
    out = np.empty((n_units, MLP_INPUTS), dtype=np.float32)
    check(lib().race_schedule_features(h, int(k), _np_ptr(out, ctypes.c_float)))
    return out


def race_schedule_simulate(h, cost, flush_frac, workers):
    cost = np.ascontiguousarray(cost, dtype=np.float32)
    out = ctypes.c_double()
    check(lib().race_schedule_simulate(h, _np_ptr(cost, ctypes.c_float), float(flush_frac), int(workers),
                                       ctypes.byref(out)))
    return out.value


def race_schedule_flow_grid(h, k=1):
    g = ctypes.c_int32()
    check(lib().race_schedule_flow_grid(h, int(k), ctypes.byref(g)))
    return g.value


def race_mlp_forward_host(theta, X):
    theta = np.ascontiguousarray(theta, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, MLP_INPUTS)
    y = np.empty(X.shape[0], dtype=np.float32)
    check(lib().race_mlp_forward_host(_np_ptr(theta, ctypes.c_float), _np_ptr(X, ctypes.c_float), X.shape[0],
                                      _np_ptr(y, ctypes.c_float)))
    return y


def race_mlp_forward(theta, X, y, stream=None):
    check(lib().race_mlp_forward(_dev_ptr(theta), _dev_ptr(X), int(X.shape[0]), _dev_ptr(y), _stream_ptr(stream)))


def race_mlp_workspace(n):
    out = ctypes.c_int64()
    check(lib().race_mlp_workspace(int(n), ctypes.byref(out)))
    return out.value


def race_mlp_loss_grad(theta, X, t, workspace, grad, loss=None, stream=None):
    check(lib().race_mlp_loss_grad(_dev_ptr(theta), _dev_ptr(X), _dev_ptr(t), int(X.shape[0]), _dev_ptr(workspace),
                                   _dev_ptr(grad), _dev_ptr(loss) if loss is not None else None, _stream_ptr(stream)))


def race_mlp_adam(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(lib().race_mlp_adam(_dev_ptr(theta), _dev_ptr(grad), _dev_ptr(m), _dev_ptr(v), int(step), float(lr),
                              float(beta1), float(beta2), float(eps), _stream_ptr(stream)))
