"""ctypes mirror of include/lbgrid.h (argument marshalling only).

The library is the in-tree ``liblbgrid.so`` next to this file; if it has not
been built, every entry point raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbgrid.so")

LB_OK, LB_E_INVAL, LB_E_STATE, LB_E_HIP, LB_E_NOMEM, LB_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
LB_FP32, LB_FP32_KAHAN, LB_FP64 = 0, 1, 2
LB_PLAIN, LB_PERSISTENT, LB_PLAIN_GRAPH, LB_PERSISTENT_EAGER = 0, 1, 2, 3
LB_LOAD_WORK, LB_LOAD_TIME = 0, 1
LB_GREEDY, LB_REFINE, LB_REFINESWAP, LB_GREEDY_THEN_REFINESWAP = 0, 1, 2, 3
LB_MAX_HOT = 4
LB_NBUF = 3

PRECISIONS = {"fp32": LB_FP32, "fp32_kahan": LB_FP32_KAHAN, "kahan": LB_FP32_KAHAN, "fp64": LB_FP64}
MODES = {"plain": LB_PLAIN, "persistent": LB_PERSISTENT, "plain_graph": LB_PLAIN_GRAPH,
         "persistent_eager": LB_PERSISTENT_EAGER}
SOURCES = {"work": LB_LOAD_WORK, "time": LB_LOAD_TIME}
STRATEGIES = {"greedy": LB_GREEDY, "refine": LB_REFINE, "refineswap": LB_REFINESWAP,
              "greedy_then_refineswap": LB_GREEDY_THEN_REFINESWAP}

I32P = C.POINTER(C.c_int32)
DBLP = C.POINTER(C.c_double)


class LbConfig(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nfields", C.c_int32),
        ("px", C.c_int32), ("py", C.c_int32),
        ("xsplit", I32P), ("ysplit", I32P),
        ("precision", C.c_int32),
        ("c_center", C.c_double), ("c_nbr", C.c_double), ("eps", C.c_double),
        ("nhot", C.c_int32),
        ("hx0", C.c_int32 * LB_MAX_HOT), ("hy0", C.c_int32 * LB_MAX_HOT),
        ("hvx", C.c_int32 * LB_MAX_HOT), ("hvy", C.c_int32 * LB_MAX_HOT),
        ("sigma", C.c_double),
        ("kmin", C.c_int32), ("kmax", C.c_int32), ("alpha_work", C.c_int32),
        ("nslots", C.c_int32), ("nqueues", C.c_int32), ("wg_per_queue", C.c_int32),
        ("tile_x", C.c_int32), ("tile_y", C.c_int32),
        ("steal", C.c_int32), ("graph_steps", C.c_int32), ("item_split", C.c_int32),
        ("stage_rows", C.c_int32), ("physics", C.c_int32), ("tail_split", C.c_int32),
        ("item_alpha", C.c_int32), ("march", C.c_int32), ("queue_order", C.c_int32), ("hot_cut", C.c_int32), ("item_grid", C.c_int32), ("fuse_steps", C.c_int32), ("lane_levels", C.c_int32), ("xcd_group", C.c_int32), ("t0", C.c_int64), ("seed", C.c_uint64),
    ]


class LbBuffers(C.Structure):
    _fields_ = [("ptr", C.c_void_p * LB_NBUF), ("bytes", C.c_size_t * LB_NBUF)]


class LbStats(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("nchunks", C.c_int32), ("ntiles", C.c_int32),
        ("nrows", C.c_int32), ("nitems", C.c_int32), ("nslots", C.c_int32),
        ("nqueues", C.c_int32), ("nwg", C.c_int32), ("block", C.c_int32),
        ("tile_x", C.c_int32), ("tile_y", C.c_int32),
        ("clock_hz", C.c_double), ("last_checksum", C.c_double),
        ("measured_steps", C.c_int64),
        ("host_balance_us", C.c_double), ("host_plan_us", C.c_double),
        ("busy_slots", C.c_int32), ("block2", C.c_int32),
        ("block3", C.c_int32), ("pad1", C.c_int32),
    ]


# Every symbol the header declares, with its ctypes signature.
SIGNATURES = {
    "lb_config_default": (None, [C.POINTER(LbConfig)]),
    "lb_query": (C.c_int, [C.POINTER(LbConfig), C.POINTER(LbBuffers)]),
    "lb_grid_init": (C.c_int, [C.POINTER(LbConfig), C.POINTER(LbBuffers), C.c_void_p, C.c_void_p,
                               C.POINTER(C.c_void_p)]),
    "lb_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "lb_measure": (C.c_int, [C.c_void_p, C.c_int32, DBLP, C.c_int32]),
    "lb_measure_begin": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "lb_field_sum_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p]),
    "lb_measure_end": (C.c_int, [C.c_void_p, DBLP]),
    "lb_rebalance": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, DBLP, I32P, I32P, DBLP]),
    "lb_set_map": (C.c_int, [C.c_void_p, I32P, DBLP]),
    "lb_fields": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, DBLP]),
    "lb_stats": (C.c_int, [C.c_void_p, C.POINTER(LbStats)]),
    "lb_wg_busy": (C.c_int, [C.c_void_p, DBLP, C.c_int32]),
    "lb_wg_timeline": (C.c_int, [C.c_void_p, DBLP, C.c_int32]),
    "lb_visits": (C.c_int, [C.c_void_p, I32P, C.c_int32, C.c_int32]),
    "lb_checksums": (C.c_int, [C.c_void_p, DBLP, C.c_int32, I32P]),
    "lb_balance_host": (C.c_int, [DBLP, I32P, C.c_int32, C.c_int32, C.c_int32, C.c_double, I32P,
                                  I32P]),
    "lb_destroy": (None, [C.c_void_p]),
    "lb_last_error": (C.c_char_p, [C.c_void_p]),
    "lb_abi_version": (C.c_int, []),
    "lb_config_bytes": (C.c_size_t, []),
    "lb_stats_bytes": (C.c_size_t, []),
}

_lock = threading.Lock()
_lib = None


class LbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbgrid error {code}: {msg}")
        self.code = code


def lib() -> C.CDLL:
    """Load liblbgrid.so (raises if it is missing: there is no other path)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise FileNotFoundError(
                    f"{LIB_PATH} is not built; run `python -m paper_1310_4218_amd.build_lib`")
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            if L.lb_config_bytes() != C.sizeof(LbConfig) or L.lb_stats_bytes() != C.sizeof(LbStats):
                raise RuntimeError("lbgrid struct layout mismatch between library and binding")
            _lib = L
    return _lib


def check(rc: int, ctx=None) -> None:
    if rc != LB_OK:
        msg = lib().lb_last_error(ctx)
        raise LbError(rc, msg.decode() if msg else "")


def ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def make_config(nx, ny, nz, px, py, xsplit=None, ysplit=None, *, nfields=1, precision="fp32",
                c_center=0.4, c_nbr=0.1, eps=0.01, hot=(), sigma=8.0, kmin=1, kmax=1,
                alpha_work=32, nslots=256, nqueues=0, wg_per_queue=0, tile_x=0, tile_y=0, steal=1,
                graph_steps=10, item_split=2, stage_rows=0, physics=0, tail_split=4, item_alpha=-1,
                march=0, queue_order=0, hot_cut=200, item_grid=0, fuse_steps=0, lane_levels=0, xcd_group=0, t0=0, seed=0):
    """Build an LbConfig; returns (config, keepalive) -- keep both until the call returns."""
    cfg = LbConfig()
    lib().lb_config_default(C.byref(cfg))
    cfg.nx, cfg.ny, cfg.nz, cfg.nfields = nx, ny, nz, nfields
    cfg.px, cfg.py = px, py
    keep = []
    if xsplit is not None:
        xs = np.ascontiguousarray(xsplit, dtype=np.int32)
        keep.append(xs)
        cfg.xsplit = ptr(xs, C.c_int32)
    if ysplit is not None:
        ys = np.ascontiguousarray(ysplit, dtype=np.int32)
        keep.append(ys)
        cfg.ysplit = ptr(ys, C.c_int32)
    cfg.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    cfg.c_center, cfg.c_nbr, cfg.eps = c_center, c_nbr, eps
    if len(hot) > LB_MAX_HOT:
        raise ValueError("at most 4 hotspots")
    cfg.nhot = len(hot)
    for i, (x0, y0, vx, vy) in enumerate(hot):
        cfg.hx0[i], cfg.hy0[i], cfg.hvx[i], cfg.hvy[i] = x0, y0, vx, vy
    cfg.sigma, cfg.kmin, cfg.kmax = float(sigma), kmin, kmax
    cfg.alpha_work = alpha_work
    cfg.nslots, cfg.nqueues, cfg.wg_per_queue = nslots, nqueues, wg_per_queue
    cfg.tile_x, cfg.tile_y = tile_x, tile_y
    cfg.steal, cfg.graph_steps, cfg.item_split = steal, graph_steps, item_split
    cfg.stage_rows = stage_rows
    cfg.physics = physics
    cfg.tail_split = tail_split
    cfg.item_alpha = item_alpha
    cfg.march = march
    cfg.queue_order = queue_order
    cfg.hot_cut = hot_cut
    cfg.item_grid = item_grid
    cfg.fuse_steps = fuse_steps
    cfg.lane_levels = lane_levels
    cfg.xcd_group = xcd_group
    cfg.t0, cfg.seed = t0, seed
    return cfg, keep


def config_from_workload(wl, **overrides):
    kw = dict(nfields=wl.nfields, c_center=wl.c_center, c_nbr=wl.c_nbr, eps=wl.eps, hot=wl.hot,
              sigma=wl.sigma, kmin=wl.kmin, kmax=wl.kmax, alpha_work=wl.alpha_work,
              nslots=wl.nslots, t0=wl.t0, seed=wl.seed, physics=getattr(wl, "vertical", 0))
    kw.update(overrides)
    return make_config(wl.nx, wl.ny, wl.nz, wl.px, wl.py, wl.xsplit, wl.ysplit, **kw)


def query(cfg) -> list:
    b = LbBuffers()
    check(lib().lb_query(C.byref(cfg), C.byref(b)))
    return [int(b.bytes[i]) for i in range(LB_NBUF)]


def balance_host(loads, S, strategy="greedy", old_map=None, threshold=1.05):
    w = np.ascontiguousarray(loads, dtype=np.float64)
    m = np.empty(len(w), dtype=np.int32)
    nm = C.c_int32(0)
    om = None if old_map is None else np.ascontiguousarray(old_map, dtype=np.int32)
    st = STRATEGIES[strategy] if isinstance(strategy, str) else int(strategy)
    rc = lib().lb_balance_host(ptr(w, C.c_double), None if om is None else ptr(om, C.c_int32),
                               len(w), S, st, threshold, ptr(m, C.c_int32), C.byref(nm))
    check(rc)
    return m, int(nm.value)
