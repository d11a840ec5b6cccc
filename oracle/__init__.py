"""CPU oracle for the over-decomposed stencil + column-physics update and its balancers.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the library.  It shares no code with the
HIP path.  The arithmetic lives in ``oracle.c`` (plain C, FP64, one thread);
this module compiles it with gcc on first use and wraps it with ctypes.
``exhaustive`` holds the brute-force balancer checks.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

GCC_FLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, no GPU)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = C.CDLL(build())
            i32, i64, u64, dbl = C.c_int32, C.c_int64, C.c_uint64, C.c_double
            P = C.POINTER
            lib.orc_splitmix64.argtypes = [u64, u64]
            lib.orc_splitmix64.restype = u64
            lib.orc_init_field.argtypes = [i64, u64, P(dbl)]
            lib.orc_kfield.argtypes = [i32, i32, i32, P(i64), P(i64), P(i64), P(i64), i64, dbl,
                                       i32, i32, P(i32)]
            lib.orc_stencil.argtypes = [i32, i32, i32, dbl, dbl, P(dbl), P(dbl)]
            lib.orc_physics.argtypes = [i32, i32, i32, dbl, P(i32), P(dbl)]
            lib.orc_chunk_work.argtypes = [i32, i32, i32, i32, P(i32), P(i32), i32, P(i32), P(dbl)]
            lib.orc_sum.argtypes = [i64, P(dbl)]
            lib.orc_sum.restype = dbl
            lib.orc_run.argtypes = [i32, i32, i32, i32, i32, i32, P(i32), P(i32), dbl, dbl, dbl,
                                    i32, P(i64), P(i64), P(i64), P(i64), dbl, i32, i32, i32, i64,
                                    i32, P(dbl), P(dbl), P(dbl), P(i32), i32]
            lib.orc_run.restype = i32
            lib.orc_physics_vertical.argtypes = [i32, i32, i32, dbl, P(i32), P(dbl)]
            lib.orc_greedy.argtypes = [P(dbl), i32, i32, P(i32)]
            lib.orc_greedy.restype = i32
            lib.orc_refine.argtypes = [P(dbl), P(i32), i32, i32, dbl, P(i32)]
            lib.orc_refine.restype = i32
            lib.orc_refineswap.argtypes = [P(dbl), P(i32), i32, i32, dbl, P(i32)]
            lib.orc_refineswap.restype = i32
            lib.orc_run_window.argtypes = [i32, i32, i32, i32, i32, i32, i32, dbl, dbl, dbl, i32,
                                           P(i64), P(i64), P(i64), P(i64), dbl, i32, i32, i64,
                                           i32, P(dbl), i32]
            lib.orc_run_window.restype = i32
            lib.orc_init_window.argtypes = [i32, i32, i32, i32, i32, i32, i32, i32, u64, P(dbl)]
            _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _hot_arrays(hot):
    h = np.zeros((4, max(1, len(hot))), dtype=np.int64)
    for i, (x0, y0, vx, vy) in enumerate(hot):
        h[:, i] = (x0, y0, vx, vy)
    return [np.ascontiguousarray(h[j]) for j in range(4)]


def splitmix64(seed: int, n: int) -> int:
    return int(_load().orc_splitmix64(seed, n))


def init_field(nx, ny, nz, seed, nfields=1) -> np.ndarray:
    q = np.empty((nfields, ny, nx, nz), dtype=np.float64)
    _load().orc_init_field(q.size, seed, _p(q, C.c_double))
    return q


def kfield(nx, ny, hot, t, sigma, kmin, kmax) -> np.ndarray:
    hx, hy, vx, vy = _hot_arrays(hot)
    k = np.empty((ny, nx), dtype=np.int32)
    _load().orc_kfield(nx, ny, len(hot), _p(hx, C.c_int64), _p(hy, C.c_int64),
                       _p(vx, C.c_int64), _p(vy, C.c_int64), t, sigma, kmin, kmax,
                       _p(k, C.c_int32))
    return k


def stencil(q, cc=0.4, cn=0.1) -> np.ndarray:
    """One Jacobi update of a single field q[ny, nx, nz]."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    ny, nx, nz = q.shape
    s = np.empty_like(q)
    _load().orc_stencil(nx, ny, nz, cc, cn, _p(q, C.c_double), _p(s, C.c_double))
    return s


def physics(s, k, eps=0.01, vertical=False) -> np.ndarray:
    s = np.array(s, dtype=np.float64, copy=True, order="C")
    ny, nx, nz = s.shape
    k = np.ascontiguousarray(k, dtype=np.int32)
    fn = _load().orc_physics_vertical if vertical else _load().orc_physics
    fn(nx, ny, nz, eps, _p(k, C.c_int32), _p(s, C.c_double))
    return s


def chunk_work(k, nz, xs, ys, alpha) -> np.ndarray:
    k = np.ascontiguousarray(k, dtype=np.int32)
    ny, nx = k.shape
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    px, py = len(xs) - 1, len(ys) - 1
    w = np.empty(px * py, dtype=np.float64)
    _load().orc_chunk_work(nx, nz, px, py, _p(xs, C.c_int32), _p(ys, C.c_int32), alpha,
                           _p(k, C.c_int32), _p(w, C.c_double))
    return w


def run(wl, q0=None, nsteps=None, t0=None):
    """Run a workload (paper_1310_4218_amd.workloads.Workload or any object with the same
    attributes) for nsteps steps from q0 (default: the seeded field).  Returns
    (q, work[T, C], cksum[T], k_last)."""
    nsteps = wl.steps if nsteps is None else nsteps
    t0 = wl.t0 if t0 is None else t0
    if q0 is None:
        q = init_field(wl.nx, wl.ny, wl.nz, wl.seed, wl.nfields)
    else:
        q = np.array(q0, dtype=np.float64, copy=True, order="C").reshape(
            wl.nfields, wl.ny, wl.nx, wl.nz)
    xs = np.ascontiguousarray(wl.xsplit, dtype=np.int32)
    ys = np.ascontiguousarray(wl.ysplit, dtype=np.int32)
    hx, hy, vx, vy = _hot_arrays(wl.hot)
    C_ = wl.px * wl.py
    work = np.zeros((max(nsteps, 1), C_), dtype=np.float64)
    ck = np.zeros(max(nsteps, 1), dtype=np.float64)
    klast = np.zeros((wl.ny, wl.nx), dtype=np.int32)
    rc = _load().orc_run(wl.nx, wl.ny, wl.nz, wl.nfields, wl.px, wl.py, _p(xs, C.c_int32),
                         _p(ys, C.c_int32), wl.c_center, wl.c_nbr, wl.eps, len(wl.hot),
                         _p(hx, C.c_int64), _p(hy, C.c_int64), _p(vx, C.c_int64),
                         _p(vy, C.c_int64), wl.sigma, wl.kmin, wl.kmax, wl.alpha_work, t0,
                         nsteps, _p(q, C.c_double), _p(work, C.c_double), _p(ck, C.c_double),
                         _p(klast, C.c_int32), int(getattr(wl, "vertical", 0)))
    if rc != 0:
        raise MemoryError("oracle run failed")
    return q, work[:nsteps], ck[:nsteps], klast


def greedy(w, S) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    m = np.empty(len(w), dtype=np.int32)
    if _load().orc_greedy(_p(w, C.c_double), len(w), S, _p(m, C.c_int32)) != 0:
        raise ValueError("bad balancer arguments")
    return m


def refine(w, old_map, S, thr) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    om = np.ascontiguousarray(old_map, dtype=np.int32)
    m = np.empty(len(w), dtype=np.int32)
    if _load().orc_refine(_p(w, C.c_double), _p(om, C.c_int32), len(w), S, thr,
                          _p(m, C.c_int32)) != 0:
        raise ValueError("bad balancer arguments")
    return m


def refineswap(w, old_map, S, thr) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    om = np.ascontiguousarray(old_map, dtype=np.int32)
    m = np.empty(len(w), dtype=np.int32)
    if _load().orc_refineswap(_p(w, C.c_double), _p(om, C.c_int32), len(w), S, thr,
                              _p(m, C.c_int32)) != 0:
        raise ValueError("bad balancer arguments")
    return m


def greedy_then_refineswap(w, old_map, S, thr, first) -> np.ndarray:
    """The balancer policy of Experiment C (Section VI, Table V; Section VII): the
    first rebalance of a run uses Greedy, every later one RefineSwap from the
    map in force."""
    return greedy(w, S) if first else refineswap(w, old_map, S, thr)


def init_window(wl, ox, oy, nxw, nyw, f=0) -> np.ndarray:
    """Seeded initial values of a window of field f: local column (x, y) is global column
    ((ox + x) mod nx, (oy + y) mod ny)."""
    q = np.empty((nyw, nxw, wl.nz), dtype=np.float64)
    _load().orc_init_window(nxw, nyw, wl.nz, ox, oy, wl.nx, wl.ny, f, wl.seed, _p(q, C.c_double))
    return q


def run_window(wl, q0, ox, oy, nsteps, t0=None) -> np.ndarray:
    """Advance a window (see init_window) by nsteps steps starting at time t0 (default
    wl.t0); only columns at least nsteps away from the window border are exact."""
    t0 = wl.t0 if t0 is None else t0
    q = np.array(q0, dtype=np.float64, copy=True, order="C")
    nyw, nxw, nz = q.shape
    hx, hy, vx, vy = _hot_arrays(wl.hot)
    rc = _load().orc_run_window(nxw, nyw, nz, ox, oy, wl.nx, wl.ny, wl.c_center, wl.c_nbr, wl.eps,
                                len(wl.hot), _p(hx, C.c_int64), _p(hy, C.c_int64),
                                _p(vx, C.c_int64), _p(vy, C.c_int64), wl.sigma, wl.kmin,
                                wl.kmax, t0, nsteps, _p(q, C.c_double),
                                int(getattr(wl, "vertical", 0)))
    if rc != 0:
        raise MemoryError("oracle window run failed")
    return q


def block_map(C_, S) -> np.ndarray:
    """Initial placement: contiguous blocks of chunks per slot (Table V's first row)."""
    if C_ >= S:
        return np.array([(c * S) // C_ for c in range(C_)], dtype=np.int32)
    return np.arange(C_, dtype=np.int32)


def slot_loads(w, m, S) -> np.ndarray:
    L = np.zeros(S, dtype=np.float64)
    for c in range(len(w)):
        L[m[c]] += w[c]
    return L


def imbalance(w, m, S) -> float:
    """max over slots of the slot load divided by the average slot load W/S."""
    L = slot_loads(w, m, S)
    W = float(np.sum(w))
    return float(L.max() / (W / S)) if W > 0 else 1.0
