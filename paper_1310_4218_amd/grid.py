"""Python handle on one liblbgrid context.

PyTorch provides the device memory (three uint8 tensors sized by lb_query)
and the stream; every step of the computation runs in the library's HIP
kernels.  Nothing here computes anything about the method itself.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _abi
from ._abi import check, ptr


class Grid:
    """One over-decomposed grid on a GPU.

    ``wl`` is a :class:`paper_1310_4218_amd.workloads.Workload`; keyword
    overrides go to the library configuration (precision, nslots, nqueues, wg_per_queue,
    tile_x, tile_y, steal, graph_steps, ...).  ``init_field`` (optional) is a
    host or device array of nfields*ny*nx*nz values in the field precision.
    """

    def __init__(self, wl, device: str = "cuda:0", stream=None, init_field=None, **overrides):
        import torch

        self._torch = torch
        self.wl = wl
        self.device = torch.device(device)
        cfg, self._keep = _abi.config_from_workload(wl, **overrides)
        self.cfg = cfg
        sizes = _abi.query(cfg)
        self.precision = cfg.precision
        self.dtype = torch.float64 if cfg.precision == _abi.LB_FP64 else torch.float32
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._bufs = [torch.empty(max(n, 256), dtype=torch.uint8, device=self.device) for n in sizes]
        b = _abi.LbBuffers()
        for i, t in enumerate(self._bufs):
            if t.data_ptr() % 256:
                raise RuntimeError("device buffer is not 256-byte aligned")
            b.ptr[i] = t.data_ptr()
            b.bytes[i] = t.numel()
        init_ptr = None
        self._init_keep = None
        if init_field is not None:
            if isinstance(init_field, torch.Tensor):
                src = init_field.to(self.dtype).contiguous()
                init_ptr = src.data_ptr()
            else:
                src = np.ascontiguousarray(init_field,
                                           dtype=np.float64 if self.dtype == torch.float64
                                           else np.float32)
                init_ptr = src.ctypes.data
            n = src.numel() if isinstance(src, torch.Tensor) else src.size
            if n != wl.nfields * wl.ny * wl.nx * wl.nz:
                raise ValueError("init_field has the wrong number of values")
            self._init_keep = src
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = _abi.lib().lb_grid_init(C.byref(cfg), C.byref(b), C.c_void_p(self.stream.cuda_stream),
                                         C.c_void_p(init_ptr) if init_ptr else None, C.byref(h))
        check(rc)
        self._h = h
        self._init_keep = None
        st = self.stats()
        self.nchunks, self.ntiles, self.nslots, self.nwg = (st["nchunks"], st["ntiles"],
                                                            st["nslots"], st["nwg"])
        self.nqueues = st["nqueues"]
        self.nrows = st["nrows"]
        # output buffers of the per-window calls, allocated once (converting a
        # numpy array to a ctypes pointer costs microseconds per call)
        n = max(self.nchunks, 1)
        self._loads_out = (C.c_double * n)()
        self._map_out = (C.c_int32 * n)()
        self._nm_out = C.c_int32(0)
        self._lam_out = (C.c_double * 2)()

    # ---- lifecycle -------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _abi.lib().lb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("grid is closed")
        return self._h

    # ---- the method ------------------------------------------------------
    def step(self, n: int = 1, mode: str = "persistent") -> None:
        check(_abi.lib().lb_step(self.handle, int(n), _abi.MODES[mode]), self.handle)

    def measure(self, source: str = "work", reset: bool = True) -> np.ndarray:
        h = self.handle
        check(_abi.lib().lb_measure(h, _abi.SOURCES[source], self._loads_out, int(reset)), h)
        return np.frombuffer(self._loads_out, dtype=np.float64, count=self.nchunks).copy()

    def measure_begin(self, source: str = "work", reset: bool = True) -> None:
        """Enqueue the window's load snapshot without waiting (see measure_end)."""
        h = self.handle
        check(_abi.lib().lb_measure_begin(h, _abi.SOURCES[source], int(reset)), h)

    def measure_end(self) -> np.ndarray:
        """Wait for the snapshot of measure_begin only and return its loads."""
        h = self.handle
        check(_abi.lib().lb_measure_end(h, self._loads_out), h)
        return np.frombuffer(self._loads_out, dtype=np.float64, count=self.nchunks).copy()

    def rebalance(self, strategy: str = "greedy", threshold: float = 1.05,
                  loads: Optional[np.ndarray] = None):
        """Returns (map, nmigrated, (lambda_before, lambda_after))."""
        h = self.handle
        w = None if loads is None else np.ascontiguousarray(loads, dtype=np.float64)
        check(_abi.lib().lb_rebalance(h, _abi.STRATEGIES[strategy], threshold,
                                      None if w is None else ptr(w, C.c_double),
                                      self._map_out, C.byref(self._nm_out), self._lam_out), h)
        m = np.frombuffer(self._map_out, dtype=np.int32, count=self.nchunks).copy()
        return m, int(self._nm_out.value), (float(self._lam_out[0]), float(self._lam_out[1]))

    def set_map(self, m, cost=None) -> None:
        m = np.ascontiguousarray(m, dtype=np.int32)
        c = None if cost is None else np.ascontiguousarray(cost, dtype=np.float64)
        check(_abi.lib().lb_set_map(self.handle, ptr(m, C.c_int32),
                                    None if c is None else ptr(c, C.c_double)), self.handle)

    # ---- read-back -------------------------------------------------------
    def field(self, f: int = 0, device: str = "cpu"):
        """Field f of the current step as a (ny, nx, nz) tensor."""
        t = self._torch.empty((self.wl.ny, self.wl.nx, self.wl.nz), dtype=self.dtype,
                              device=device)
        check(_abi.lib().lb_fields(self.handle, f, C.c_void_p(t.data_ptr()),
                                   t.numel() * t.element_size(), None), self.handle)
        return t

    def checksum(self, f: int = 0) -> float:
        ck = C.c_double(0.0)
        check(_abi.lib().lb_fields(self.handle, f, None, 0, C.byref(ck)), self.handle)
        return float(ck.value)

    def stats(self) -> dict:
        s = _abi.LbStats()
        check(_abi.lib().lb_stats(self.handle, C.byref(s)), self.handle)
        return {k: getattr(s, k) for k, _ in _abi.LbStats._fields_}

    def wg_busy(self) -> np.ndarray:
        """Busy ticks per persistent workgroup, or per compute unit (unused slots 0) when
        balanced steps launch one workgroup per item."""
        n = self.stats()["busy_slots"]
        out = np.empty(n, dtype=np.float64)
        check(_abi.lib().lb_wg_busy(self.handle, ptr(out, C.c_double), n), self.handle)
        return out

    def wg_timeline(self) -> np.ndarray:
        """(nwg, 4) microseconds of the last persistent launch: start, first item start,
        last item end, exit, from the earliest workgroup start."""
        out = np.empty(4 * self.nwg, dtype=np.float64)
        check(_abi.lib().lb_wg_timeline(self.handle, ptr(out, C.c_double), 4 * self.nwg),
              self.handle)
        return out.reshape(self.nwg, 4)

    def visits(self, reset: bool = False) -> np.ndarray:
        out = np.empty(self.nrows, dtype=np.int32)
        check(_abi.lib().lb_visits(self.handle, ptr(out, C.c_int32), self.nrows, int(reset)),
              self.handle)
        return out

    def checksums(self, n: int = 1024) -> np.ndarray:
        out = np.empty(max(n, 1), dtype=np.float64)
        got = C.c_int32(0)
        check(_abi.lib().lb_checksums(self.handle, ptr(out, C.c_double), n, C.byref(got)),
              self.handle)
        return out[:got.value]
