"""Seeded synthetic inputs for the over-decomposed grid workloads.

This module only *describes* inputs: grid sizes, chunk split points, hotspot
parameters, seeds and run lengths.  It holds none of the method's arithmetic
(no stencil, no column loop, no cost field, no balancer), so both the HIP
library and the CPU oracle can take their inputs from it without sharing any
computation.

The workloads follow the paper's synthetic application (Section IV and
Section VI): a 3D Jacobi-like stencil over a 2D-decomposed grid of
sub-domains (Section IV, 2D domain decomposition), followed by a per-column
"physics" loop whose trip count is controlled by an array that is moved
across the domain over time (Section VI, Fig. 4 and the load-control array C).
The paper fixes only the shape of this application; the concrete sizes below
are synthetic stand-ins chosen to span cache-resident and HBM-bound regimes.

Split points for uneven chunks come from a seeded Dirichlet draw: widths are
``N * dirichlet([alpha_d] * p)`` rounded to integers, then forced to be at
least one cell wide (forward pass) and to end at ``N`` (backward pass).
"""
from __future__ import annotations

import copy
from dataclasses import dataclass, field, asdict
from typing import List, Optional, Tuple

import numpy as np

MAX_HOT = 4


@dataclass
class Workload:
    """One synthetic problem instance (grid, decomposition, cost field, run)."""

    name: str
    nx: int
    ny: int
    nz: int
    px: int
    py: int
    xsplit: List[int]
    ysplit: List[int]
    # hotspots: (x0, y0, vx, vy) in integer cells and cells/step
    hot: List[Tuple[int, int, int, int]]
    sigma: float
    kmin: int
    kmax: int
    steps: int
    nfields: int = 1
    c_center: float = 0.4
    c_nbr: float = 0.1
    eps: float = 0.01
    alpha_work: int = 32
    nslots: int = 256
    rebalance_every: int = 0          # 0 = never
    strategy: str = "greedy"          # greedy | refine | refineswap | greedy_then_refineswap
    threshold: float = 1.05
    t0: int = 0
    seed: int = 0
    split_kind: str = "equal"
    alpha_d: float = 0.0
    vertical: int = 0                 # 1: column physics with the vertical dependency

    @property
    def nchunks(self) -> int:
        return self.px * self.py

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def replace(self, **kw) -> "Workload":
        w = copy.deepcopy(self)
        for k, v in kw.items():
            setattr(w, k, v)
        return w

    def to_dict(self) -> dict:
        return asdict(self)


def equal_split(n: int, p: int) -> List[int]:
    """Equal split points s_i = floor(i*n/p), i = 0..p."""
    if p < 1 or p > n:
        raise ValueError(f"cannot split {n} cells into {p} parts")
    return [(i * n) // p for i in range(p + 1)]


def dirichlet_split(n: int, p: int, rng: np.random.Generator, alpha_d: float) -> List[int]:
    """Uneven split points from a Dirichlet(alpha_d) draw of part widths."""
    if p < 1 or p > n:
        raise ValueError(f"cannot split {n} cells into {p} parts")
    w = rng.dirichlet([alpha_d] * p)
    cs = np.cumsum(w)
    s = [0] + [int(np.rint(n * cs[i])) for i in range(p - 1)] + [n]
    for i in range(1, p + 1):          # every part at least one cell wide
        s[i] = max(s[i], s[i - 1] + 1)
    s[p] = n
    for i in range(p - 1, 0, -1):      # and still ending at n
        s[i] = min(s[i], s[i + 1] - 1)
    return s


def make_splits(nx: int, ny: int, px: int, py: int, kind: str = "equal",
                alpha_d: float = 20.0, seed: int = 0) -> Tuple[List[int], List[int]]:
    if kind == "equal":
        return equal_split(nx, px), equal_split(ny, py)
    if kind == "dirichlet":
        rng = np.random.default_rng(seed)
        xs = dirichlet_split(nx, px, rng, alpha_d)
        ys = dirichlet_split(ny, py, rng, alpha_d)
        return xs, ys
    raise ValueError(f"unknown split kind {kind!r}")


def _mk(name, nx, ny, nz, px, py, hot, sigma, kmin, kmax, steps, *, split="equal",
        alpha_d=20.0, split_seed=0, seed=0, **kw) -> Workload:
    xs, ys = make_splits(nx, ny, px, py, split, alpha_d, split_seed)
    return Workload(name=name, nx=nx, ny=ny, nz=nz, px=px, py=py, xsplit=xs, ysplit=ys,
                    hot=list(hot), sigma=float(sigma), kmin=kmin, kmax=kmax, steps=steps,
                    seed=seed, split_kind=split, alpha_d=alpha_d if split != "equal" else 0.0,
                    **kw)


def small() -> Workload:
    """64x64x32, 4x4 equal chunks, static centre hotspot, sigma 8, k in 1..32, 10 steps."""
    return _mk("small-64x64x32-c16", 64, 64, 32, 4, 4, [(32, 32, 0, 0)], 8.0, 1, 32, 10,
               seed=1001, nslots=4)


def moving() -> Workload:
    """256x256x64, 8x8 equal chunks, hotspot moving +1 x-cell/step, sigma 24, k in 1..200,
    100 steps, loads measured every step, GreedyLB onto 256 slots every 10 steps."""
    return _mk("moving-256x256x64-c64", 256, 256, 64, 8, 8, [(128, 128, 1, 0)], 24.0, 1, 200,
               100, seed=1002, nslots=256, rebalance_every=10, strategy="greedy")


def sweep(vp: int) -> Workload:
    """512x512x64 with vp in {16, 64, 256, 1024} uneven (Dirichlet) chunks, static centre
    hotspot (sigma 48, k in 1..200), 20 steps."""
    p = int(round(vp ** 0.5))
    if p * p != vp:
        raise ValueError("vp must be a square")
    return _mk(f"sweep-512x512x64-c{vp}", 512, 512, 64, p, p, [(256, 256, 0, 0)], 48.0, 1, 200,
               20, split="dirichlet", alpha_d=20.0, split_seed=2003, seed=1003, nslots=256,
               rebalance_every=10, strategy="greedy")


def precision() -> Workload:
    """1024x1024x64, 32x32 equal chunks, two static hotspots (sigma 32, k in 1..500),
    50 steps."""
    return _mk("precision-1024x1024x64-c1024", 1024, 1024, 64, 32, 32,
               [(256, 256, 0, 0), (768, 768, 0, 0)], 32.0, 1, 500, 50, seed=1004, nslots=256,
               rebalance_every=10, strategy="greedy")


def large() -> Workload:
    """2048x2048x80, 64x64 uneven (Dirichlet) chunks, hotspot moving diagonally
    2 cells/step (sigma 64, k in 1..400), 200 steps, RefineLB(1.05) every 10 steps."""
    return _mk("large-2048x2048x80-c4096", 2048, 2048, 80, 64, 64, [(1024, 1024, 2, 2)], 64.0,
               1, 400, 200, split="dirichlet", alpha_d=20.0, split_seed=2005, seed=1005,
               nslots=256, rebalance_every=10, strategy="refine", threshold=1.05)


def fields(nf: int) -> Workload:
    """The paper's per-step volume: 1024x1024x40 with nf fields (50 in Experiments B and C,
    100 in Table I and Experiment A), 16 chunks as 1 x 16 bands along y (the 1D
    decomposition of Fig. 5), 4 slots (P = 4), one wide hotspot (sigma 256, k in 1..3, so
    about twice the physics inside it) moving along y by 16 cells/step, 40 steps, Greedy
    on the first rebalance and RefineSwap after (Experiment C) every 10 steps."""
    return _mk(f"fields{nf}-1024x1024x40-c16", 1024, 1024, 40, 1, 16, [(512, 0, 0, 16)], 256.0, 1, 3,
               40, seed=1006, nslots=4, rebalance_every=10, strategy="greedy_then_refineswap",
               nfields=nf)


PRESETS = {
    "small": small,
    "moving": moving,
    "sweep16": lambda: sweep(16),
    "sweep64": lambda: sweep(64),
    "sweep256": lambda: sweep(256),
    "sweep1024": lambda: sweep(1024),
    "precision": precision,
    "large": large,
    "fields50": lambda: fields(50),
    "fields100": lambda: fields(100),
}


def get(name: str) -> Workload:
    try:
        return PRESETS[name]()
    except KeyError:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(PRESETS)}") from None


def shrink(w: Workload, nx: int, ny: int, nz: Optional[int] = None, steps: Optional[int] = None,
           px: Optional[int] = None, py: Optional[int] = None) -> Workload:
    """A smaller instance with the same structure (hotspots and sigma scaled with nx)."""
    px = px or min(w.px, nx)
    py = py or min(w.py, ny)
    f = nx / w.nx
    hot = [(int(hx * f) % nx, int(hy * ny / w.ny) % ny, vx, vy) for hx, hy, vx, vy in w.hot]
    xs, ys = make_splits(nx, ny, px, py, w.split_kind, w.alpha_d or 20.0, 7)
    return w.replace(name=w.name + f"-shrunk{nx}x{ny}", nx=nx, ny=ny, nz=nz or w.nz, px=px, py=py,
                     xsplit=xs, ysplit=ys, hot=hot, sigma=max(1.0, w.sigma * f),
                     steps=steps if steps is not None else w.steps)


def random_field(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """Uniform [-1, 1) values that are multiples of 2^-23 (exact in FP32 and FP64)."""
    rng = np.random.default_rng(seed)
    m = rng.integers(0, 1 << 24, size=shape, dtype=np.int64)
    return ((m - (1 << 23)) * 2.0 ** -23).astype(dtype)
