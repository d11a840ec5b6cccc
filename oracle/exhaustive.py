"""Brute-force checks for the balancers (test infrastructure only).

``optimum`` enumerates every chunk->slot map (S**C of them, C <= 10) and returns
the smallest possible maximum slot load: the exact optimum of the makespan
problem that GreedyLB approximates (Section VI, Experiment A).  Greedy's
largest-first rule is list scheduling in decreasing order, so its result is
bounded by (4/3 - 1/(3S)) * optimum (Graham, "Bounds on multiprocessing timing
anomalies", SIAM J. Appl. Math. 1969).
"""
from __future__ import annotations

import itertools

import numpy as np


def optimum(w, S) -> float:
    w = [float(x) for x in w]
    C = len(w)
    if C == 0:
        return 0.0
    best = float("inf")
    # chunk 0 can be pinned to slot 0 by symmetry of the slots
    for rest in itertools.product(range(S), repeat=C - 1):
        L = [0.0] * S
        L[0] = w[0]
        for c, s in enumerate(rest, start=1):
            L[s] += w[c]
        m = max(L)
        if m < best:
            best = m
    return best


def max_load(w, m, S) -> float:
    L = np.zeros(S)
    for c, s in enumerate(m):
        L[s] += w[c]
    return float(L.max())


def refine_postconditions(w, old_map, new_map, S, thr):
    """Conditions every correct move-only refinement must meet; returns a list of
    violated conditions (empty when all hold)."""
    bad = []
    w = [float(x) for x in w]
    C = len(w)
    W = sum(w)
    limit = (W / S) * thr
    L0 = [0.0] * S
    L1 = [0.0] * S
    for c in range(C):
        L0[old_map[c]] += w[c]
        L1[new_map[c]] += w[c]
    if max(L1) > max(L0) + 1e-9 * max(1.0, max(L0)):
        bad.append("maximum load increased")
    moved = [c for c in range(C) if old_map[c] != new_map[c]]
    if len(moved) > C:
        bad.append("more moves than chunks")
    for c in moved:
        if L1[new_map[c]] > limit * (1 + 1e-12):
            bad.append(f"chunk {c} landed on a slot above the limit")
        if L0[old_map[c]] <= limit:
            bad.append(f"chunk {c} left a slot that was not overloaded")
    # a slot still above the limit must have no chunk that fits onto the least loaded slot
    q = int(np.argmin(L1))
    for p in range(S):
        if L1[p] > limit:
            for c in range(C):
                if new_map[c] == p and p != q and L1[q] + w[c] <= limit:
                    bad.append(f"slot {p} still overloaded although chunk {c} fits on slot {q}")
    return bad
