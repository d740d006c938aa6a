"""Choice of the combination index set from profits (Sec. 4.2 of the paper),
one-shot (knapsack) and iterative (dimension-adaptive).

For every multi-index b of a downward-closed set the detail
Delta_b(u) = sum over z in {0,1}^d of (-1)^|z| u_(b-z) (u of a negative level
is zero) measures what grid b adds to the combination; its L2 norm is the
revenue of b and the unknowns of grid b its cost, profit = revenue / cost.

All arithmetic runs in the library: one plan over the whole set with every
index planned (``keep_all``), one batched solve of all its grids, and the
detail norms by ``iga_sg_detail_norms`` (grid values at the caller's
quadrature points, details and weighted sums on the GPU).  This module only
orders those calls and makes the host-side choices:

  - ``dantzig``: the knapsack heuristic of Sec. 4.2, multi-indices in
    decreasing profit while the summed cost fits a budget, then closed
    downward;
  - ``adaptive``: the iterative variant (the dimension-adaptive scheme of
    Gerstner and Griebel, 2003): start from {0}; repeatedly move the
    admissible index of largest profit from the active set to the old set and
    make its forward neighbours active once all their backward neighbours are
    old; stop at a cost budget or when the active revenues sum below a
    tolerance.
"""
from __future__ import annotations

from itertools import product
from typing import Any, Dict, Iterable, List, Optional, Tuple

import numpy as np

from . import Plan

Index = Tuple[int, ...]


def _box(b: Index) -> List[Index]:
    return list(product(*[range(v + 1) for v in b]))


def _check_closed(cand: List[Index]) -> None:
    cs = set(cand)
    for b in cand:
        for k in range(len(b)):
            if b[k] > 0:
                c = list(b)
                c[k] -= 1
                if tuple(c) not in cs:
                    raise ValueError("index set is not downward closed")


def profits(wl: Dict[str, Any], candidates: Iterable[Index], xi, wq, solve_kw: Dict[str, Any]):
    """Revenue ||Delta_b(u)||_L2 (quadrature weights wq at the parametric
    points xi, including |det DF|), cost (unknowns of grid b) and profit of
    every b of a downward-closed set: one plan, one batched solve, the
    details on the GPU."""
    cand = sorted({tuple(int(v) for v in b) for b in candidates})
    _check_closed(cand)
    P = Plan(wl, index_set=cand, keep_all=True)
    P.bind()
    P.assemble()
    P.solve(**solve_kw)
    rev = P.detail_norms(xi, wq)
    out = {}
    for c in range(P.ncomp):
        b = tuple(int(v) for v in P.levels[c])
        cost = int(P.ndof[c])
        out[b] = {"revenue": float(rev[c]), "cost": cost, "profit": float(rev[c]) / cost}
    return out


def dantzig(prof: Dict[Index, Dict[str, float]], budget: int) -> List[Index]:
    """Multi-indices in decreasing profit while the summed cost stays within
    the budget, then closed downward (every predecessor of a chosen index is
    added)."""
    chosen, spent = set(), 0
    for b in sorted(prof, key=lambda b: (-prof[b]["profit"], b)):
        if spent + prof[b]["cost"] > budget:
            break
        chosen.add(b)
        spent += prof[b]["cost"]
    closed = set()
    for b in chosen:
        closed.update(_box(b))
    return sorted(closed)


def adaptive(wl: Dict[str, Any], xi, wq, solve_kw: Dict[str, Any], budget: int, tol: float = 0.0,
             max_level: int = 12, max_steps: int = 500):
    """Iterative (dimension-adaptive) choice of a downward-closed index set.

    Returns (index set, trace); the set is the old set plus the active set at
    the stop (downward closed), the trace one entry per step: the index moved
    to the old set, its profit, the cost of the set and the sum of the active
    revenues (the scheme's error indicator)."""
    d = int(wl["dim"])
    zero = tuple([0] * d)
    old: set = set()
    active: set = {zero}
    trace = []
    for _ in range(max_steps):
        prof = profits(wl, sorted(old | active), xi, wq, solve_kw)
        cost = sum(prof[b]["cost"] for b in old | active)
        indicator = sum(prof[b]["revenue"] for b in active)
        if not active or cost > budget or indicator <= tol:
            break
        best = max(sorted(active), key=lambda b: prof[b]["profit"])
        active.remove(best)
        old.add(best)
        for k in range(d):
            c = list(best)
            c[k] += 1
            c = tuple(c)
            if c[k] > max_level or c in old or c in active:
                continue
            if all(tuple(c[j] - (j == i) for j in range(d)) in old for i in range(d) if c[i] > 0):
                active.add(c)
        trace.append({"index": best, "profit": prof[best]["profit"], "cost": cost, "indicator": indicator})
    return sorted(old | active), trace
