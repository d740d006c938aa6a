"""Knapsack choice of the combination index set (Sec. 4.2 of the paper).

For every multi-index b of a downward-closed candidate set the detail
Delta_b(u) = sum over z in {0,1}^d of (-1)^|z| u_(b-z) (u of a negative level
is zero) is formed from the component solutions, its L2 norm is the revenue
and the unknowns of grid b the cost; the Dantzig heuristic takes the
multi-indices in decreasing revenue / cost until the budget is spent, and the
chosen set is closed downward so that the combination technique applies to
it (``Plan(wl, index_set=...)``).

Every component u_b is solved by the library (a plan whose index set is the
box below b holds grid b alone, coefficient 1) and evaluated by its
combination kernel at caller-given quadrature points; this module only
orders library calls and sums the evaluated values with the quadrature
weights."""
from __future__ import annotations

from itertools import product
from typing import Any, Dict, Iterable, List, Tuple

import numpy as np

from . import Plan

Index = Tuple[int, ...]


def _box(b: Index) -> List[Index]:
    return list(product(*[range(v + 1) for v in b]))


def component_values(wl: Dict[str, Any], indices: Iterable[Index], xi, solve_kw: Dict[str, Any]):
    """u_b at the points xi ([n, d] parametric) for every b, solved on the GPU;
    returns ({b: values}, {b: unknowns of grid b})."""
    import torch
    xt = torch.as_tensor(np.asarray(xi, dtype=np.float64), device="cuda").contiguous()
    vals, cost = {}, {}
    for b in indices:
        P = Plan(wl, index_set=_box(b))
        P.bind()
        P.assemble()
        P.solve(**solve_kw)
        vals[b] = P.combine(xt).cpu().numpy()
        cost[b] = int(P.ndof.sum())
    return vals, cost


def profits(wl: Dict[str, Any], candidates: Iterable[Index], xi, wq, solve_kw: Dict[str, Any]):
    """Revenue ||Delta_b(u)||_L2 (quadrature weights wq at the points xi,
    including |det DF|), cost (unknowns of grid b) and profit for every b of a
    downward-closed candidate set."""
    cand = sorted({tuple(int(v) for v in b) for b in candidates})
    cs = set(cand)
    for b in cand:
        for k in range(len(b)):
            if b[k] > 0:
                c = list(b)
                c[k] -= 1
                if tuple(c) not in cs:
                    raise ValueError("candidate set is not downward closed")
    vals, cost = component_values(wl, cand, xi, solve_kw)
    wq = np.asarray(wq, dtype=np.float64)
    out = {}
    d = len(cand[0])
    for b in cand:
        delta = np.zeros_like(vals[b])
        for z in range(1 << d):
            bz = tuple(b[k] - ((z >> k) & 1) for k in range(d))
            if min(bz) >= 0:
                delta += (-1) ** bin(z).count("1") * vals[bz]
        rev = float(np.sqrt(np.sum(wq * delta ** 2)))
        out[b] = {"revenue": rev, "cost": cost[b], "profit": rev / cost[b]}
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
