"""Autotuner of the launch shape: operator tile size (2D or 3D) and the
fast-diagonalisation task target of the plan, chosen by timing assembly +
solve of the caller's workload on the device.

Every candidate is a separate plan (the shape fixes the task lists and the
LDS layout); candidates the plan rejects (LDS over the limit) are skipped.
The timed region is the one the solve is measured on: assembly and the
persistent solve, HIP events on the plan's stream, the median of `repeats`
runs after one untimed run.
"""
from __future__ import annotations

from typing import Any, Dict, Iterable, List, Optional

import numpy as np

from . import IgaError, Plan

OP_TILE_2D = (64, 96, 128, 192, 256)
OP_TILE_3D = (128, 256, 512, 1024)
FD_TASKS = (256, 1 << 20)


def candidates(dim: int) -> List[Dict[str, int]]:
    if dim == 2:
        return [{"op_tile": t, "fd_tasks": f} for t in OP_TILE_2D for f in FD_TASKS]
    return [{"op_tile3": t} for t in OP_TILE_3D]


def time_shape(wl: Dict[str, Any], shape: Dict[str, int], solve_kw: Dict[str, Any], repeats: int = 3,
               nsamples: int = 1, fields: Optional[Dict[str, Any]] = None) -> float:
    """Median milliseconds of assembly + solve with the given launch shape."""
    import torch
    P = Plan(wl, nsamples=nsamples, shape=shape)
    P.bind()
    fields = fields or {}
    P.assemble(**fields)
    P.solve_async(**solve_kw)
    times = []
    for _ in range(repeats):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(P.stream)
        P.assemble(**fields)
        P.solve_async(**solve_kw)
        ev[1].record(P.stream)
        torch.cuda.synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    return float(np.median(times))


def autotune(wl: Dict[str, Any], solve_kw: Dict[str, Any], shapes: Optional[Iterable[Dict[str, int]]] = None,
             repeats: int = 3, nsamples: int = 1, fields: Optional[Dict[str, Any]] = None) -> Dict[str, Any]:
    """Best launch shape for the workload and solve options, with the timings
    of every candidate tried ({"shape": ..., "ms": ..., "tried": [...]})."""
    shapes = list(shapes) if shapes is not None else candidates(int(wl["dim"]))
    tried = []
    for sh in shapes:
        try:
            ms = time_shape(wl, sh, solve_kw, repeats, nsamples, fields)
        except IgaError:
            continue  # e.g. the tile does not fit in LDS
        tried.append({"shape": dict(sh), "ms": ms})
    if not tried:
        raise IgaError(1, "no launch shape could be planned")
    best = min(tried, key=lambda t: t["ms"])
    return {"shape": best["shape"], "ms": best["ms"], "tried": tried}
