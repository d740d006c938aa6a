"""Training data and training loop of the learned preconditioner.

Pairs (r, e) with A e = r come from the iterates of the plain FD-preconditioned
CG on the training samples: x* from a converged solve, x_k after k iterations,
r_k = b - A x_k and e_k = x* - x_k.  Every arithmetic step runs in the
library's kernels (residual, fast diagonalisation, pair normalisation,
network forward/backward, Adam); this module only orders the calls and
batches tensors of equal grid shape.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import Network, make_pair


def grid_shape(plan, comp: int) -> Tuple[int, int, int]:
    """(n1, n2, n3) interior unknowns per direction of component comp."""
    wl = plan.wl
    p, r = int(wl["p"]), int(wl["r"])
    ni = []
    for lev in plan.levels[comp]:
        nb = p + 1 + (2 ** int(lev) - 1) * (p - r)
        ni.append(nb - 2)
    while len(ni) < 3:
        ni.append(1)
    return tuple(ni)


def collect_pairs(plan, snapshots: Sequence[int] = (0, 1, 2, 3, 4, 6, 8, 12, 16), tol: float = 1e-12,
                  pairs: Dict[int, List] = None, head: int = 0, scaled: bool = True) -> Dict[int, List]:
    """Append the pairs of one assembled plan (one coefficient sample) to
    pairs[comp] as (x [3, n], t [n]) FP32 device tensors.  scaled selects the
    preconditioner the network corrects (the diagonally scaled one or the
    plain pencil), as in the solves it is used in."""
    pairs = {} if pairs is None else pairs
    fd = "fds64" if scaled else "fd64"
    plan.solve(precision="fp64", tol=tol, maxit=1000, max_refine=3, scaled=scaled)
    xs = [plan.coeffs(c) for c in range(plan.ncomp)]
    la = [plan.loga(c) for c in range(plan.ncomp)]
    for k in snapshots:
        if k > 0:
            # k plain iterations, then the residual replacement ends the solve
            plan.solve(precision="fp64", tol=1e-30, maxit=k, max_refine=1, check=False, scaled=scaled)
        for c in range(plan.ncomp):
            xk = plan.coeffs(c) if k > 0 else None
            if xk is None:
                import torch
                zero = torch.zeros_like(xs[c])
                r = plan.apply(c, "res64", zero)
            else:
                r = plan.apply(c, "res64", xk)
            zfd = plan.apply(c, fd, r)
            x, t = make_pair(r, zfd, la[c], xs[c], xk, head=head)
            pairs.setdefault(c, []).append((x, t))
    return pairs


def train(net: Network, pairs: Dict[int, List], shapes: Dict[int, Tuple[int, int, int]], steps: int,
          lr: float = 2e-3, batch: int = 16, seed: int = 1) -> List[float]:
    """Adam on the mean squared error; each step takes one component's pairs
    (equal shapes), a seeded random batch of them."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = sorted(pairs)
    losses = []
    for step in range(steps):
        c = keys[int(rng.integers(len(keys)))]
        P = pairs[c]
        sel = rng.choice(len(P), size=min(batch, len(P)), replace=False)
        n1, n2, n3 = shapes[c]
        X = torch.stack([P[i][0] for i in sel]).view(len(sel), 3, n3, n2, n1).contiguous()
        T = torch.stack([P[i][1] for i in sel]).view(len(sel), 1, n3, n2, n1).contiguous()
        loss = net.gradient(X, T)
        net.adam(lr=lr)
        if step % 50 == 0 or step == steps - 1:
            losses.append(float(loss.item()))
    return losses


def evaluate(net: Network, pairs: Dict[int, List], shapes: Dict[int, Tuple[int, int, int]],
             batch: int = 64) -> float:
    """Mean training loss over every pair (no parameter update), weighted by
    the number of unknowns."""
    import torch
    tot, cnt = 0.0, 0
    for c in sorted(pairs):
        n1, n2, n3 = shapes[c]
        P = pairs[c]
        for i in range(0, len(P), batch):
            sel = P[i:i + batch]
            X = torch.stack([q[0] for q in sel]).view(len(sel), 3, n3, n2, n1).contiguous()
            T = torch.stack([q[1] for q in sel]).view(len(sel), 1, n3, n2, n1).contiguous()
            tot += float(net.gradient(X, T).item()) * T.numel()
            cnt += T.numel()
    return tot / max(cnt, 1)


def init_params(channels: Sequence[int], seed: int = 0) -> np.ndarray:
    """He-initialised weights, zero biases, in the library's flat layout; the
    last layer starts at zero so that the untrained preconditioner is FD."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for li, (cin, cout) in enumerate(zip(channels[:-1], channels[1:])):
        std = np.sqrt(2.0 / (27 * cin))
        w = rng.standard_normal(cout * cin * 27) * std
        if li == len(channels) - 2:
            w[:] = 0.0
        out.append(w)
        out.append(np.zeros(cout))
    return np.concatenate(out).astype(np.float32)
