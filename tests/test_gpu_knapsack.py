"""Knapsack choice of the index set (Sec. 4.2) from GPU solves: on the
regular annulus the profits of the details Delta_b fall with |b| (the paper
observes equal profit along b1 + b2 = const, which makes the chosen set the
sparse-grid simplex); the set chosen for the budget of the level-6 sparse
grid is that simplex, and the GPU combination over it matches the oracle's
combination of its own solves."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    import paper_1707_09598_amd as S
    S.lib()
    assert torch.cuda.is_available()
    return S


def test_knapsack_index_set_regular_annulus(S):
    from paper_1707_09598_amd import knapsack
    from quadrature import annulus_quadrature
    wl = W.config("cfg2", w=8, f=W._field("annulus_rhs", 0.0), a=W._field("const", 1.0),
                  exact=W._field("annulus_u"))
    xi, wq = annulus_quadrature(128)
    cand = [b for b in np.ndindex(9, 9) if sum(b) <= 8]
    kw = dict(precision="fp64", tol=1e-12, maxit=600, max_refine=3)
    prof = knapsack.profits(wl, cand, xi, wq, kw)
    # profits fall with |b| away from the axes: the median profit of each
    # anti-diagonal decreases, and the spread along one is far smaller than
    # the fall over the candidate range
    med = [np.median([prof[b]["profit"] for b in prof if sum(b) == s and min(b) >= 1]) for s in range(2, 9)]
    log("  median profit per |b| (interior indices):", " ".join(f"{m:.2e}" for m in med))
    assert all(med[i + 1] < med[i] for i in range(len(med) - 1))
    spread = max(max(prof[b]["profit"] for b in prof if sum(b) == s and min(b) >= 1) /
                 min(prof[b]["profit"] for b in prof if sum(b) == s and min(b) >= 1) for s in range(2, 9))
    assert spread < med[0] / med[-1]
    # a budget of the level-6 sparse grid's summed unknowns
    sg6 = [b for b in cand if sum(b) <= 6]
    budget = sum(prof[b]["cost"] for b in sg6)
    I = knapsack.dantzig(prof, budget)
    log(f"  chosen set ({len(I)} indices): {I}")
    Is = set(I)
    assert all(tuple(c) in Is for b in I for c in np.ndindex(*[v + 1 for v in b]))
    # the paper's observation: the chosen set is the sparse-grid simplex
    assert Is == set(sg6)
    P = S.Plan(wl, index_set=I)
    P.bind()
    P.assemble()
    P.solve(**kw)
    pts, _ = W.eval_points(2, 4096, seed=31)
    u = P.combine(pts).cpu().numpy()
    Po = O.Problem(wl)
    ref = np.zeros(len(pts))
    for lv, c in zip(P.levels, P.coef):
        coef, _ = Po.solve([int(v) for v in lv])
        ref += c * Po.eval([int(v) for v in lv], coef, pts)
    assert np.linalg.norm(u - ref) <= 1e-10 * np.linalg.norm(ref)


def test_knapsack_index_set_low_regular_annulus(S):
    """On the low-regular problem (f = 1) the paper finds optimal sets closer
    to a rectangle than to a triangle, with profits decaying more slowly in
    the second (angular) direction: most mirrored pairs b = (i, j), i < j,
    have the larger profit on the angular side, and the set chosen for the
    budget of the level-6 sparse grid is not that simplex but reaches beyond
    |b| = 6."""
    from paper_1707_09598_amd import knapsack
    from quadrature import annulus_quadrature, low_regular_annulus
    wl = low_regular_annulus(W, 9)
    xi, wq = annulus_quadrature(128)
    cand = [b for b in np.ndindex(8, 8) if sum(b) <= 9]
    kw = dict(precision="fp64", tol=1e-12, maxit=600, max_refine=3)
    prof = knapsack.profits(wl, cand, xi, wq, kw)
    pairs = [(i, j) for (i, j) in cand if i < j and (j, i) in prof]
    angular = sum(prof[(i, j)]["profit"] > prof[(j, i)]["profit"] for (i, j) in pairs)
    log(f"  angular side larger in {angular} of {len(pairs)} mirrored pairs")
    assert angular >= 0.7 * len(pairs)
    sg6 = [b for b in cand if sum(b) <= 6]
    budget = sum(prof[b]["cost"] for b in sg6)
    I = knapsack.dantzig(prof, budget)
    log(f"  chosen set ({len(I)} indices): {I}")
    assert set(I) != set(sg6) and max(sum(b) for b in I) > 6
