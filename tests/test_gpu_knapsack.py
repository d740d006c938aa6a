"""Choice of the index set from profits (Sec. 4.2) on the GPU: on the regular
annulus the profits of the details Delta_b fall with |b| (the paper observes
equal profit along b1 + b2 = const, which makes the chosen set the
sparse-grid simplex); the set chosen for the budget of the level-6 sparse
grid is that simplex, and the GPU combination over it matches the oracle's
combination of its own solves.  The detail norms themselves are checked
against details formed from the oracle's direct solves, and the iterative
(dimension-adaptive) variant is checked on both annulus problems."""
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


def test_profits_match_oracle_details(S):
    """The library's detail norms (one plan over the candidate set, one
    batched solve, details and weighted sums on the GPU) against the same
    details formed from the oracle's own direct solves of every grid."""
    from paper_1707_09598_amd import knapsack
    from quadrature import annulus_quadrature
    wl = W.config("cfg2", w=6, f=W._field("annulus_rhs", 0.0), a=W._field("const", 1.0),
                  exact=W._field("annulus_u"))
    xi, wq = annulus_quadrature(48)
    cand = [b for b in np.ndindex(7, 7) if sum(b) <= 6]
    kw = dict(precision="fp64", tol=1e-13, maxit=800, max_refine=3)
    prof = knapsack.profits(wl, cand, xi, wq, kw)
    Po = O.Problem(wl)
    vals = {}
    for b in cand:
        coef, _ = Po.solve(list(b))
        vals[b] = Po.eval(list(b), coef, xi)
    unorm = np.sqrt(np.sum(wq * vals[(6, 0)] ** 2))
    worst = 0.0
    for b in cand:
        delta = np.zeros(len(xi))
        for z in np.ndindex(2, 2):
            bz = (b[0] - z[0], b[1] - z[1])
            if min(bz) >= 0:
                delta += (-1) ** sum(z) * vals[bz]
        rev = np.sqrt(np.sum(wq * delta ** 2))
        err = abs(prof[b]["revenue"] - rev)
        worst = max(worst, err / (1e-10 * unorm + 1e-6 * rev))
        assert err <= 1e-10 * unorm + 1e-6 * rev, (b, prof[b]["revenue"], rev)
        assert prof[b]["cost"] == Po.ndof(list(b))
    log(f"  {len(cand)} detail norms, worst difference {worst:.2f} of the bar")


@pytest.mark.parametrize("problem", ["regular", "low_regular"])
def test_adaptive_index_set(S, problem):
    """The iterative (dimension-adaptive) choice: grow the set from {0} by
    largest profit until the summed unknowns reach the budget of the level-7
    sparse grid.  The set is downward closed, its error indicator (the
    active revenues) falls, the GPU combination over it equals the oracle's
    combination of its own solves, and its shape follows the problem: close
    to the simplex on the regular problem (it contains the level-5 simplex),
    deeper in the angular direction on the low-regular one."""
    from paper_1707_09598_amd import knapsack
    from quadrature import annulus_quadrature, low_regular_annulus
    if problem == "regular":
        wl = W.config("cfg2", w=7, f=W._field("annulus_rhs", 0.0), a=W._field("const", 1.0),
                      exact=W._field("annulus_u"))
    else:
        wl = low_regular_annulus(W, 7)
    xi, wq = annulus_quadrature(64)
    kw = dict(precision="fp64", tol=1e-12, maxit=800, max_refine=3)
    budget = int(S.Plan(wl).ndof.sum())
    I, trace = knapsack.adaptive(wl, xi, wq, kw, budget=budget, max_level=10)
    log(f"  {problem}: {len(trace)} steps, {len(I)} indices, indicator {trace[0]['indicator']:.2e} -> "
        f"{trace[-1]['indicator']:.2e}")
    log(f"  set: {I}")
    Is = set(I)
    assert all(tuple(c) in Is for b in I for c in np.ndindex(*[v + 1 for v in b]))
    assert trace[-1]["indicator"] < 1e-2 * trace[0]["indicator"]
    if problem == "regular":
        assert all(b in Is for b in np.ndindex(6, 6) if sum(b) <= 5)
    else:
        depth1 = max(b[0] for b in I if b[1] == 0)
        depth2 = max(b[1] for b in I if b[0] == 0)
        log(f"  depth along the axes: radial {depth1}, angular {depth2}")
        assert depth2 >= depth1
    P = S.Plan(wl, index_set=I)
    P.bind()
    P.assemble()
    P.solve(**kw)
    pts, _ = W.eval_points(2, 4096, seed=33)
    u = P.combine(pts).cpu().numpy()
    Po = O.Problem(wl)
    ref = np.zeros(len(pts))
    for lv, c in zip(P.levels, P.coef):
        coef, _ = Po.solve([int(v) for v in lv])
        ref += c * Po.eval([int(v) for v in lv], coef, pts)
    assert np.linalg.norm(u - ref) <= 1e-10 * np.linalg.norm(ref)
