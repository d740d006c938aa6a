"""Host-side checks of the full tensor plans (no GPU needed).

  - the 1D prolongations of a full tensor plan reproduce every coarse basis
    function from the fine ones, checked pointwise with the oracle's
    Cox-de Boor evaluation (an independent basis code), on uniform, radical
    and one-sided graded knots and for C^0 and C^{p-1} continuity;
  - full grids too large for the LDS of one workgroup plan as whole-device
    solves (2D level 8, 3D level 5) instead of failing, and the sparse-grid
    plan at the same level still plans per-workgroup solves.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def S():
    import paper_1707_09598_amd as S
    if not os.path.exists(S.LIB_PATH):
        from paper_1707_09598_amd import build as B
        B.build(force=False)
    S.lib()
    return S


@pytest.mark.parametrize("p,r,grading", [(3, 2, ("uniform", 1.0)), (2, 1, ("radical", 2.0)),
                                         (3, 0, ("uniform", 1.0)), (2, 0, ("toward0", 3.0)),
                                         (4, 3, ("toward1", 1.5))])
def test_prolongation_reproduces_coarse_basis(S, p, r, grading):
    J = 5
    wl = W.config("cfg1", p=p, r=r, w=J, grading=[grading, grading])
    P = S.Plan(wl, full=True)
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.random(200), [0.0, 1.0, 0.5, 0.25]])
    Uf = O.knots(p, r, J, grading[0], grading[1])
    Nf = np.array([O.basis_all(p, Uf, x)[0] for x in xs])[:, 1:-1]
    for lev in range(J):
        T = P.prolongation(0, lev)
        Uc = O.knots(p, r, lev, grading[0], grading[1])
        Nc = np.array([O.basis_all(p, Uc, x)[0] for x in xs])[:, 1:-1]
        assert T.shape == (Nf.shape[1], Nc.shape[1])
        assert np.abs(Nf @ T - Nc).max() < 1e-12, lev
    # direction 2 has the same knots here
    assert np.array_equal(P.prolongation(1, 2), P.prolongation(0, 2))


def test_prolongation_of_a_planted_mistake_fails():
    """The check above fails for a prolongation with one wrong entry (a
    mistake planted in a copy on the CPU)."""
    import paper_1707_09598_amd as S
    P = S.Plan(W.config("cfg1", p=2, r=1, w=4), full=True)
    T = P.prolongation(0, 2).copy()
    T[3, 1] += 0.25
    xs = np.linspace(0, 1, 101)
    Nf = np.array([O.basis_all(2, O.knots(2, 1, 4), x)[0] for x in xs])[:, 1:-1]
    Nc = np.array([O.basis_all(2, O.knots(2, 1, 2), x)[0] for x in xs])[:, 1:-1]
    assert np.abs(Nf @ T - Nc).max() > 1e-3


def test_large_full_grids_plan_as_whole_device_solves(S):
    P2 = S.Plan(W.config("cfg2", w=8), full=True)
    assert int(P2.ndof.sum()) == 257 * 257
    P3 = S.Plan(W.config("cfg3", w=5), full=True)
    assert int(P3.ndof.sum()) == 33 ** 3
    for P in (P2, P3):
        st = P.stats()
        assert st["lds_bytes"] <= 160 * 1024
    # the sparse grid of the same level keeps per-workgroup solves
    Ps = S.Plan(W.config("cfg2", w=8))
    assert Ps.stats()["lds_bytes"] <= 160 * 1024


def test_twolevel_rejects_plans_that_do_not_nest(S):
    import ctypes as C
    full = S.Plan(W.config("cfg2", w=6), full=True)
    other = S.Plan(W.config("cfg2", w=7))          # levels above the full grid's
    o = S._Opts(0, 1, 1e-10, 0.0, 100, 3, 0, 0, 0, 0, 0, 0, 0)
    rc = S.lib().iga_sg_solve_twolevel(full.h, other.h, C.byref(o), C.byref(o), 1, C.POINTER(S._Report)())
    assert rc == 1  # IGA_ERR_INVALID_ARG
    rc = S.lib().iga_sg_solve_twolevel(other.h, full.h, C.byref(o), C.byref(o), 1, C.POINTER(S._Report)())
    assert rc == 1
