"""Pins of the oracle's knot vectors, Gauss rules and Cox-de Boor basis.

Each check compares against something other than the oracle itself: numpy's
Gauss-Legendre rule, scipy's B-spline implementation, closed forms
(Bernstein polynomials, Greville reproduction) or finite differences.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle as O


@pytest.mark.parametrize("n", range(1, 11))
def test_gauss_legendre_matches_numpy(n):
    x, w = O.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, atol=1e-15, rtol=0)
    assert np.allclose(w, wr, atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_gauss_exact_degree(n):
    # exact for polynomials of degree 2n-1, not for degree 2n
    x, w = O.gauss_legendre(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14
    assert abs(np.dot(w, x ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-6


@pytest.mark.parametrize("p,r", [(1, 0), (2, 0), (2, 1), (3, 0), (3, 1), (3, 2), (4, 3)])
@pytest.mark.parametrize("level", [0, 1, 3, 5])
def test_knot_counts_and_multiplicity(p, r, level):
    U = O.knots(p, r, level)
    ne = 2 ** level
    n = len(U) - p - 1
    # n = p + 1 + (2^l - 1)(p - r); sum of multiplicities = n + p + 1 (Sec. 2.2)
    assert n == p + 1 + (ne - 1) * (p - r)
    zeta, mult = np.unique(U, return_counts=True)
    assert len(zeta) == ne + 1
    assert mult.sum() == n + p + 1
    assert mult[0] == mult[-1] == p + 1
    assert np.all(mult[1:-1] == p - r)
    assert np.allclose(zeta, np.arange(ne + 1) / ne, atol=1e-15)


@pytest.mark.parametrize("kind,gamma", [("uniform", 1.0), ("radical", 3.0), ("toward0", 3.0),
                                        ("toward1", 2.5)])
def test_grading_map(kind, gamma):
    t = np.linspace(0, 1, 1001)
    g = np.array([O.grade(kind, gamma, v) for v in t])
    assert g[0] == 0.0 and abs(g[-1] - 1.0) < 1e-15
    assert np.all(np.diff(g) > 0)
    # nested breakpoints: level l breakpoints are a subset of level l+1
    for lev in range(0, 6):
        a = np.unique(O.knots(2, 1, lev, kind, gamma))
        b = np.unique(O.knots(2, 1, lev + 1, kind, gamma))
        assert np.allclose(a, b[::2], atol=0, rtol=0)
    if kind == "radical":
        # the printed two-sided map is continuous at t = 1/2 with value 1/2
        assert abs(O.grade(kind, gamma, 0.5) - 0.5) < 1e-15
        assert abs(O.grade(kind, gamma, 0.25) - 2 ** (gamma - 1) * 0.25 ** gamma) < 1e-15
    # gamma = 1 recovers the uniform mesh
    assert abs(O.grade(kind, 1.0, 0.3) - 0.3) < 1e-15


def _scipy_basis(p, U, x, nu=0):
    n = len(U) - p - 1
    vals = np.zeros(n)
    for i in range(n):
        c = np.zeros(n)
        c[i] = 1.0
        s = BSpline(U, c, p, extrapolate=False)
        v = s(x, nu=nu)
        vals[i] = 0.0 if np.isnan(v) else v
    return vals


@pytest.mark.parametrize("p,r,level,grading", [
    (1, 0, 2, "uniform"), (2, 1, 3, "uniform"), (2, 0, 2, "radical"), (3, 2, 3, "uniform"),
    (3, 1, 2, "toward0"), (4, 3, 2, "toward1"), (3, 0, 1, "uniform")])
def test_cox_de_boor_matches_scipy(p, r, level, grading):
    U = O.knots(p, r, level, grading, 3.0)
    rng = np.random.default_rng(7)
    xs = np.concatenate([rng.random(40), [0.0, 0.5, 0.125]])
    for x in xs:
        v, d = O.basis_all(p, U, x)
        assert np.allclose(v, _scipy_basis(p, U, x), atol=1e-14, rtol=0)
        assert np.allclose(d, _scipy_basis(p, U, x, nu=1), atol=1e-11, rtol=1e-12)


@pytest.mark.parametrize("p,r", [(1, 0), (2, 1), (3, 2), (3, 0), (4, 2)])
def test_partition_of_unity_including_right_end(p, r):
    U = O.knots(p, r, 3, "radical", 2.0)
    for x in np.concatenate([np.linspace(0, 1, 97), [1.0]]):
        v, d = O.basis_all(p, U, x)
        assert abs(v.sum() - 1.0) < 1e-14
        assert v.min() >= -1e-15
        assert abs(d.sum()) < 1e-11
    # interpolatory at the first and last knot (Sec. 2.2)
    v0, _ = O.basis_all(p, U, 0.0)
    v1, _ = O.basis_all(p, U, 1.0)
    assert v0[0] == 1.0 and v1[-1] == 1.0


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_bernstein_on_single_element(p):
    U = O.knots(p, 0, 0)
    for x in np.linspace(0, 1, 11):
        v, _ = O.basis_all(p, U, x)
        ref = [math.comb(p, i) * x ** i * (1 - x) ** (p - i) for i in range(p + 1)]
        assert np.allclose(v, ref, atol=1e-15)


@pytest.mark.parametrize("p,r", [(2, 1), (3, 2), (3, 0), (2, 0)])
def test_greville_reproduces_linear(p, r):
    U = O.knots(p, r, 3, "toward0", 2.0)
    n = len(U) - p - 1
    grev = np.array([U[i + 1:i + p + 1].mean() for i in range(n)])
    for x in np.linspace(0, 1, 53):
        v, d = O.basis_all(p, U, x)
        assert abs(np.dot(grev, v) - x) < 1e-14
        assert abs(np.dot(grev, d) - 1.0) < 1e-12


@pytest.mark.parametrize("p,r", [(2, 1), (3, 2), (3, 1), (2, 0), (3, 0)])
def test_derivative_central_difference_and_continuity(p, r):
    U = O.knots(p, r, 2)
    h = 1e-6
    for x in [0.1, 0.33, 0.6, 0.9]:
        _, d = O.basis_all(p, U, x)
        vp, _ = O.basis_all(p, U, x + h)
        vm, _ = O.basis_all(p, U, x - h)
        assert np.allclose(d, (vp - vm) / (2 * h), atol=1e-7)
    # at an interior knot of multiplicity p - r: C^r.  Values are continuous for
    # r >= 0; first derivatives jump when r == 0 (C^0).
    z, eps = 0.5, 1e-11
    vl, dl = O.basis_all(p, U, z - eps)
    vr, dr = O.basis_all(p, U, z + eps)
    assert np.allclose(vl, vr, atol=1e-9)
    if r == 0:
        assert np.abs(dl - dr).max() > 1.0
    else:
        assert np.allclose(dl, dr, atol=1e-8)
