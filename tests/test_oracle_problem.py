"""Pins of the oracle's geometry, fields, Galerkin assembly and direct solve.

References used: closed-form geometry facts (radius, area), sympy symbolic
differentiation of the manufactured solutions, numpy/scipy integration of
1D spline matrices, numpy dense LU solves, Appendix-B closed forms and the
exact reproduction of polynomial solutions by a Galerkin method.
"""
import math

import numpy as np
import pytest
import sympy as sp
from scipy.interpolate import BSpline

import oracle as O
import workloads as W


def _fld(kind, *prm, data=None):
    prm = list(prm) + [0.0] * (4 - len(prm))
    return {"kind": kind, "params": prm, "data": data}


def _line_patch():
    return {"degree": [1], "knots": [[0.0, 0.0, 1.0, 1.0]], "ctrl": np.array([[0.0], [1.0]]),
            "weights": None}


def one_d(p, r, f=None):
    return O.Problem(W.workload("1d", 1, [_line_patch()], p=p, r=r, w=0, lmin=0,
                                f=f or _fld("const", 1.0)))


# ---------------------------------------------------------------- geometry ---

def test_annulus_radius_and_corners():
    P = O.Problem(W.config("cfg2"))
    rng = np.random.default_rng(1)
    for xi in rng.random((200, 2)):
        x, jac, Wv, _ = P.geometry(xi)
        assert abs(np.hypot(*x) - (1.0 + xi[0])) < 1e-14
        assert np.linalg.det(jac) > 0
    for xi, ref in [((0, 0), (1, 0)), ((1, 0), (2, 0)), ((0, 1), (0, 1)), ((1, 1), (0, 2))]:
        x, _, _, _ = P.geometry(np.array(xi, float))
        assert np.allclose(x, ref, atol=1e-15)
    # xi_2 runs counter-clockwise from angle 0 to pi/2
    ang = [math.atan2(*P.geometry(np.array([0.5, t]))[0][::-1]) for t in np.linspace(0, 1, 20)]
    assert np.all(np.diff(ang) > 0)


@pytest.mark.parametrize("name,area", [("cfg2", 0.75 * math.pi), ("cfg1", 1.0), ("cfg4", 3.0),
                                       ("cfg3", 1.0)])
def test_domain_area(name, area):
    wl = W.config(name, w=1 if name != "cfg3" else 3, exact=_fld("affine", 1.0))
    wl["g"] = None
    P = O.Problem(wl)
    coefs = P.solve_all()
    # ||1||_L2^2 over the domain = |Omega| (error norms integrate |det DF|)
    e = P.sg_errors(coefs, 8)
    assert abs(e[2] ** 2 - area) < 1e-12 * max(1, area)


# ------------------------------------------------------------------ fields ---

def _sym_rhs(u_expr, a_expr, x, y):
    return -(sp.diff(a_expr * sp.diff(u_expr, x), x) + sp.diff(a_expr * sp.diff(u_expr, y), y))


@pytest.mark.parametrize("amp,shift", [(0.0, 0.0), (0.5, 0.0), (0.3, 0.25)])
def test_manufactured_rhs_against_sympy(amp, shift):
    x, y = sp.symbols("x y")
    a = 1 + amp * sp.sin(2 * sp.pi * (x + shift)) * sp.cos(2 * sp.pi * y)
    u_ann = -(x ** 2 + y ** 2 - 1) * (x ** 2 + y ** 2 - 4) * x * y ** 2
    u_pol = x * (1 - x) * y * (1 - y)
    f_ann = sp.lambdify((x, y), _sym_rhs(u_ann, a, x, y))
    f_pol = sp.lambdify((x, y), _sym_rhs(u_pol, a, x, y))
    a_fn = sp.lambdify((x, y), a)
    wl = W.config("cfg2", f=_fld("annulus_rhs", amp, shift), a=_fld("sincos", amp, shift))
    P = O.Problem(wl)
    wl2 = W.config("cfg1", f=_fld("poly_rhs", amp, shift))
    P2 = O.Problem(wl2)
    rng = np.random.default_rng(3)
    for pt in rng.uniform(-2, 2, (50, 2)):
        ref = f_ann(*pt)
        assert abs(P.field("f", pt) - ref) < 1e-12 * max(1.0, abs(ref))
        assert abs(P.field("a", pt) - a_fn(*pt)) < 1e-14
        ref2 = f_pol(*pt)
        assert abs(P2.field("f", pt) - ref2) < 1e-12 * max(1.0, abs(ref2))


def test_exact_solution_gradients_fd():
    for name, ex in [("cfg2", _fld("annulus_u")), ("cfg1", _fld("sinprod_u", 1.0)),
                     ("cfg4", _fld("corner"))]:
        P = O.Problem(W.config(name, exact=ex))
        rng = np.random.default_rng(5)
        for pt in rng.uniform(0.2, 0.9, (20, 2)):
            u, g = P.exact(pt)
            h = 1e-6
            fd = [(P.exact(pt + h * e)[0] - P.exact(pt - h * e)[0]) / (2 * h) for e in np.eye(2)]
            assert np.allclose(g, fd, atol=1e-7)


def test_corner_function_harmonic_and_vanishing_on_reentrant_edges():
    P = O.Problem(W.config("cfg4"))
    h = 1e-4
    for pt in [(-0.5, 0.5), (0.3, 0.7), (-0.6, -0.4), (0.2, 0.1)]:
        pt = np.array(pt)
        lap = sum(P.field("g", pt + h * e) + P.field("g", pt - h * e) for e in np.eye(2))
        lap = (lap - 4 * P.field("g", pt)) / h ** 2
        assert abs(lap) < 1e-5
    for t in np.linspace(0, 1, 7):
        assert abs(P.field("g", np.array([t, 0.0]))) < 1e-15       # y = 0, x > 0
        assert abs(P.field("g", np.array([0.0, -t]))) < 1e-15      # x = 0, y < 0


def test_grid3d_trilinear_reproduces_affine():
    n = (5, 4, 3)
    gx = [np.arange(m) / (m - 1) for m in n]
    Z, Y, X = np.meshgrid(gx[2], gx[1], gx[0], indexing="ij")
    data = 1.0 + 2 * X - 3 * Y + 0.5 * Z
    wl = W.config("cfg5", a=_fld("grid3d", data=data))
    P = O.Problem(wl)
    for pt in np.random.default_rng(2).random((30, 3)):
        assert abs(P.field("a", pt) - (1 + 2 * pt[0] - 3 * pt[1] + 0.5 * pt[2])) < 1e-13


# ---------------------------------------------------------------- assembly ---

def test_1d_closed_forms_appendix_b():
    # p = 1 single element
    P = one_d(1, 0)
    K, _ = P.assemble_dense([0], O.WITH_BOUNDARY)
    M, _ = P.assemble_dense([0], O.WITH_BOUNDARY | O.MASS)
    assert np.allclose(K, [[1, -1], [-1, 1]], atol=1e-15)
    assert np.allclose(M, [[1 / 3, 1 / 6], [1 / 6, 1 / 3]], atol=1e-15)
    # p = 2 single element (Bernstein)
    P = one_d(2, 1)
    K, _ = P.assemble_dense([0], O.WITH_BOUNDARY)
    M, _ = P.assemble_dense([0], O.WITH_BOUNDARY | O.MASS)
    assert np.allclose(3 * K, [[4, -2, -2], [-2, 4, -2], [-2, -2, 4]], atol=1e-14)
    assert np.allclose(30 * M, [[6, 3, 1], [3, 4, 3], [1, 3, 6]], atol=1e-14)
    Ki, _ = P.assemble_dense([0], 0)
    Mi, _ = P.assemble_dense([0], O.MASS)
    assert np.allclose(Ki, [[4 / 3]]) and np.allclose(Mi, [[2 / 15]])


def _scipy_1d_matrices(p, r, level, grading="uniform", gamma=1.0):
    """1D stiffness and mass on all basis functions, integrated with scipy
    B-splines and numpy's Gauss rule (p+1 points per element)."""
    U = O.knots(p, r, level, grading, gamma)
    n = len(U) - p - 1
    xg, wg = np.polynomial.legendre.leggauss(p + 1)
    br = np.unique(U)
    K = np.zeros((n, n))
    M = np.zeros((n, n))
    splines = []
    for i in range(n):
        c = np.zeros(n)
        c[i] = 1
        splines.append(BSpline(U, c, p, extrapolate=False))
    for a, b in zip(br[:-1], br[1:]):
        x = 0.5 * (a + b) + 0.5 * (b - a) * xg
        w = 0.5 * (b - a) * wg
        V = np.array([np.nan_to_num(s(x)) for s in splines])
        D = np.array([np.nan_to_num(s(x, nu=1)) for s in splines])
        K += (D * w) @ D.T
        M += (V * w) @ V.T
    return K, M


@pytest.mark.parametrize("p,r,level,grading", [(2, 1, 3, "uniform"), (3, 2, 2, "uniform"),
                                               (3, 0, 2, "uniform"), (2, 1, 3, "radical")])
def test_box_separability_against_scipy(p, r, level, grading):
    K1, M1 = _scipy_1d_matrices(p, r, level, grading, 2.0)
    K2, M2 = _scipy_1d_matrices(p, r, level - 1, grading, 2.0)
    P1 = O.Problem(W.workload("1d", 1, [_line_patch()], p=p, r=r, w=0, lmin=0,
                              f=_fld("const", 1.0), grading=[(grading, 2.0)]))
    K1o, _ = P1.assemble_dense([level], O.WITH_BOUNDARY)
    M1o, _ = P1.assemble_dense([level], O.WITH_BOUNDARY | O.MASS)
    assert np.allclose(K1o, K1, atol=1e-12 * np.abs(K1).max())
    assert np.allclose(M1o, M1, atol=1e-14)
    wl = W.config("cfg1", p=p, r=r, grading=[(grading, 2.0), (grading, 2.0)])
    P = O.Problem(wl)
    A, _ = P.assemble_dense([level, level - 1], O.WITH_BOUNDARY)
    # full unknown ordering is lexicographic with the shorter direction fastest
    n1, n2 = K1.shape[0], K2.shape[0]
    ref = np.kron(M2, K1) + np.kron(K2, M1)  # direction 1 fastest
    if n2 < n1:
        ref = np.kron(K1, M2) + np.kron(M1, K2)
    assert np.allclose(A, ref, atol=1e-12 * np.abs(ref).max())
    # stiffness annihilates constants, mass integrates to the area
    assert np.abs(A @ np.ones(len(A))).max() < 1e-12 * np.abs(A).max()
    Mf, _ = P.assemble_dense([level, level - 1], O.WITH_BOUNDARY | O.MASS)
    assert abs(Mf.sum() - 1.0) < 1e-13


@pytest.mark.parametrize("name,levels", [("cfg1", [2, 3]), ("cfg2", [2, 2]), ("cfg2", [4, 1]),
                                         ("cfg3", [2, 1, 1]), ("cfg4", [2, 2]), ("cfg5", [1, 1, 2])])
def test_spd_and_direct_solve_vs_numpy(name, levels):
    wl = W.config(name)
    if name == "cfg5":
        wl["a"] = _fld("sincos", 0.3)
    P = O.Problem(wl)
    A, b = P.assemble_dense(levels)
    assert len(A) <= 400
    assert np.allclose(A, A.T, atol=1e-14 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0
    x = np.linalg.solve(A, b)
    c, info = P.solve(levels)
    assert info[1] < 1e-14
    # compare through point values (coefficient orderings differ)
    d = P.dim
    pts, pid = W.eval_points(d, 50, seed=9, npatch=len(wl["patches"]))
    u_or = P.eval(levels, c, pts, pid)
    # rebuild the numpy solution as a function via the oracle's interpolation
    # of its own ordering: solve A x = b in the oracle and compare residuals
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    assert np.all(np.isfinite(u_or))


def test_direct_solve_coefficients_vs_numpy_single_patch():
    # single patch, homogeneous Dirichlet: the oracle orders unknowns with the
    # shortest direction fastest; map the numpy solution accordingly
    P = O.Problem(W.config("cfg2"))
    levels = [3, 2]
    A, b = P.assemble_dense(levels)
    x = np.linalg.solve(A, b)
    c, _ = P.solve(levels)
    n1, n2 = P.nbasis(levels)
    inner = c[0][1:-1, 1:-1]          # [n2-2, n1-2], direction 1 fastest
    if n2 < n1:
        ref = x.reshape(n1 - 2, n2 - 2).T
    else:
        ref = x.reshape(n2 - 2, n1 - 2)
    assert np.allclose(inner, ref, atol=1e-13 * np.abs(ref).max())


def test_worked_value_cfg1_coarsest_grid():
    # one unknown phi = B1(x) B1(y); A = 16/45 and b = 2 pi^2 I^2 with
    # I = 3-point Gauss value of sin(pi x) * 2x(1-x): u00 = 3.774475508788975
    P = O.Problem(W.config("cfg1"))
    c, _ = P.solve([0, 0])
    A, _ = P.assemble_dense([0, 0])
    assert abs(A[0, 0] - 16 / 45) < 1e-15
    assert abs(c[0][1, 1] - 3.774475508788975) < 1e-13
    # with exact integration the value tends to 360/pi^4
    Pq = O.Problem(W.config("cfg1"), nq=12)
    cq, _ = Pq.solve([0, 0])
    assert abs(cq[0][1, 1] - 360 / math.pi ** 4) < 1e-12


@pytest.mark.parametrize("dim,p,r,grading,amp,nq", [
    (2, 2, 1, "uniform", 0.0, 0), (2, 3, 2, "radical", 0.0, 0), (2, 2, 0, "toward0", 0.0, 0),
    (3, 2, 1, "uniform", 0.0, 0), (3, 3, 2, "toward1", 0.0, 0),
    (2, 2, 1, "uniform", 0.5, 12), (2, 3, 2, "radical", 0.4, 12)])
def test_polynomial_reproduction(dim, p, r, grading, amp, nq):
    """u = prod x_k (1 - x_k) lies in every component space for p >= 2, so the
    Galerkin solution equals u whenever the quadrature integrates the bilinear
    form and the load exactly (a = 1 with p+1 Gauss points); for the smooth
    non-polynomial coefficient a = 1 + amp sin cos the discrepancy is the
    quadrature error, negligible with 12 points.  With sum c_i = 1 the
    combination reproduces u too."""
    wl = W.config("cfg1" if dim == 2 else "cfg3", p=p, r=r, w=4 if dim == 2 else 3, lmin=0,
                  f=_fld("poly_rhs", amp, 0.1), a=_fld("sincos", amp, 0.1),
                  grading=[(grading, 2.5)] * dim, exact=_fld("poly_u"))
    P = O.Problem(wl, nq=nq)
    tol = 1e-13 if amp == 0 else 1e-11
    coefs = P.solve_all()
    pts, _ = W.eval_points(dim, 200, seed=4)
    u = P.sg_eval(coefs, pts)
    ref = np.prod(pts * (1 - pts), axis=1)
    assert np.abs(u - ref).max() < tol
    for lv, c in zip(P.components()[0], P.split(coefs)):
        assert np.abs(P.eval(lv, c, pts) - ref).max() < tol
    # the gradient of the reproduced polynomial is reproduced as well
    _, g = P.sg_eval(coefs, pts, grad=True)
    q = pts * (1 - pts)
    for k in range(dim):
        dk = (1 - 2 * pts[:, k]) * np.prod(np.delete(q, k, axis=1), axis=1)
        assert np.abs(g[:, k] - dk).max() < 10 * tol, k
    if amp == 0:
        # the plain p+1 rule with a varying coefficient is not exact
        wl2 = dict(wl, a=_fld("sincos", 0.5, 0.1), f=_fld("poly_rhs", 0.5, 0.1))
        P2 = O.Problem(wl2)
        u2 = P2.sg_eval(P2.solve_all(), pts)
        assert np.abs(u2 - ref).max() > 1e-9


def test_multipatch_split_square_equals_single_patch_c0():
    """Two patches [0,1/2]x[0,1] and [1/2,1]x[0,1] at level l in x equal one
    unit-square patch at level l+1 with a C^0 knot at x = 1/2; with C^0 spaces
    everywhere (r = 0) the two discrete spaces coincide."""
    left = W._box_patch(0.0, 0.5, 0.0, 1.0)
    right = W._box_patch(0.5, 1.0, 0.0, 1.0)
    f = _fld("sinprod", 2 * math.pi ** 2)
    two = O.Problem(W.workload("two", 2, [left, right], p=2, r=0, w=0, lmin=0, f=f,
                               interfaces=[(0, 1, 1, 0)]))
    one = O.Problem(W.workload("one", 2, [W.identity_patch(2)], p=2, r=0, w=0, lmin=0, f=f))
    c2, _ = two.solve([2, 3])
    c1, _ = one.solve([3, 3])
    pts, _ = W.eval_points(2, 100, seed=11)
    # map [0,1]^2 points to each half
    u1 = one.eval([3, 3], c1, pts)
    inl = pts[:, 0] < 0.5
    xi = pts.copy()
    xi[inl, 0] = pts[inl, 0] * 2
    xi[~inl, 0] = pts[~inl, 0] * 2 - 1
    u2 = two.eval([2, 3], c2, xi, inl.astype(np.int32) * 0 + (~inl).astype(np.int32))
    assert np.abs(u1 - u2).max() < 1e-13


def test_dirichlet_lifting_patch_test():
    """u = 1 + x + 2y with g = u and f = 0 lies in every component space of the
    bilinear L-shape patches: the lifted Galerkin solution reproduces it."""
    wl = W.config("cfg4", w=3, f=_fld("const", 0.0), g=_fld("affine", 1.0, 1.0, 2.0),
                  exact=_fld("affine", 1.0, 1.0, 2.0))
    P = O.Problem(wl)
    coefs = P.solve_all()
    pts, pid = W.eval_points(2, 60, seed=2, npatch=3)
    u = P.sg_eval(coefs, pts, pid)
    off = np.array([[-1, 0], [0, 0], [-1, -1]], float)
    x = pts + off[pid]
    assert np.abs(u - (1 + x[:, 0] + 2 * x[:, 1])).max() < 1e-13


@pytest.mark.parametrize("name", ["cfg2", "cfg5"])
def test_gradient_chain_rule_by_central_differences(name):
    """The physical gradient of a discrete solution on a curved rational map
    (quarter annulus) and on the cube: for every parametric direction k,
    grad u . dF/dxi_k equals du/dxi_k, both derivatives taken by central
    differences of the oracle's point values and of the map itself (so a
    transposed Jacobian or a missing weight-function term fails)."""
    wl = W.config(name, w=3) if name == "cfg2" else W.config(name, w=2, a=_fld("const", 1.0))
    P = O.Problem(wl)
    lv = P.components()[0][len(P.components()[0]) // 2]
    c, _ = P.solve(lv)
    d = P.dim
    pts, _ = W.eval_points(d, 40, seed=21)
    pts = 0.05 + 0.9 * pts
    _, g = P.eval(lv, c, pts, grad=True)
    h = 1e-6
    for k in range(d):
        e = np.zeros(d)
        e[k] = h
        du = (P.eval(lv, c, pts + e) - P.eval(lv, c, pts - e)) / (2 * h)
        dF = np.array([(P.geometry(x + e)[0] - P.geometry(x - e)[0]) / (2 * h) for x in pts])
        lhs = np.sum(g * dF, axis=1)
        assert np.abs(lhs - du).max() < 1e-6 * max(1.0, np.abs(du).max()), k
