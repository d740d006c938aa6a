"""Several patches and Dirichlet data on the GPU (through the C-ABI): the
L-shaped domain of three bilinear patches with one-sided radical knots toward
the re-entrant corner and the corner singularity r^(2/3) sin(2 theta / 3) as
Dirichlet data (f = 0).

  - patch test: g = 1 + x + 2y lies in every component space, so every
    component solution and u_sg reproduce it (to rounding);
  - parity: u_sg and its gradient at points of all three patches against the
    oracle's lifted multipatch direct solves (relative L2 1e-10 FP64, 1e-9
    mixed; gradient within ten times that bar);
  - two patches splitting the unit square against the oracle's two-patch
    solve with homogeneous Dirichlet data (interfaces without a lift).
"""
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


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _kw(precision):
    # a tolerance below what the graded meshes allow at the higher levels: the
    # solve may end at its refinement limit (status 5); the accuracy against
    # the oracle is what the tests assert
    return dict(precision=precision, tol=1e-13, tol_inner=1e-5, maxit=3000,
                max_refine=8 if precision == "fp64" else 20, continue_cg=precision != "fp64", check=False)


def _oracle_patch_error(w):
    """Largest error of the oracle's own direct solve on the affine patch test
    at level w (its accuracy on these graded meshes: the conditioning of the
    scaled stiffness grows with the element-size ratio, about (2^-w)^-3)."""
    aff = W._field("affine", 1.0, 1.0, 2.0)
    Po = O.Problem(W.config("cfg4", w=w, f=W._field("const", 0.0), g=aff, exact=aff))
    xi, pid = W.eval_points(2, 500, lattice=8, seed=2, npatch=3)
    off = np.array([[-1, 0], [0, 0], [-1, -1]], float)
    x = xi + off[pid]
    return float(np.abs(Po.sg_eval(Po.solve_all(), xi, pid) - (1 + x[:, 0] + 2 * x[:, 1])).max())


@pytest.mark.parametrize("precision,w", [("fp64", 3), ("fp32", 3), ("fp64", 6), ("fp32", 6)])
def test_lshape_patch_test_affine(S, precision, w):
    """At level 6 the graded 1D pencils exceed the eigenvalue ratio FP32
    factors can hold: the mixed request runs in FP64 (the report says so)."""
    log(f"case L-shape affine patch test w={w} {precision}")
    aff = W._field("affine", 1.0, 1.0, 2.0)
    wl = W.config("cfg4", w=w, f=W._field("const", 0.0), g=aff, exact=aff)
    P = S.Plan(wl)
    P.bind()
    P.assemble()
    rep = P.solve(**dict(_kw(precision), tol=1e-14))
    log(f"  ran in {rep['precision']} (1D eigenvalue ratio {rep['lam_ratio']:.1e})")
    assert rep["precision"] == (precision if rep["lam_ratio"] <= 1e7 else "fp64")
    if w >= 6:
        assert rep["precision"] == "fp64"
    log(f"  iterations {rep['iters'].tolist()} status {rep['status'].tolist()}")
    assert np.all((rep["status"] == 0) | (rep["status"] == 5))
    xi, pid = W.eval_points(2, 500, lattice=8, seed=2, npatch=3)
    u, g = P.combine(xi, patch=pid, grad=True)
    u, g = u.cpu().numpy(), g.cpu().numpy()
    off = np.array([[-1, 0], [0, 0], [-1, -1]], float)
    x = xi + off[pid]
    ref = 1 + x[:, 0] + 2 * x[:, 1]
    log(f"  max |u - (1 + x + 2y)| {np.abs(u - ref).max():.2e}, grad error {np.abs(g - [1.0, 2.0]).max():.2e}")
    Po = O.Problem(wl)
    for c, refc in enumerate(Po.split(Po.solve_all())):
        cf = P.coeffs_full(c).cpu().numpy()
        err = np.abs(cf - refc).max()
        if err > 1e-10:
            log(f"  component {c} levels {P.levels[c].tolist()}: max coefficient difference {err:.2e} at "
                f"{np.unravel_index(np.argmax(np.abs(cf - refc)), cf.shape)}")
    bar = max(1e-11 if precision == "fp64" else 1e-9, 10 * _oracle_patch_error(w))
    assert np.abs(u - ref).max() < bar
    assert np.abs(g - np.array([1.0, 2.0])).max() < 1e3 * bar
    for c in range(P.ncomp):
        uc = P.eval(c, xi, patch=pid).cpu().numpy()
        assert np.abs(uc - ref).max() < bar, c


@pytest.mark.parametrize("precision,w,graded", [("fp64", 5, True), ("fp32", 5, True), ("fp64", 6, True),
                                                 ("fp64", 8, True), ("fp64", 10, True), ("fp64", 6, False),
                                                 ("fp32", 6, False),
                                                 ("fp64", 9, False), ("fp32", 9, False)])
def test_lshape_parity_with_oracle(S, precision, w, graded):
    """The bar is 1e-10 (FP64) / 1e-9 (mixed), widened to ten times the
    oracle's own error on the affine patch test at the same level where the
    graded meshes' conditioning makes the oracle less accurate (levels 8 and
    10: 4e-9 and 6e-8).
    graded = False: the same problem on uniform knots, where the mixed mode
    runs (FP32 operator and factors inside FP64 refinement)."""
    log(f"case L-shape corner singularity w={w} {precision} graded={graded}")
    wl = W.config("cfg4", w=w)
    if not graded:
        wl = dict(wl, grading_per_patch=[[("uniform", 1.0), ("uniform", 1.0)]] * 3,
                  grading=[("uniform", 1.0), ("uniform", 1.0)])
    P = S.Plan(wl)
    P.bind()
    P.assemble()
    rep = P.solve(**_kw(precision))
    log(f"  ran in {rep['precision']} (1D eigenvalue ratio {rep['lam_ratio']:.1e})")
    log(f"  iterations {rep['iters'].tolist()} status {rep['status'].tolist()}")
    log(f"  relres {np.array2string(rep['relres'], precision=1)}")
    if not graded:
        assert rep["precision"] == precision
    assert np.all((rep["status"] == 0) | (rep["status"] == 5))
    Po = O.Problem(wl)
    co = Po.solve_all()
    # full per-patch coefficients (unknowns and lift) against the oracle's
    worst = 0.0
    for c, ref in enumerate(Po.split(co)):
        worst = max(worst, rel(P.coeffs_full(c).cpu().numpy().ravel(), ref.ravel()))
    bar = max(1e-10 if precision == "fp64" else 1e-9, 10 * _oracle_patch_error(w) if graded else 0.0)
    log(f"  worst full-coefficient rel {worst:.2e} (bar {bar:.1e})")
    assert worst < bar
    xi, pid = W.eval_points(2, 2000, lattice=16, seed=5, npatch=3)
    u, g = P.combine(xi, patch=pid, grad=True)
    uo, go = Po.sg_eval(co, xi, pid, grad=True)
    eu, eg = rel(u.cpu().numpy(), uo), rel(g.cpu().numpy().ravel(), go.ravel())
    log(f"  u_sg rel L2 {eu:.2e}, grad rel L2 {eg:.2e}")
    assert eu < bar and eg < 10 * bar
    # one component through iga_sg_eval
    c = P.ncomp // 2
    ue = P.eval(c, xi, patch=pid).cpu().numpy()
    assert rel(ue, Po.eval(P.levels[c], Po.split(co)[c], xi, pid)) < bar


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_split_square_two_patches(S, precision):
    log(f"case split square two patches {precision}")
    left = W._box_patch(0.0, 0.5, 0.0, 1.0)
    right = W._box_patch(0.5, 1.0, 0.0, 1.0)
    wl = W.workload("split", 2, [left, right], p=2, r=1, w=6, lmin=0,
                    f=W._field("sinprod", 2 * np.pi ** 2), interfaces=[(0, 1, 1, 0)])
    P = S.Plan(wl)
    P.bind()
    P.assemble()
    rep = P.solve(**dict(_kw(precision), tol=1e-12))
    assert np.all(rep["status"] == 0)
    Po = O.Problem(wl)
    co = Po.solve_all()
    xi, pid = W.eval_points(2, 1000, lattice=8, seed=9, npatch=2)
    u = P.combine(xi, patch=pid).cpu().numpy()
    uo = Po.sg_eval(co, xi, pid)
    e = rel(u, uo)
    log(f"  u_sg rel L2 {e:.2e}")
    assert e < (1e-10 if precision == "fp64" else 1e-9)
