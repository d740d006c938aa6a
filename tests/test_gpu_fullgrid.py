"""Full tensor grids on the whole device (schedule 4) and the sparse-grid
combination as a preconditioner of the full problem, through the C-ABI.

  - whole-device FD-preconditioned CG against the oracle's direct solve of the
    full grid: 2D annulus at levels 6-8 (up to 66,049 unknowns), the forced
    whole-device path on a grid the persistent solve also takes (the two agree),
    3D unit cube at level 4 (constant and random-field coefficient);
  - 3D level 5 (35,937 unknowns), too large for the oracle's direct solve in a
    test: u = prod x_k (1 - x_k) lies in the spline space (p = 3, identity
    map, a = 1, quadrature exact), so the Galerkin solution reproduces it;
  - two-level preconditioner (iga_sg_solve_twolevel): the solution equals the
    oracle's direct full-grid solve, and the combination's coarse correction
    on every iteration cuts the outer iterations below those of the fast
    diagonalisation alone (CPU model of the same preconditioner with direct
    component solves: 36 -> 22 on the annulus at level 6).
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


def _full_array(P, Po, J, d):
    nb = Po.nbasis([J] * d)
    full = np.zeros(nb[::-1])
    full[tuple(slice(1, -1) for _ in nb)] = P.coeffs(0).cpu().numpy().reshape([n - 2 for n in nb][::-1])
    return full


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("J", [6, 7, 8])
def test_full_grid_whole_device_2d_parity(S, J):
    log(f"case full grid whole-device annulus J={J}")
    wl = W.config("cfg2", w=J)
    P = S.Plan(wl, full=True)
    P.bind()
    P.assemble()
    rep = P.solve(precision="fp64", tol=1e-12, maxit=2000, max_refine=3, timing=True)
    log(f"  iterations {rep['iters'][0]} restarts {rep['refinements'][0]} relres {rep['relres'][0]:.2e} "
        f"prelres {rep['prelres'][0]:.2e} solve {rep['kernel_ms'][1]:.2f} ms")
    assert rep["status"][0] == 0 and rep["precision"] == "fp64"
    Po = O.Problem(wl)
    ref, _ = Po.solve([J, J])
    e = rel(_full_array(P, Po, J, 2), ref[0])
    log(f"  rel L2 vs oracle direct solve {e:.2e}")
    assert e <= 1e-10


def test_full_grid_forced_whole_device_matches_persistent(S):
    J = 5
    wl = W.config("cfg2", w=J)
    P = S.Plan(wl, full=True)
    P.bind()
    P.assemble()
    P.solve(precision="fp64", tol=1e-12, maxit=800, max_refine=3)
    a = P.coeffs(0).cpu().numpy()
    rep = P.solve(precision="fp32", tol=1e-12, maxit=800, max_refine=3, schedule="stream")
    assert rep["precision"] == "fp64"  # the whole-device path runs FP64
    b = P.coeffs(0).cpu().numpy()
    log(f"  persistent vs whole-device {rel(b, a):.2e}")
    assert rel(b, a) <= 1e-11
    Po = O.Problem(wl)
    ref, _ = Po.solve([J, J])
    assert rel(_full_array(P, Po, J, 2), ref[0]) <= 1e-10


@pytest.mark.parametrize("field", ["const", "grf"])
def test_full_grid_whole_device_3d_parity(S, field):
    J = 4
    log(f"case full grid whole-device cube J={J} a={field}")
    if field == "const":
        wl = W.config("cfg3", w=J)
    else:
        wl = W.config("cfg5", w=J, a=W._field("grid3d", data=W.grf_samples(1, n=24)[0]))
    P = S.Plan(wl, full=True)
    P.bind()
    P.assemble()
    rep = P.solve(precision="fp64", tol=1e-12, maxit=2000, max_refine=3, schedule="stream")
    log(f"  iterations {rep['iters'][0]} relres {rep['relres'][0]:.2e}")
    assert rep["status"][0] == 0
    Po = O.Problem(wl)
    ref, _ = Po.solve([J, J, J])
    e = rel(_full_array(P, Po, J, 3), ref[0])
    log(f"  rel L2 vs oracle direct solve {e:.2e}")
    assert e <= 1e-10


def test_full_grid_whole_device_3d_level5_reproduces_quadratic(S):
    J = 5
    wl = W.config("cfg3", w=J, f=W._field("poly_rhs", 0.0, 0.0), exact=W._field("poly_u"))
    P = S.Plan(wl, full=True)
    assert int(P.ndof.sum()) == 33 ** 3
    P.bind()
    P.assemble()
    rep = P.solve(precision="fp64", tol=1e-13, maxit=2000, max_refine=3, timing=True)
    log(f"  3D level 5: iterations {rep['iters'][0]} relres {rep['relres'][0]:.2e} "
        f"solve {rep['kernel_ms'][1]:.2f} ms")
    assert rep["status"][0] == 0
    xi, _ = W.eval_points(3, 4096, lattice=0, seed=4)
    u = P.combine(xi).cpu().numpy()
    ref = np.prod(xi * (1 - xi), axis=1)
    err = np.abs(u - ref).max() / np.abs(ref).max()
    log(f"  max error against prod x(1-x): {err:.2e}")
    assert err <= 1e-10


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_twolevel_sparse_grid_preconditioner(S, inner):
    J = 6
    log(f"case two-level annulus J={J} inner {inner}")
    wl = W.config("cfg2", w=J)
    F = S.Plan(wl, full=True)
    F.bind()
    F.assemble()
    plain = F.solve(precision="fp64", tol=1e-12, maxit=2000, max_refine=3, schedule="stream")
    G = S.Plan(wl)
    G.bind(stream=F.stream)
    G.assemble()
    rep = F.solve_twolevel(G, tol=1e-12, maxit=500, inner_tol=1e-8, inner_precision=inner, coarse_every=1)
    log(f"  FD-PCG {plain['iters'][0]} iterations; two-level {rep['iters']} outer, {rep['inner_iters']} inner "
        f"CG iterations, status {rep['status']}")
    assert rep["status"] == 0
    assert rep["iters"] < plain["iters"][0]
    Po = O.Problem(wl)
    ref, _ = Po.solve([J, J])
    e = rel(_full_array(F, Po, J, 2), ref[0])
    log(f"  rel L2 vs oracle direct solve {e:.2e}")
    assert e <= 1e-10
    # the combination as the first direction only
    rep0 = F.solve_twolevel(G, tol=1e-12, maxit=500, inner_tol=1e-8, inner_precision=inner, coarse_every=0)
    log(f"  coarse correction on the first direction only: {rep0['iters']} outer iterations")
    assert rep0["status"] == 0
    assert rel(_full_array(F, Po, J, 2), ref[0]) <= 1e-10
