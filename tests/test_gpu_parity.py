"""GPU parity of the HIP path against the CPU oracle (through the C-ABI).

Element-wise comparisons on seeded inputs:
  - load vectors and operator applications against the oracle's assembled
    dense systems (FP64 to 1e-13, FP32 operator to 1e-5 relative);
  - the fast-diagonalisation preconditioner against a dense solve with the
    Kronecker pencil of the 1D matrices (FP64 1e-12, FP32 1e-5, BF16 2e-2);
  - per-component coefficients and the combined solution u_sg against the
    oracle's direct solves: relative L2 <= 1e-10 in FP64, <= 1e-9 for the
    mixed-precision modes, at seeded random and lattice points (plain l2) and
    at the Gauss points of a uniform parametric mesh weighted by
    w_q |det DF| (the L2 norm on the domain); the physical gradient within
    ten times that bar.
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


def oracle_perm(nb):
    """GPU interior lexicographic index (direction 1 fastest) -> index of the
    oracle's dense assembly: single patch, directions ordered by basis count
    (the oracle's exchange sort), the first one fastest."""
    d = len(nb)
    ni = [n - 2 for n in nb]
    order = list(range(d))
    for a in range(d):
        for b in range(a + 1, d):
            if nb[order[b]] < nb[order[a]]:
                order[a], order[b] = order[b], order[a]
    idx = np.arange(int(np.prod(ni)))
    ik = [idx % ni[0], (idx // ni[0]) % ni[1]] + ([idx // (ni[0] * ni[1])] if d == 3 else [])
    out, mult = np.zeros_like(idx), 1
    for k in order:
        out += ik[k] * mult
        mult *= ni[k]
    return out


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _bound(S, wl):
    P = S.Plan(wl)
    P.bind()
    P.assemble()
    return P


def _config(name, w):
    """Workload by name; the random-field cube takes its first coefficient sample
    (a = exp(g) on a 24^3 vertex grid, seed 0).  Variants: '_c0' / '_c1'
    lower the continuity (interior knots of multiplicity p or p - 1),
    '_graded' uses radical knots (two-sided in direction 1, toward 0 in
    direction 2; eq. of Sec. 4.4), '_p<k>' degree k with maximal continuity."""
    if name == "cfg5":
        a = W.grf_samples(1, n=24)[0]
        return W.config(name, w=w, a=W._field("grid3d", data=a))
    base, _, var = name.partition("_")
    if var == "c0":
        return W.config(base, w=w, r=0)
    if var == "c1":
        return W.config(base, w=w, r=1)
    if var == "graded":
        return W.config(base, w=w, grading=[("radical", 3.0), ("toward0", 2.0)] +
                        ([("uniform", 1.0)] if base in ("cfg3", "cfg5") else []))
    if var.startswith("p"):
        deg = int(var[1:])
        return W.config(base, w=w, p=deg, r=deg - 1)
    return W.config(name, w=w)


@pytest.mark.parametrize("name,w,comps", [("cfg1", 4, None), ("cfg2", 5, None), ("cfg2", 7, None),
                                          ("cfg2", 10, [0, 1, 9, 10, 11, 19, 20]),
                                          ("cfg3", 5, None), ("cfg3", 7, [0, 1, 2, 5, 9, 14]),
                                          ("cfg5", 4, [0, 3, 6, 10]),
                                          ("cfg1_c0", 4, None), ("cfg2_c1", 5, [0, 2, 5, 8, 10]),
                                          ("cfg2_graded", 5, [0, 3, 7, 10]), ("cfg3_c1", 4, None),
                                          # 3D degrees 1, 2, 4: element layers summed over groups of 2,
                                          # 4 (one padding lane) and 8 lanes
                                          ("cfg3_p1", 5, None), ("cfg3_p2", 4, None), ("cfg3_p4", 4, [0, 1])])
def test_rhs_and_operator_parity(S, name, w, comps):
    wl = _config(name, w)
    log(f"case rhs/operator {name} w={w}")
    P = _bound(S, wl)
    Po = O.Problem(wl)
    for c, lv in enumerate(P.levels):
        if comps is not None and c not in comps:
            continue
        A, b = Po.assemble_dense(lv)
        perm = oracle_perm(Po.nbasis(lv))
        Ag = A[np.ix_(perm, perm)]
        bg = P.rhs(c).cpu().numpy()
        assert rel(bg, b[perm]) < 1e-13, (c, lv)
        x = W.random_vector(len(b), seed=100 + c)
        y = P.apply(c, "op64", x).cpu().numpy()
        assert rel(y, Ag @ x) < 1e-13, (c, lv)
        y32 = P.apply(c, "op32", x).cpu().numpy()
        assert rel(y32, Ag @ x) < 1e-5, (c, lv)


@pytest.mark.parametrize("name,w,comps", [("cfg1", 5, None), ("cfg2", 7, None),
                                          ("cfg2", 10, [0, 1, 9, 10, 11, 19, 20]),
                                          ("cfg3", 6, None), ("cfg3", 8, [0, 4, 11, 20, 45])])
def test_fast_diagonalisation_parity(S, name, w, comps):
    wl = W.config(name, w=w)
    log(f"case fd {name} w={w}")
    P = _bound(S, wl)
    d = len(P.levels[0])
    for c, lv in enumerate(P.levels):
        if comps is not None and c not in comps:
            continue
        KM = [P.matrices_1d(k, int(lv[k])) for k in range(d)]
        if d == 2:
            (K1, M1), (K2, M2) = KM
            Pk = np.kron(M2, K1) + np.kron(K2, M1)  # direction 1 fastest
        else:
            (K1, M1), (K2, M2), (K3, M3) = KM
            Pk = (np.kron(M3, np.kron(M2, K1)) + np.kron(M3, np.kron(K2, M1)) +
                  np.kron(K3, np.kron(M2, M1)))
        x = W.random_vector(len(Pk), seed=7 + c)
        # dense reference with one refinement step (residual in extended
        # precision) so that its own error stays well below the FP64 bar
        ref = np.linalg.solve(Pk, x)
        res = (x.astype(np.longdouble) - Pk.astype(np.longdouble) @ ref.astype(np.longdouble)).astype(np.float64)
        ref = ref + np.linalg.solve(Pk, res)
        # the transform is backward stable: its forward error is about
        # kappa(P) eps, with kappa(P) from the 1D eigenvalues
        lam = [P.fd_factor(k, int(lv[k]))[1] for k in range(d)]
        kappa = sum(l.max() for l in lam) / sum(l.min() for l in lam)
        tol64 = max(1e-12, 100 * 2.2e-16 * kappa)
        for which, tol in (("fd64", tol64), ("fd32", 1e-5), ("fd16", 2e-2)):
            z = P.apply(c, which, x).cpu().numpy()
            assert rel(z, ref) < tol, (c, lv, which, rel(z, ref))


@pytest.mark.parametrize("name,w,comps", [("cfg1", 5, None), ("cfg2", 7, None),
                                          ("cfg2", 10, [0, 9, 19, 20]), ("cfg3", 6, [0, 5, 10]),
                                          ("cfg5", 4, [0, 3, 6, 10, 14]),
                                          ("cfg1_c0", 4, [0, 2, 5]), ("cfg2_c1", 5, [0, 5, 10]),
                                          ("cfg2_graded", 5, [0, 3, 7, 10]), ("cfg3_c1", 4, None)])
def test_scaled_fast_diagonalisation_parity(S, name, w, comps):
    """z = S P^-1 S x with S = sqrt(diag(P) / diag(A)): diag(A) from the
    oracle's dense assembly, P the Kronecker pencil of the 1D matrices."""
    wl = _config(name, w)
    log(f"case scaled fd {name} w={w}")
    P = _bound(S, wl)
    Po = O.Problem(wl)
    d = len(P.levels[0])
    for c, lv in enumerate(P.levels):
        if comps is not None and c not in comps:
            continue
        A, _ = Po.assemble_dense(lv)
        perm = oracle_perm(Po.nbasis(lv))
        dA = np.diag(A)[perm]
        KM = [P.matrices_1d(k, int(lv[k])) for k in range(d)]
        if d == 2:
            (K1, M1), (K2, M2) = KM
            Pk = np.kron(M2, K1) + np.kron(K2, M1)
        else:
            (K1, M1), (K2, M2), (K3, M3) = KM
            Pk = (np.kron(M3, np.kron(M2, K1)) + np.kron(M3, np.kron(K2, M1)) +
                  np.kron(K3, np.kron(M2, M1)))
        sc = np.sqrt(np.diag(Pk) / dA)
        x = W.random_vector(len(Pk), seed=17 + c)
        ref = sc * np.linalg.solve(Pk, sc * x)
        lam = [P.fd_factor(k, int(lv[k]))[1] for k in range(d)]
        kappa = sum(l.max() for l in lam) / sum(l.min() for l in lam)
        z = P.apply(c, "fds64", x).cpu().numpy()
        assert rel(z, ref) < max(1e-12, 100 * 2.2e-16 * kappa), (c, lv, rel(z, ref))


def _solve_and_compare(S, wl, precision, batched, tol_coef, tol_sg, npts=4096, scaled=True):
    P = _bound(S, wl)
    rep = P.solve(precision=precision, tol=1e-11, tol_inner=1e-5, maxit=400, max_refine=6,
                  batched=batched, check=False, scaled=scaled)
    log(f"  code {rep['code']} status {rep['status'].tolist()}")
    log(f"  iters {rep['iters'].tolist()} refine {rep['refinements'].tolist()}")
    log(f"  relres {np.array2string(rep['relres'], precision=2)}")
    log(f"  prelres {np.array2string(rep['prelres'], precision=2)}")
    assert rep["code"] == 0 and np.all(rep["status"] == 0)
    Po = O.Problem(wl)
    coefs = Po.solve_all()
    worst = 0.0
    for c, (lv, co) in enumerate(zip(P.levels, Po.split(coefs))):
        g = P.coeffs(c).cpu().numpy()
        ref = co[0][(slice(1, -1),) * len(lv)].reshape(-1)
        e = rel(g, ref)
        worst = max(worst, e)
        assert e < tol_coef, (c, lv, e)
    dim = len(P.levels[0])
    xi, _ = W.eval_points(dim, npts, lattice=32 if dim == 2 else 8, seed=12345)
    u = P.combine(xi).cpu().numpy()
    u_ref = Po.sg_eval(coefs, xi)
    e_sg = rel(u, u_ref)
    # the Gauss part of E weighted by w_q |det DF| (relative L2 norm on Omega)
    from quadrature import weighted_points, weighted_rel
    xq, wq = weighted_points(wl, 16 if dim == 2 else 4)
    e_w = weighted_rel(P.combine(xq).cpu().numpy(), Po.sg_eval(coefs, xq), wq)
    log(f"  worst coefficient rel {worst:.3e}; u_sg rel L2: points {e_sg:.3e}, weighted Gauss points {e_w:.3e}")
    assert e_sg < tol_sg and e_w < tol_sg
    # the physical gradient of u_sg (the H1 part of the errors of Sec. 4)
    u2, g = P.combine(xi, grad=True)
    assert np.array_equal(u2.cpu().numpy(), u)
    _, g_ref = Po.sg_eval(coefs, xi, grad=True)
    e_g = rel(g.cpu().numpy().ravel(), g_ref.ravel())
    log(f"  grad u_sg rel L2 {e_g:.3e}")
    assert e_g < 10 * tol_sg
    # one component through iga_sg_eval
    c = len(P.levels) // 2
    ue, ge = P.eval(c, xi, grad=True)
    ue_ref, ge_ref = Po.eval(P.levels[c], Po.split(coefs)[c], xi, grad=True)
    assert rel(ue.cpu().numpy(), ue_ref) < tol_sg
    assert rel(ge.cpu().numpy().ravel(), ge_ref.ravel()) < 10 * tol_sg
    return rep


@pytest.mark.parametrize("batched", [True, False])
def test_solve_parity_cfg1(S, batched):
    log(f"case solve cfg1 batched={batched}")
    _solve_and_compare(S, W.config("cfg1"), "fp64", batched, 1e-10, 1e-10)


@pytest.mark.parametrize("scaled", [True, False])
def test_solve_parity_cfg2_fp64(S, scaled):
    log(f"case solve cfg2 fp64 scaled={scaled}")
    _solve_and_compare(S, W.config("cfg2"), "fp64", True, 1e-10, 1e-10, scaled=scaled)


@pytest.mark.parametrize("precision", ["fp32", "bf16fd"])
def test_solve_parity_cfg2_mixed(S, precision):
    log(f"case solve cfg2 {precision}")
    _solve_and_compare(S, W.config("cfg2"), precision, True, 1e-9, 1e-9)


@pytest.mark.parametrize("precision,w", [("fp64", 6), ("bf16fd", 6), ("fp64", 8), ("bf16fd", 8)])
def test_solve_parity_cube(S, precision, w):
    log(f"case solve cfg3 w={w} {precision}")
    tol = 1e-10 if precision == "fp64" else 1e-9
    _solve_and_compare(S, W.config("cfg3", w=w), precision, True, tol, tol)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solve_parity_random_field_full_size(S, precision):
    """The random-field cube at its full size (w=7, 85 grids, a = exp(g) on a
    64^3 vertex grid, first sample)."""
    log(f"case solve cfg5 w=7 {precision}")
    a = W.grf_samples(1, n=64)[0]
    wl = W.config("cfg5", a=W._field("grid3d", data=a))
    tol = 1e-10 if precision == "fp64" else 1e-9
    _solve_and_compare(S, wl, precision, True, tol, tol, npts=2048)


def test_combine_at_knots_corners_and_edges(S):
    """Points on knots, on the boundary (xi = 0 and 1: the last span is closed
    on the right) and at the corners, and an empty point set."""
    import torch
    log("case combine at knots and boundary cfg2 w=7")
    wl = W.config("cfg2", w=7)
    P = _bound(S, wl)
    P.solve(precision="fp64", tol=1e-12, maxit=400, max_refine=3)
    t = np.array([0.0, 1.0 / 128, 0.25, 0.5, 0.75, 1.0 - 1.0 / 128, 1.0])
    xi = np.array([[a, b] for a in t for b in t])
    Po = O.Problem(wl)
    coefs = Po.solve_all()
    u = P.combine(xi).cpu().numpy()
    u_ref = Po.sg_eval(coefs, xi)
    scale = np.abs(u_ref).max()
    assert np.abs(u - u_ref).max() < 1e-10 * scale
    on_edge = (xi == 0.0).any(axis=1) | (xi == 1.0).any(axis=1)
    assert np.abs(u[on_edge]).max() < 1e-12 * scale  # homogeneous Dirichlet data
    c = P.ncomp // 2
    ue = P.eval(c, xi).cpu().numpy()
    ue_ref = Po.eval(P.levels[c], Po.split(coefs)[c], xi)
    assert np.abs(ue - ue_ref).max() < 1e-10 * np.abs(ue_ref).max()
    empty = P.combine(np.zeros((0, 2)))
    assert isinstance(empty, torch.Tensor) and empty.numel() == 0


def test_single_component_edge_case(S):
    """w = 0: one 1x1 grid; the coefficient equals the closed-form value."""
    log("case w=0 single grid")
    P = _bound(S, W.config("cfg1", w=0))
    P.solve(precision="fp64")
    assert P.ncomp == 1 and int(P.ndof[0]) == 1
    assert abs(P.coeffs(0).item() - 3.774475508788975) < 1e-13


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32", 1e-9)])
def test_index_set_combination_parity(S, precision, bar):
    """Combination over a caller's anisotropic downward-closed index set
    {2 b1 + b2 <= 10} on the annulus (the kind of set the knapsack selection
    of Sec. 4.2 produces): GPU u_I against the oracle's sum of c_b u_b over
    its own direct solves, coefficients of the general form."""
    log(f"case index set {precision}")
    wl = W.config("cfg2")
    I = [b for b in np.ndindex(6, 11) if 2 * b[0] + b[1] <= 10]
    P = S.Plan(wl, index_set=I)
    P.bind()
    P.assemble()
    rep = P.solve(precision=precision, tol=1e-11, tol_inner=1e-5, maxit=400,
                  max_refine=12 if precision != "fp64" else 3, continue_cg=precision != "fp64")
    assert np.all(rep["status"] == 0)
    xi, _ = W.eval_points(2, 4096, seed=21)
    u = P.combine(xi).cpu().numpy()
    Po = O.Problem(wl)
    ref = np.zeros(len(xi))
    for lv, c in zip(P.levels, P.coef):
        coef, _ = Po.solve([int(v) for v in lv])
        ref += c * Po.eval([int(v) for v in lv], coef, xi)
    assert rel(u, ref) < bar


@pytest.mark.parametrize("name", ["cfg2", "cfg5"])
def test_fields_sampled_at_gauss_points(S, name):
    """iga_sg_quad_points and IGA_FIELD_QP_SAMPLES: the points and weights
    equal the oracle's map and |det DF| at the same parametric Gauss points,
    the weights integrate 1 to the domain's area on every grid, and the
    coordinates lie in
    the domain; coefficient and load sampled at those points by the caller
    give the solve of the same fields given analytically (to rounding of
    the two evaluations of the same formulas), and that solve matches the
    oracle's."""
    import torch
    if name == "cfg2":
        wl = W.config("cfg2", w=7)
        area = 3 * np.pi / 4
    else:
        wl = W.config("cfg5", w=5, a=W._field("const", 1.0), f=W._field("sinprod", 3 * np.pi ** 2))
        area = 1.0
    P = S.Plan(wl)
    P.bind()
    xq, wq = P.quad_points(weights=True)
    x, w = xq.cpu().numpy(), wq.cpu().numpy()
    assert x.shape == (len(w), wl["dim"])
    # every grid's points are the tensor Gauss rule of its uniform elements
    # (direction 1 fastest): coordinates and weights against the oracle's
    # geometry map at the same parametric points, and the weights' sum
    # against the area (exact for the cube; the annulus's rational |det DF|
    # is not integrated exactly by p+1 points on its coarsest grids: 8.7e-6
    # on the grid with one element around the arc)
    Po = O.Problem(wl)
    g1, w1 = np.polynomial.legendre.leggauss(wl["p"] + 1)
    g1, w1 = (g1 + 1) / 2, w1 / 2
    off = 0
    for c in range(P.ncomp):
        axes = []
        for l in P.levels[c]:
            E = 2 ** int(l)
            axes.append((((np.arange(E)[:, None] + g1[None, :]) / E).ravel(), np.tile(w1, E) / E))
        nq = int(np.prod([len(t) for t, _ in axes]))
        mesh = np.meshgrid(*[t for t, _ in axes][::-1], indexing="ij")
        wmesh = np.meshgrid(*[ww for _, ww in axes][::-1], indexing="ij")
        xi = np.stack([m.ravel() for m in mesh[::-1]], axis=1)
        wpar = np.prod(np.stack([m.ravel() for m in wmesh], axis=1), axis=1)
        pick = np.random.default_rng(c).choice(nq, size=min(nq, 200), replace=False)
        for i in pick:
            xp, jac, _, _ = Po.geometry(xi[i])
            assert np.abs(x[off + i] - xp).max() < 1e-13
            assert abs(w[off + i] - wpar[i] * abs(np.linalg.det(jac))) < 1e-13 * max(w[off + i], 1e-300) + 1e-300
        assert abs(w[off:off + nq].sum() - area) < (1e-4 if name == "cfg2" else 1e-12) * area
        off += nq
    assert off == len(w)
    if name == "cfg2":
        r = np.hypot(x[:, 0], x[:, 1])
        assert r.min() > 1 - 1e-12 and r.max() < 2 + 1e-12 and x.min() > -1e-12
        a_q = 1 + 0.5 * np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
        fa = {"kind": "qp_samples", "data": torch.as_tensor(a_q, device="cuda")}
        ff = None
    else:
        assert x.min() > -1e-15 and x.max() < 1 + 1e-15
        f_q = 3 * np.pi ** 2 * np.prod(np.sin(np.pi * x), axis=1)
        fa = None
        ff = {"kind": "qp_samples", "data": torch.as_tensor(f_q, device="cuda")}
    P.assemble()
    P.solve(precision="fp64", tol=1e-12, maxit=800, max_refine=3)
    ref = [P.coeffs(c).cpu().numpy() for c in range(P.ncomp)]
    P.assemble(a=fa, f=ff)
    P.solve(precision="fp64", tol=1e-12, maxit=800, max_refine=3)
    for c in range(P.ncomp):
        got = P.coeffs(c).cpu().numpy()
        assert np.linalg.norm(got - ref[c]) <= 1e-12 * np.linalg.norm(ref[c]), c
    pts, _ = W.eval_points(wl["dim"], 4096, lattice=0, seed=21)
    u = P.combine(pts).cpu().numpy()
    uo = Po.sg_eval(Po.solve_all(), pts)
    assert np.linalg.norm(u - uo) <= 1e-10 * np.linalg.norm(uo)
