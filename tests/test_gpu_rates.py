"""Convergence of the sparse-grid solution computed on the GPU, against the
paper's measured rates (Table 2, regular quarter annulus, d = 2, p = 3, C^2:
SG-IGA L2 / H1 rates 4.15 / 3.06; Table 1 proves 4 / 3).

Component solves run through the C-ABI (batched persistent solve, FP64 and the
mixed FP32/FP64 mode); the H1 and L2 errors of u_sg against the exact solution
are integrated by the oracle's error functional from the GPU coefficients, and
must equal the errors of the oracle's own direct solves at every level to the
parity bar (1e-10 of the norm of u in FP64, 1e-9 in the mixed mode).  Rates are least-squares slopes of log2(error) against the level
over levels 5-8 (the paper does not state its fit levels; the oracle's pin of
the same rates allows 0.3 from the provable rates and 0.4 from the printed
ones)."""
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


def _annulus_paper(J):
    # the paper's regular annulus problem: a = 1, f = -Laplace(u) (Sec. 4.2)
    return W.config("cfg2", w=J, f=W._field("annulus_rhs", 0.0), a=W._field("const", 1.0),
                    exact=W._field("annulus_u"))


def _oracle_layout(P, Po):
    """GPU interior coefficients of every component (direction 1 fastest) as
    the oracle's concatenated full-basis arrays (zero boundary values)."""
    out = []
    for c, lv in enumerate(P.levels):
        nb = Po.nbasis(lv)
        full = np.zeros(nb[::-1])
        inner = tuple(slice(1, -1) for _ in nb)
        full[inner] = P.coeffs(c).cpu().numpy().reshape([n - 2 for n in nb][::-1])
        out.append(full.ravel())
    return np.concatenate(out)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gpu_sparse_grid_rates_regular_annulus(S, precision):
    rows = []
    for J in range(5, 9):
        log(f"case rates annulus J={J} {precision}")
        wl = _annulus_paper(J)
        P = S.Plan(wl)
        P.bind()
        P.assemble()
        rep = P.solve(precision=precision, tol=1e-12, tol_inner=1e-4, maxit=600,
                      max_refine=12 if precision != "fp64" else 3, continue_cg=precision != "fp64")
        assert np.all(rep["status"] == 0)
        Po = O.Problem(wl)
        co = Po.solve_all()
        e_gpu = Po.sg_errors(_oracle_layout(P, Po), 128)
        e_orc = Po.sg_errors(co, 128)
        # the GPU solution itself, value and gradient, at weighted Gauss points
        from quadrature import annulus_quadrature, weighted_rel
        xq, wq = annulus_quadrature(32)
        ug, gg = P.combine(xq, grad=True)
        uo, go = Po.sg_eval(co, xq, grad=True)
        bar_u = 1e-10 if precision == "fp64" else 1e-9
        assert weighted_rel(ug.cpu().numpy(), uo, wq) <= bar_u
        gn = np.sqrt(np.sum(wq[:, None] * go ** 2))
        assert np.sqrt(np.sum(wq[:, None] * (gg.cpu().numpy() - go) ** 2)) <= 10 * bar_u * gn
        # [L2 error, H1 error, L2 norm, H1 norm]: the errors differ by at most
        # the distance between the two solutions (triangle inequality), which
        # the parity bar bounds relative to the norm of u
        bar = 1e-10 if precision == "fp64" else 1e-9
        assert abs(e_gpu[0] - e_orc[0]) <= bar * e_orc[2] and abs(e_gpu[1] - e_orc[1]) <= bar * e_orc[3]
        rows.append((J, e_gpu[0] / e_gpu[2], e_gpu[1] / e_gpu[3]))
        log(f"  J={J} ndof={int(P.ndof.sum())} relative L2 {rows[-1][1]:.3e} H1 {rows[-1][2]:.3e}")
    r = np.array(rows)
    l2 = -np.polyfit(r[:, 0], np.log2(r[:, 1]), 1)[0]
    h1 = -np.polyfit(r[:, 0], np.log2(r[:, 2]), 1)[0]
    log(f"  rates over J=5..8: L2 {l2:.2f} (Table 2: 4.15), H1 {h1:.2f} (Table 2: 3.06)")
    assert abs(l2 - 4.0) < 0.3 and abs(h1 - 3.0) < 0.3
    assert abs(l2 - 4.15) < 0.4 and abs(h1 - 3.06) < 0.4


@pytest.fixture(scope="module")
def low_regular_reference():
    """Oracle solutions of the low-regular annulus problem at the quadrature
    points, values and physical gradients: the level-12 reference and levels
    5-9."""
    from quadrature import annulus_quadrature, low_regular_annulus
    xi, wq = annulus_quadrature(256)
    sols = {}
    for J in (12, 5, 6, 7, 8, 9):
        Po = O.Problem(low_regular_annulus(W, J))
        sols[J] = Po.sg_eval(Po.solve_all(), xi, grad=True)
        log(f"  oracle level {J} evaluated")
    return xi, wq, sols


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gpu_rate_low_regular_annulus(S, precision, low_regular_reference):
    """The paper's low-regular problem (quarter annulus, f = 1; Table 3, d = 2,
    p = 3, C^2: SG-IGA L2 rate 1.58, provable 1.5; H1 rate 1.19, provable 1)
    solved on the GPU at levels 5-9: the GPU values and gradients at the
    quadrature points (Gauss, 256 x 256 cells, weights w_q |det DF|) equal
    the oracle's solution of the same level to the parity bar, the L2 and H1
    errors against the oracle's level-12 solution equal the oracle's own, and
    the fitted L2 rate is within 0.2 of 1.5 and 0.3 of 1.58, the H1 rate
    within 0.3 of 1 and of 1.19."""
    import torch
    from quadrature import low_regular_annulus, weighted_rel
    xi, wq, sols = low_regular_reference
    ur, gr = sols[12]
    nrm = np.sqrt(np.sum(wq * ur ** 2))
    gnrm = np.sqrt(np.sum(wq[:, None] * gr ** 2))
    xt = torch.as_tensor(xi, device="cuda")
    bar = 1e-10 if precision == "fp64" else 1e-9
    rows = []
    for J in range(5, 10):
        log(f"case low-regular annulus J={J} {precision}")
        P = S.Plan(low_regular_annulus(W, J))
        P.bind()
        P.assemble()
        rep = P.solve(precision=precision, tol=1e-12, tol_inner=1e-4, maxit=600,
                      max_refine=12 if precision != "fp64" else 3, continue_cg=precision != "fp64")
        assert np.all(rep["status"] == 0)
        u, g = P.combine(xt, grad=True)
        u, g = u.cpu().numpy(), g.cpu().numpy()
        uo, go = sols[J]
        assert weighted_rel(u, uo, wq) <= bar
        assert np.sqrt(np.sum(wq[:, None] * (g - go) ** 2)) <= 10 * bar * gnrm
        e_gpu = np.sqrt(np.sum(wq * (u - ur) ** 2)) / nrm
        e_orc = np.sqrt(np.sum(wq * (uo - ur) ** 2)) / nrm
        h_gpu = np.sqrt(np.sum(wq[:, None] * (g - gr) ** 2)) / gnrm
        h_orc = np.sqrt(np.sum(wq[:, None] * (go - gr) ** 2)) / gnrm
        assert abs(e_gpu - e_orc) <= bar and abs(h_gpu - h_orc) <= 10 * bar
        rows.append((J, e_gpu, h_gpu))
        log(f"  J={J} ndof={int(P.ndof.sum())} relative L2 {e_gpu:.3e} H1 {h_gpu:.3e}")
    r = np.array(rows)
    l2 = -np.polyfit(r[:, 0], np.log2(r[:, 1]), 1)[0]
    h1 = -np.polyfit(r[:, 0], np.log2(r[:, 2]), 1)[0]
    log(f"  rates over J=5..9: L2 {l2:.2f} (Table 3: 1.58, provable 1.5), H1 {h1:.2f} (Table 3: 1.19, provable 1)")
    assert abs(l2 - 1.5) < 0.2 and abs(l2 - 1.58) < 0.3
    assert abs(h1 - 1.0) < 0.3 and abs(h1 - 1.19) < 0.3


@pytest.mark.parametrize("gamma", [2.0, 3.0])
def test_gpu_rate_low_regular_annulus_radical_mesh(S, gamma):
    """Radical knots (Sec. 4.4, two-sided map with exponent gamma in both
    directions) on the low-regular problem: the paper reports that the rate
    grows with gamma up to a maximum (its rate-against-gamma figure).  GPU
    solves at levels 5-9 against the oracle's level-12 solution on the same
    mesh family: errors equal the oracle's to the FP64 parity bar, and the L2
    rate is at least 2, against 1.47 on uniform knots."""
    import torch
    from quadrature import annulus_quadrature, low_regular_annulus

    def wl(J):
        w = low_regular_annulus(W, J)
        return dict(w, grading=[("radical", gamma), ("radical", gamma)])

    xi, wq = annulus_quadrature(256)
    Pr = O.Problem(wl(12))
    ur = Pr.sg_eval(Pr.solve_all(), xi)
    nrm = np.sqrt(np.sum(wq * ur ** 2))
    xt = torch.as_tensor(xi, device="cuda")
    rows = []
    for J in range(5, 10):
        log(f"case radical gamma={gamma} J={J}")
        P = S.Plan(wl(J))
        P.bind()
        P.assemble()
        rep = P.solve(precision="fp64", tol=1e-12, maxit=800, max_refine=3)
        assert np.all(rep["status"] == 0)
        u = P.combine(xt).cpu().numpy()
        Po = O.Problem(wl(J))
        uo = Po.sg_eval(Po.solve_all(), xi)
        assert np.sqrt(np.sum(wq * (u - uo) ** 2)) <= 1e-10 * np.sqrt(np.sum(wq * uo ** 2))
        e_gpu = np.sqrt(np.sum(wq * (u - ur) ** 2)) / nrm
        e_orc = np.sqrt(np.sum(wq * (uo - ur) ** 2)) / nrm
        assert abs(e_gpu - e_orc) <= 1e-10
        rows.append((J, e_gpu))
        log(f"  J={J} relative L2 {e_gpu:.3e}")
    r = np.array(rows)
    l2 = -np.polyfit(r[:, 0], np.log2(r[:, 1]), 1)[0]
    log(f"  gamma={gamma}: L2 rate over J=5..9 {l2:.2f}")
    assert l2 >= 2.0
