"""Quadrature for L2 norms of differences of solutions (test infrastructure):
Gauss points of uniform parametric meshes weighted by |det DF| of the
workload's map; the quarter annulus in closed form.

The map of the quarter annulus with radii 1 and 2 is F(xi) = (1 + xi_1) A(xi_2)
with A the rational quadratic quarter arc of the unit circle (control points
(1,0), (1,1), (0,1), weights 1, 1/sqrt 2, 1), so |det DF| = (1 + xi_1)
|A x A'|.  Points and weights: nq Gauss-Legendre points in each of nc x nc
parametric cells, weights times |det DF|."""
import numpy as np


def param_gauss(dim: int, nc: int, nq: int = 4):
    """Tensor Gauss-Legendre points of a uniform parametric mesh of [0,1]^dim
    with nc cells per direction (direction 1 fastest) and their parametric
    weights."""
    g, w = np.polynomial.legendre.leggauss(nq)
    g, w = (g + 1.0) / 2.0, w / 2.0
    t = ((np.arange(nc)[:, None] + g[None, :]) / nc).ravel()
    wt = np.tile(w, nc) / nc
    grids = np.meshgrid(*([t] * dim), indexing="ij")
    wgs = np.meshgrid(*([wt] * dim), indexing="ij")
    xi = np.stack([gk.ravel() for gk in grids], axis=1)
    wq = np.prod(np.stack([wk.ravel() for wk in wgs], axis=1), axis=1)
    return xi, wq


def annulus_detjac(xi):
    """|det DF| of the quarter annulus map at parametric points xi [n, 2]."""
    s = 1.0 / np.sqrt(2.0)
    u = xi[:, 1]
    B = [(1 - u) ** 2, 2 * u * (1 - u), u ** 2]
    dB = [-2 * (1 - u), 2 - 4 * u, 2 * u]
    wts = [1.0, s, 1.0]
    P = [(1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]
    Wt = sum(wk * b for wk, b in zip(wts, B))
    dW = sum(wk * b for wk, b in zip(wts, dB))
    N = [sum(wk * b * p[c] for wk, b, p in zip(wts, B, P)) for c in range(2)]
    dN = [sum(wk * b * p[c] for wk, b, p in zip(wts, dB, P)) for c in range(2)]
    A = [n / Wt for n in N]
    dA = [(dn * Wt - n * dW) / Wt ** 2 for n, dn in zip(N, dN)]
    return (1.0 + xi[:, 0]) * np.abs(A[0] * dA[1] - A[1] * dA[0])


def annulus_quadrature(nc: int, nq: int = 4):
    xi, wq = param_gauss(2, nc, nq)
    return xi, wq * annulus_detjac(xi)


def weighted_points(wl, nc: int):
    """Gauss points (p+1 per direction) of a uniform parametric mesh and the
    weights w_q |det DF| of the workload's map: the quarter annulus in closed
    form; identity maps (unit square and cube) have det DF = 1."""
    d = int(wl["dim"])
    xi, wq = param_gauss(d, nc, int(wl["p"]) + 1)
    pt = wl["patches"][0]
    if len(wl["patches"]) == 1 and pt.get("weights") is not None:
        wq = wq * annulus_detjac(xi)
    return xi, wq


def weighted_rel(u, ref, wq):
    """Relative L2 error of u against ref under the quadrature weights wq."""
    return float(np.sqrt(np.sum(wq * (u - ref) ** 2) / np.sum(wq * ref ** 2)))


def low_regular_annulus(W, J, r=2):
    """The paper's low-regular problem: quarter annulus, a = 1, f = 1, no exact
    solution (Sec. 4.3, Table 3)."""
    return W.config("cfg2", w=J, r=r, f=W._field("const", 1.0), a=W._field("const", 1.0), exact=None)


def graded_gauss(level: int, kind: str, gamma: float, nq: int):
    """Tensor Gauss points of the level-`level` parametric mesh graded by the
    radical map of Sec. 4.4 in both directions (breakpoints f(k / 2^level))
    and their parametric weights: exact for piecewise polynomials on that
    mesh and on every coarser mesh of the same grading."""
    import oracle as O
    t = np.array([O.grade(kind, gamma, k / 2 ** level) for k in range(2 ** level + 1)])
    g, w = np.polynomial.legendre.leggauss(nq)
    g, w = (g + 1.0) / 2.0, w / 2.0
    h = np.diff(t)
    x1 = (t[:-1, None] + h[:, None] * g[None, :]).ravel()
    w1 = (h[:, None] * w[None, :]).ravel()
    X2, X1 = np.meshgrid(x1, x1, indexing="ij")  # direction 1 fastest
    W2, W1 = np.meshgrid(w1, w1, indexing="ij")
    xi = np.stack([X1.ravel(), X2.ravel()], axis=1)
    return xi, (W1 * W2).ravel()


def golden_rates(name: str):
    """Rows of a printed rate table (tests/golden/<name>.txt): {(continuity,
    degree, method): {"d2_H1": .., "d2_L2": .., "d3_H1": .., "d3_L2": ..,
    "prov_H1": .., "prov_L2": ..}}."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name + ".txt")
    cols = ["d2_H1", "d2_L2", "d3_H1", "d3_L2", "prov_H1", "prov_L2"]
    out = {}
    with open(path) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            t = line.split()
            out[(t[0], int(t[1]), t[2])] = dict(zip(cols, map(float, t[3:])))
    return out
