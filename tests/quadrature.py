"""Quadrature on the quarter annulus for the L2 norm of a difference of two
solutions (test infrastructure).

The map of the quarter annulus with radii 1 and 2 is F(xi) = (1 + xi_1) A(xi_2)
with A the rational quadratic quarter arc of the unit circle (control points
(1,0), (1,1), (0,1), weights 1, 1/sqrt 2, 1), so |det DF| = (1 + xi_1)
|A x A'|.  Points and weights: nq Gauss-Legendre points in each of nc x nc
parametric cells, weights times |det DF|."""
import numpy as np


def annulus_quadrature(nc: int, nq: int = 4):
    g, w = np.polynomial.legendre.leggauss(nq)
    g, w = (g + 1.0) / 2.0, w / 2.0
    t = ((np.arange(nc)[:, None] + g[None, :]) / nc).ravel()
    wt = np.tile(w, nc) / nc
    X1, X2 = np.meshgrid(t, t, indexing="ij")
    W1, W2 = np.meshgrid(wt, wt, indexing="ij")
    xi = np.stack([X1.ravel(), X2.ravel()], axis=1)
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
    det = (1.0 + xi[:, 0]) * np.abs(A[0] * dA[1] - A[1] * dA[0])
    return xi, W1.ravel() * W2.ravel() * det


def low_regular_annulus(W, J, r=2):
    """The paper's low-regular problem: quarter annulus, a = 1, f = 1, no exact
    solution (Sec. 4.3, Table 3)."""
    return W.config("cfg2", w=J, r=r, f=W._field("const", 1.0), a=W._field("const", 1.0), exact=None)
