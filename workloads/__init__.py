"""Seeded synthetic workloads for the sparse-grid isogeometric solver.

This module holds problem *data* only: domain geometries given by their
control points, the names and parameters of the right-hand side, coefficient
and boundary fields, discretisation parameters, seeded evaluation points and
seeded random-field samples.  It contains none of the method's arithmetic
(no basis functions, quadrature, assembly, solves or combination); both the
CPU oracle and the GPU library consume the dictionaries built here, each with
its own implementation of the method.

Field names understood by both sides:

  const           value = params[0]
  sinprod         value = params[0] * prod_k sin(pi x_k)
  sincos          value = 1 + params[0] * sin(2 pi (x + params[1])) * cos(2 pi y)
  annulus_rhs     -div(a grad u) for u = -(x^2+y^2-1)(x^2+y^2-4) x y^2 and
                  a = sincos(params[0], params[1])  (params[0] = 0 gives a = 1)
  poly_rhs        -div(a grad u) for u = prod_k x_k (1 - x_k) and a = sincos(...)
  grid3d          trilinear interpolation of samples on a vertex grid of [0,1]^3
  corner          r^(2/3) sin(2 theta / 3), theta in [0, 2 pi) from the +x axis
  affine          params[0] + params[1] x + params[2] y + params[3] z

Exact-solution names (used by the oracle's error norms in tests):
  annulus_u, sinprod_u, poly_u, corner, affine.
"""
from __future__ import annotations

import math
from typing import Any, Dict, List, Optional

import numpy as np

__all__ = [
    "identity_patch",
    "quarter_annulus_patch",
    "lshape_patches",
    "workload",
    "config",
    "CONFIG_NAMES",
    "eval_points",
    "random_vector",
    "grf_samples",
]


# --------------------------------------------------------------------------
# geometries (control nets; weights None means a polynomial B-spline map)
# --------------------------------------------------------------------------

def identity_patch(dim: int) -> Dict[str, Any]:
    """Degree-1 map of [0,1]^dim onto itself: control points at the corners."""
    shape = (2,) * dim
    ctrl = np.zeros(shape + (dim,))
    for idx in np.ndindex(*shape):
        # idx is (j_dim, ..., j_1); the point is (j_1, ..., j_dim)
        ctrl[idx] = np.array(idx[::-1], dtype=float)
    return {
        "degree": [1] * dim,
        "knots": [[0.0, 0.0, 1.0, 1.0] for _ in range(dim)],
        "ctrl": ctrl,
        "weights": None,
    }


def quarter_annulus_patch(r_in: float = 1.0, r_out: float = 2.0) -> Dict[str, Any]:
    """Quarter annulus as an exact rational quadratic map.

    xi_1 is the radial direction (degree 1, radius r_in -> r_out); xi_2 is the
    angular direction (degree 2, angle 0 -> pi/2), built from the usual
    three-point rational arc: corner points (R,0), (R,R), (0,R) with weights
    1, 1/sqrt(2), 1.
    """
    ctrl = np.zeros((3, 2, 2))
    wts = np.zeros((3, 2))
    s = 1.0 / math.sqrt(2.0)
    for j1, rad in enumerate((r_in, r_out)):
        ctrl[0, j1] = (rad, 0.0)
        ctrl[1, j1] = (rad, rad)
        ctrl[2, j1] = (0.0, rad)
        wts[0, j1], wts[1, j1], wts[2, j1] = 1.0, s, 1.0
    return {
        "degree": [1, 2],
        "knots": [[0.0, 0.0, 1.0, 1.0], [0.0, 0.0, 0.0, 1.0, 1.0, 1.0]],
        "ctrl": ctrl,
        "weights": wts,
    }


def _box_patch(x0: float, x1: float, y0: float, y1: float) -> Dict[str, Any]:
    ctrl = np.zeros((2, 2, 2))
    for j2, y in enumerate((y0, y1)):
        for j1, x in enumerate((x0, x1)):
            ctrl[j2, j1] = (x, y)
    return {
        "degree": [1, 1],
        "knots": [[0.0, 0.0, 1.0, 1.0], [0.0, 0.0, 1.0, 1.0]],
        "ctrl": ctrl,
        "weights": None,
    }


def lshape_patches() -> List[Dict[str, Any]]:
    """L-shaped domain [-1,1]^2 minus [0,1]x[-1,0] as three unit-square patches.

    Patch 0 = [-1,0]x[0,1], patch 1 = [0,1]x[0,1], patch 2 = [-1,0]x[-1,0];
    xi_1 runs along +x and xi_2 along +y in every patch.  Patch 0 touches
    patch 1 along x = 0 (its side xi_1 = 1 against side xi_1 = 0 of patch 1)
    and patch 2 along y = 0 (its side xi_2 = 0 against side xi_2 = 1 of
    patch 2).  Interfaces are listed as (patch_a, side_a, patch_b, side_b) with
    side 0: xi_1 = 0, 1: xi_1 = 1, 2: xi_2 = 0, 3: xi_2 = 1.
    """
    return [_box_patch(-1, 0, 0, 1), _box_patch(0, 1, 0, 1), _box_patch(-1, 0, -1, 0)]


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def _field(kind: str, *params: float, data: Optional[np.ndarray] = None) -> Dict[str, Any]:
    prm = [float(v) for v in params] + [0.0] * (4 - len(params))
    return {"kind": kind, "params": prm[:4], "data": data}


def workload(
    name: str,
    dim: int,
    patches: List[Dict[str, Any]],
    p: int,
    r: int,
    w: int,
    lmin: int,
    f: Dict[str, Any],
    a: Optional[Dict[str, Any]] = None,
    g: Optional[Dict[str, Any]] = None,
    exact: Optional[Dict[str, Any]] = None,
    grading: Optional[List] = None,
    **extra: Any,
) -> Dict[str, Any]:
    """Assemble a workload dictionary.

    grading: per direction a pair (kind, gamma) with kind one of
    'uniform', 'radical' (two-sided), 'toward0', 'toward1'.
    """
    if grading is None:
        grading = [("uniform", 1.0)] * dim
    wl = {
        "name": name,
        "dim": dim,
        "patches": patches,
        "p": p,
        "r": r,
        "w": w,
        "lmin": lmin,
        "grading": [(str(k), float(gm)) for k, gm in grading],
        "f": f,
        "a": a if a is not None else _field("const", 1.0),
        "g": g,
        "exact": exact,
    }
    wl.update(extra)
    return wl


CONFIG_NAMES = ("cfg1", "cfg2", "cfg3", "cfg4", "cfg5")


def config(name: str, **override: Any) -> Dict[str, Any]:
    """The five synthetic workloads (sizes and data of the paper's test problems).

    cfg1  unit square Poisson, u = sin(pi x) sin(pi y), p=2 C^1, w=6
    cfg2  quarter annulus, a = 1 + 0.5 sin(2 pi x) cos(2 pi y), u = the paper's
          regular annulus solution, p=3 C^2, w=10
    cfg3  unit cube Poisson, u = prod sin(pi x_k), p=3 C^2, w=8, lmin=1
    cfg4  L-shape, 3 patches, u = r^(2/3) sin(2 theta/3), p=2 C^1, graded
          toward the re-entrant corner with exponent 3, w=11
    cfg5  unit cube, a = exp(GRF), f = 1, p=3 C^2, w=7, 256 field samples
    Keyword overrides replace top-level entries (e.g. w=4 for a small case).
    """
    pi2 = math.pi ** 2
    if name == "cfg1":
        wl = workload(
            "cfg1", 2, [identity_patch(2)], p=2, r=1, w=6, lmin=0,
            f=_field("sinprod", 2.0 * pi2), exact=_field("sinprod_u", 1.0),
            tol=1e-12, modes=("fp64",),
        )
    elif name == "cfg2":
        wl = workload(
            "cfg2", 2, [quarter_annulus_patch()], p=3, r=2, w=10, lmin=0,
            f=_field("annulus_rhs", 0.5, 0.0), a=_field("sincos", 0.5, 0.0),
            exact=_field("annulus_u"), tol=1e-12, modes=("fp64", "fp32"),
        )
    elif name == "cfg3":
        wl = workload(
            "cfg3", 3, [identity_patch(3)], p=3, r=2, w=8, lmin=1,
            f=_field("sinprod", 3.0 * pi2), exact=_field("sinprod_u", 1.0),
            tol=1e-12, modes=("fp64", "bf16fd"),
        )
    elif name == "cfg4":
        # one-sided radical grading toward the re-entrant corner (0,0): in patch
        # 0 the corner sits at xi = (1,0), in patch 1 at (0,0), in patch 2 at (1,1)
        gp = [[("toward1", 3.0), ("toward0", 3.0)],
              [("toward0", 3.0), ("toward0", 3.0)],
              [("toward1", 3.0), ("toward1", 3.0)]]
        wl = workload(
            "cfg4", 2, lshape_patches(), p=2, r=1, w=11, lmin=0,
            f=_field("const", 0.0), g=_field("corner"), exact=_field("corner"),
            grading=gp[1], grading_per_patch=gp,
            interfaces=[(0, 1, 1, 0), (0, 2, 2, 3)],
            tol=1e-12, modes=("fp64", "fp32"),
        )
    elif name == "cfg5":
        wl = workload(
            "cfg5", 3, [identity_patch(3)], p=3, r=2, w=7, lmin=0,
            f=_field("const", 1.0), a=_field("grid3d"),
            tol=1e-10, modes=("fp64", "learned"), samples=256, train=192,
            grf={"n": 64, "ell": 0.2, "sigma": 1.0},
        )
    else:
        raise ValueError(f"unknown config {name!r}")
    wl.update(override)
    return wl


# --------------------------------------------------------------------------
# seeded inputs
# --------------------------------------------------------------------------

def eval_points(dim: int, n_random: int, lattice: int = 0, seed: int = 12345,
                npatch: int = 1):
    """Parametric evaluation points (and patch ids).

    n_random points drawn uniformly in [0,1]^dim (numpy PCG64, given seed),
    followed by the lattice^dim cell midpoints (i + 1/2)/lattice of a uniform
    parametric lattice; for several patches every point set is repeated per
    patch.  Returns (xi [n, dim] float64, patch [n] int32).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = [rng.random((n_random, dim))]
    if lattice > 0:
        t = (np.arange(lattice) + 0.5) / lattice
        idx = np.indices((lattice,) * dim).reshape(dim, -1)  # idx[0] slowest
        # column k holds x_{k+1}; x_1 varies fastest along the rows
        pts.append(t[idx[::-1]].T)
    xi = np.ascontiguousarray(np.concatenate(pts, axis=0))
    if npatch == 1:
        return xi, np.zeros(len(xi), dtype=np.int32)
    xs = np.concatenate([xi] * npatch, axis=0)
    pid = np.repeat(np.arange(npatch, dtype=np.int32), len(xi))
    return np.ascontiguousarray(xs), pid


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal FP64 vector (test right-hand sides/iterates)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)


def grf_samples(nsamples: int, n: int = 64, ell: float = 0.2, sigma: float = 1.0,
                first_seed: int = 0) -> np.ndarray:
    """Samples of a = exp(g), g a centred Gaussian field on the vertex grid
    x_m = m/(n-1) of [0,1]^3 with squared-exponential covariance
    sigma^2 exp(-|x-y|^2 / (2 ell^2)).

    The covariance is separable, C = C1 (x) C1 (x) C1, so g = (L1 (x) L1 (x) L1) z
    with L1 = V diag(sqrt(max(lambda,0))) V^T from the n x n eigen-decomposition
    of C1 (exact sampling on the grid), z ~ N(0, I) drawn with numpy PCG64 and
    seed first_seed + s for sample s.  Returns [nsamples, n, n, n] (x fastest).
    """
    x = np.arange(n) / (n - 1)
    c1 = sigma ** (2.0 / 3.0) * np.exp(-((x[:, None] - x[None, :]) ** 2) / (2 * ell * ell))
    lam, vec = np.linalg.eigh(c1)
    l1 = vec @ np.diag(np.sqrt(np.maximum(lam, 0.0))) @ vec.T
    out = np.empty((nsamples, n, n, n))
    for s in range(nsamples):
        z = np.random.Generator(np.random.PCG64(first_seed + s)).standard_normal((n, n, n))
        # z[k, j, i] with i fastest: apply L1 along each axis
        g = np.einsum("ai,kji->kja", l1, z)
        g = np.einsum("bj,kja->kba", l1, g)
        g = np.einsum("ck,kba->cba", l1, g)
        out[s] = np.exp(g)
    return out
