"""ctypes wrapper of the serial FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only importers.  The GPU library never
imports, links or calls anything here, and this module never touches the GPU
library: both consume the same workload dictionaries from ``workloads``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Any, Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

_FIELD_KIND = {
    None: -1, "none": -1, "const": 0, "sinprod": 1, "sincos": 2, "annulus_rhs": 3,
    "poly_rhs": 4, "grid3d": 5, "corner": 6, "affine": 7,
    "annulus_u": 100, "sinprod_u": 101, "poly_u": 102,
}
_GRADE = {"uniform": 0, "radical": 1, "toward0": 2, "toward1": 3}

MAX_PATCH = 4
WITH_BOUNDARY = 1
MASS = 2


_SO_NATIVE = os.path.join(_HERE, "liboracle_native.so")


def build(force: bool = True, native: bool = False) -> str:
    """Compile the oracle with gcc -O3: liboracle.so with portable x86-64
    flags (the library the tests load), or with native=True
    liboracle_native.so with -march=native for the host it is built on (the
    CPU baseline's timing build; the source is the same)."""
    so = _SO_NATIVE if native else _SO
    if force or not os.path.exists(so):
        arch = "-march=native" if native else "-march=x86-64-v2"
        cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", arch,
               "-o", so + ".tmp", os.path.join(_HERE, "oracle.c"), "-lm"]
        subprocess.check_call(cmd)
        os.replace(so + ".tmp", so)
    return so


def use_native() -> str:
    """Build the -march=native oracle on this host and make lib() load it;
    call before the first lib()."""
    global _SO
    if _lib is not None and _SO != _SO_NATIVE:
        raise RuntimeError("the portable oracle is already loaded")
    _SO = build(force=True, native=True)
    return _SO


class _Patch(C.Structure):
    _fields_ = [("degree", C.c_int * 3), ("nknots", C.c_int * 3),
                ("knots", C.POINTER(C.c_double) * 3), ("ctrl", C.POINTER(C.c_double)),
                ("weights", C.POINTER(C.c_double))]


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int), ("prm", C.c_double * 4), ("data", C.POINTER(C.c_double)),
                ("n", C.c_int * 3)]


class _Iface(C.Structure):
    _fields_ = [("patch_a", C.c_int), ("side_a", C.c_int), ("patch_b", C.c_int),
                ("side_b", C.c_int)]


class _Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("npatch", C.c_int), ("patches", C.POINTER(_Patch)),
                ("ninterface", C.c_int), ("interfaces", C.POINTER(_Iface)),
                ("p", C.c_int), ("r", C.c_int), ("w", C.c_int), ("lmin", C.c_int),
                ("nq", C.c_int), ("gkind", (C.c_int * 3) * MAX_PATCH),
                ("gamma", (C.c_double * 3) * MAX_PATCH),
                ("f", _Field), ("a", _Field), ("g", _Field), ("exact", _Field)]


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        L.orc_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
        L.orc_num_knots.argtypes = [C.c_int] * 3
        L.orc_make_knots.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, _dp]
        L.orc_grade.argtypes = [C.c_int, C.c_double, C.c_double]
        L.orc_grade.restype = C.c_double
        L.orc_find_span.argtypes = [C.c_int, C.c_int, _dp, C.c_double]
        L.orc_basis_all.argtypes = [C.c_int, C.c_int, _dp, C.c_double, _dp, _dp]
        L.orc_geometry.argtypes = [C.POINTER(_Problem), C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_field_value.argtypes = [C.POINTER(_Field), C.c_int, _dp]
        L.orc_field_value.restype = C.c_double
        L.orc_exact_value.argtypes = [C.POINTER(_Field), C.c_int, _dp, _dp, _dp]
        L.orc_components.argtypes = [C.POINTER(_Problem), _ip, _dp, C.c_int]
        L.orc_comb_coef_sum.argtypes = [C.c_int, C.c_int, C.c_int, _ip]
        L.orc_comb_coef_sum.restype = C.c_double
        L.orc_ndof.argtypes = [C.POINTER(_Problem), _ip]
        L.orc_ndof.restype = C.c_int64
        L.orc_assemble_dense.argtypes = [C.POINTER(_Problem), _ip, C.c_int, _dp, _dp, C.c_int64]
        L.orc_assemble_dense.restype = C.c_int64
        L.orc_solve.argtypes = [C.POINTER(_Problem), _ip, _dp, _dp]
        L.orc_solve.restype = C.c_int64
        L.orc_eval.argtypes = [C.POINTER(_Problem), _ip, _dp, C.c_int64, _dp, _ip, _dp, _dp]
        L.orc_sg_solve_all.argtypes = [C.POINTER(_Problem), _dp, C.c_int64]
        L.orc_sg_solve_all.restype = C.c_int64
        L.orc_sg_eval.argtypes = [C.POINTER(_Problem), _dp, C.c_int64, _dp, _ip, _dp, _dp]
        L.orc_sg_errors.argtypes = [C.POINTER(_Problem), _dp, C.c_int, _dp]
        L.orc_full_errors.argtypes = [C.POINTER(_Problem), _ip, _dp, C.c_int, _dp]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return _dp()
    return a.ctypes.data_as(_dp)


def _arr(x, dtype=np.float64) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


# ---------------------------------------------------------------------------
# scalar helpers
# ---------------------------------------------------------------------------

def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().orc_gauss_legendre(n, _ptr(x), _ptr(w)) != n:
        raise ValueError("bad Gauss order")
    return x, w


def grade(kind: str, gamma: float, t: float) -> float:
    return lib().orc_grade(_GRADE[kind], gamma, t)


def knots(p: int, r: int, level: int, grading: str = "uniform", gamma: float = 1.0) -> np.ndarray:
    nk = lib().orc_num_knots(p, r, level)
    if nk < 0:
        raise ValueError("invalid (p, r, level)")
    out = np.zeros(nk)
    lib().orc_make_knots(p, r, level, _GRADE[grading], gamma, _ptr(out))
    return out


def basis_all(p: int, U, x: float):
    """All B-spline values and derivatives at x (Cox-de Boor, eq. Bsp)."""
    U = _arr(U)
    n = len(U) - p - 1
    v = np.zeros(n)
    d = np.zeros(n)
    lib().orc_basis_all(p, len(U), _ptr(U), float(x), _ptr(v), _ptr(d))
    return v, d


# ---------------------------------------------------------------------------
# problems
# ---------------------------------------------------------------------------

def combination_coefficients(index_set) -> Dict[tuple, int]:
    """Combination coefficients over a downward-closed index set I (first line
    of eq. (TD-combi-tec), its outer sum running over I):
    c_b = sum over z in {0,1}^d with b + z in I of (-1)^|z|, for every b in I
    (zeros included).  Plain Python over the set."""
    I = {tuple(int(v) for v in b) for b in index_set}
    out = {}
    for b in sorted(I):
        d = len(b)
        c = 0
        for z in range(1 << d):
            bz = tuple(b[k] + ((z >> k) & 1) for k in range(d))
            if bz in I:
                c += -1 if bin(z).count("1") % 2 else 1
        out[b] = c
    return out


class Problem:
    """A workload dictionary converted to the oracle's C description."""

    def __init__(self, wl: Dict[str, Any], nq: int = 0):
        self.wl = wl
        self.dim = d = int(wl["dim"])
        self._keep = []
        pats = wl["patches"]
        if len(pats) > MAX_PATCH:
            raise ValueError("too many patches")
        parr = (_Patch * len(pats))()
        for i, pt in enumerate(pats):
            for k in range(d):
                kv = _arr(pt["knots"][k])
                self._keep.append(kv)
                parr[i].degree[k] = int(pt["degree"][k])
                parr[i].nknots[k] = len(kv)
                parr[i].knots[k] = _ptr(kv)
            ctrl = _arr(pt["ctrl"]).reshape(-1)
            self._keep.append(ctrl)
            parr[i].ctrl = _ptr(ctrl)
            if pt.get("weights") is not None:
                wt = _arr(pt["weights"]).reshape(-1)
                self._keep.append(wt)
                parr[i].weights = _ptr(wt)
            else:
                parr[i].weights = _dp()
        self._keep.append(parr)
        P = _Problem()
        P.dim = d
        P.npatch = len(pats)
        P.patches = C.cast(parr, C.POINTER(_Patch))
        ifs = wl.get("interfaces") or []
        iarr = (_Iface * max(1, len(ifs)))()
        for i, (pa, sa, pb_, sb) in enumerate(ifs):
            iarr[i].patch_a, iarr[i].side_a, iarr[i].patch_b, iarr[i].side_b = pa, sa, pb_, sb
        self._keep.append(iarr)
        P.ninterface = len(ifs)
        P.interfaces = C.cast(iarr, C.POINTER(_Iface))
        P.p, P.r, P.w, P.lmin = int(wl["p"]), int(wl["r"]), int(wl["w"]), int(wl["lmin"])
        P.nq = nq
        gpp = wl.get("grading_per_patch") or [wl["grading"]] * len(pats)
        for i in range(len(pats)):
            for k in range(d):
                kind, gam = gpp[i][k]
                P.gkind[i][k] = _GRADE[kind]
                P.gamma[i][k] = float(gam)
        self._set_field(P.f, wl.get("f"))
        self._set_field(P.a, wl.get("a"))
        self._set_field(P.g, wl.get("g"))
        self._set_field(P.exact, wl.get("exact"))
        self.P = P

    def _set_field(self, F: _Field, spec) -> None:
        if spec is None:
            F.kind = -1
            return
        F.kind = _FIELD_KIND[spec["kind"]]
        for i, v in enumerate((list(spec.get("params") or []) + [0.0] * 4)[:4]):
            F.prm[i] = float(v)
        data = spec.get("data")
        if data is not None:
            arr = _arr(data)
            self._keep.append(arr)
            F.data = _ptr(arr)
            shp = arr.shape[::-1]  # x fastest
            for k in range(3):
                F.n[k] = int(shp[k])
        else:
            F.data = _dp()

    @property
    def ref(self):
        return C.byref(self.P)

    # --- combination ------------------------------------------------------
    def components(self):
        n = lib().orc_components(self.ref, _ip(), _dp(), 0)
        lv = np.zeros((max(n, 1), self.dim), dtype=np.int32)
        cc = np.zeros(max(n, 1))
        lib().orc_components(self.ref, lv.ctypes.data_as(_ip), _ptr(cc), n)
        return lv[:n], cc[:n]

    def nbasis(self, levels):
        """Basis functions per direction of a component grid."""
        return [lib().orc_num_knots(self.P.p, self.P.r, int(l)) - self.P.p - 1 for l in levels]

    def ndof(self, levels) -> int:
        lv = _arr(levels, np.int32)
        return int(lib().orc_ndof(self.ref, lv.ctypes.data_as(_ip)))

    # --- one component ----------------------------------------------------
    def assemble_dense(self, levels, flags: int = 0):
        lv = _arr(levels, np.int32)
        n = int(lib().orc_assemble_dense(self.ref, lv.ctypes.data_as(_ip), flags, _dp(), _dp(), 0))
        if n < 0:
            raise RuntimeError(f"assembly failed ({n})")
        A = np.zeros((n, n))
        b = np.zeros(n)
        rc = lib().orc_assemble_dense(self.ref, lv.ctypes.data_as(_ip), flags, _ptr(A), _ptr(b), n)
        if rc != n:
            raise RuntimeError(f"assembly failed ({rc})")
        return A, b

    def solve(self, levels):
        """Full coefficient array per patch [npatch, n_d, ..., n_1] and info."""
        lv = _arr(levels, np.int32)
        nb = self.nbasis(levels)
        npat = len(self.wl["patches"])
        out = np.zeros(npat * int(np.prod(nb)))
        info = np.zeros(3)
        rc = lib().orc_solve(self.ref, lv.ctypes.data_as(_ip), _ptr(out), _ptr(info))
        if rc < 0:
            raise RuntimeError(f"oracle solve failed ({rc})")
        return out.reshape([npat] + nb[::-1]), info

    def eval(self, levels, coef, xi, patch=None, grad: bool = False):
        lv = _arr(levels, np.int32)
        coef = _arr(coef).reshape(-1)
        xi = _arr(xi).reshape(-1, self.dim)
        n = len(xi)
        u = np.zeros(n)
        g = np.zeros((n, self.dim)) if grad else None
        pid = _arr(patch if patch is not None else np.zeros(n), np.int32)
        lib().orc_eval(self.ref, lv.ctypes.data_as(_ip), _ptr(coef), n, _ptr(xi),
                       pid.ctypes.data_as(_ip), _ptr(u), _ptr(g))
        return (u, g) if grad else u

    # --- all components -----------------------------------------------------
    def solve_all(self) -> np.ndarray:
        lv, _ = self.components()
        npat = len(self.wl["patches"])
        total = sum(npat * int(np.prod(self.nbasis(l))) for l in lv)
        out = np.zeros(max(total, 1))
        rc = lib().orc_sg_solve_all(self.ref, _ptr(out), total)
        if rc != total:
            raise RuntimeError(f"oracle solve_all failed ({rc})")
        return out[:total]

    def split(self, coefs: np.ndarray):
        """Split a concatenated coefficient vector into per-component arrays."""
        lv, _ = self.components()
        npat = len(self.wl["patches"])
        res, off = [], 0
        for l in lv:
            nb = self.nbasis(l)
            m = npat * int(np.prod(nb))
            res.append(coefs[off:off + m].reshape([npat] + nb[::-1]))
            off += m
        return res

    def sg_eval(self, coefs, xi, patch=None, grad: bool = False):
        coefs = _arr(coefs)
        xi = _arr(xi).reshape(-1, self.dim)
        n = len(xi)
        u = np.zeros(n)
        g = np.zeros((n, self.dim)) if grad else None
        pid = _arr(patch if patch is not None else np.zeros(n), np.int32)
        lib().orc_sg_eval(self.ref, _ptr(coefs), n, _ptr(xi), pid.ctypes.data_as(_ip),
                          _ptr(u), _ptr(g))
        return (u, g) if grad else u

    def sg_errors(self, coefs, nref: int):
        out = np.zeros(4)
        lib().orc_sg_errors(self.ref, _ptr(_arr(coefs)), nref, _ptr(out))
        return out

    def full_errors(self, levels, coef, nref: int):
        out = np.zeros(4)
        lv = _arr(levels, np.int32)
        lib().orc_full_errors(self.ref, lv.ctypes.data_as(_ip), _ptr(_arr(coef).reshape(-1)),
                              nref, _ptr(out))
        return out

    # --- geometry and fields -------------------------------------------------
    def geometry(self, xi, patch: int = 0):
        xi = _arr(xi)
        x = np.zeros(self.dim)
        jac = np.zeros(self.dim * self.dim)
        W = np.zeros(1)
        dW = np.zeros(self.dim)
        lib().orc_geometry(self.ref, patch, _ptr(xi), _ptr(x), _ptr(jac), _ptr(W), _ptr(dW))
        return x, jac.reshape(self.dim, self.dim), float(W[0]), dW

    def field(self, which: str, x) -> float:
        F = getattr(self.P, which)
        return lib().orc_field_value(C.byref(F), self.dim, _ptr(_arr(x)))

    def exact(self, x):
        u = np.zeros(1)
        g = np.zeros(self.dim)
        lib().orc_exact_value(C.byref(self.P.exact), self.dim, _ptr(_arr(x)), _ptr(u), _ptr(g))
        return float(u[0]), g
