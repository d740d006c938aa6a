"""Python binding of the MI355X sparse-grid isogeometric solver (libigasg.so).

Argument marshalling only: every step of the method (basis tables,
assembly, preconditioned solves, combination) runs in the library's HIP
kernels.  PyTorch provides the device workspace and the stream.  The binding
fails loudly when the compiled library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Any, Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigasg.so")

FIELD = {None: -1, "none": -1, "const": 0, "sinprod": 1, "sincos": 2, "annulus_rhs": 3,
         "poly_rhs": 4, "grid3d": 5, "corner": 6, "affine": 7, "qp_samples": 8}
GRADE = {"uniform": 0, "radical": 1, "toward0": 2, "toward1": 3}
PREC = {"fp64": 0, "fp32": 1, "bf16fd": 2}
SCHED = {"auto": 0, "static": 1, "lists": 2, "grid": 3, "stream": 4}
STATUS = {0: "IGA_OK", 1: "IGA_ERR_INVALID_ARG", 2: "IGA_ERR_GEOMETRY", 3: "IGA_ERR_OUT_OF_MEMORY",
          4: "IGA_ERR_DEVICE", 5: "IGA_ERR_NOT_CONVERGED", 6: "IGA_ERR_BREAKDOWN", 7: "IGA_ERR_STATE"}
APPLY = {"op64": 0, "op32": 1, "fd64": 2, "fd32": 3, "fd16": 4, "res64": 5, "fds64": 6}

EXPORTS = (
    "iga_sg_plan_create", "iga_sg_workspace_bytes", "iga_sg_plan_stats", "iga_sg_bind", "iga_sg_components",
    "iga_sg_assemble", "iga_sg_solve", "iga_sg_combine", "iga_sg_eval", "iga_sg_coeffs",
    "iga_sg_apply", "iga_sg_rhs", "iga_sg_set_rhs", "iga_sg_fd_factor", "iga_sg_matrices_1d", "iga_sg_destroy",
    "iga_sg_last_error", "iga_sg_version", "iga_sg_loga", "iga_sg_set_network", "iga_sg_graph_capture",
    "iga_sg_graph_launch", "iga_sg_bind_static", "iga_sg_coeffs_full", "iga_sg_solve_twolevel",
    "iga_sg_prolongation", "iga_sg_detail_norms", "iga_sg_quad_points",
    "iga_nn_param_count", "iga_nn_forward", "iga_nn_backward", "iga_nn_adam", "iga_nn_pair",
    "iga_nn_init", "iga_nn_save", "iga_nn_load",
)


class IgaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Patch(C.Structure):
    _fields_ = [("degree", C.c_int * 3), ("nknots", C.c_int * 3),
                ("knots_host", C.POINTER(C.c_double) * 3), ("ctrl_host", C.POINTER(C.c_double)),
                ("weights_host", C.POINTER(C.c_double)), ("grading", C.c_int * 3),
                ("gamma", C.c_double * 3)]


class _Iface(C.Structure):
    _fields_ = [("patch_a", C.c_int), ("side_a", C.c_int), ("patch_b", C.c_int),
                ("side_b", C.c_int)]


class _Geometry(C.Structure):
    _fields_ = [("dim", C.c_int), ("npatch", C.c_int), ("patches", C.POINTER(_Patch)),
                ("ninterface", C.c_int), ("interfaces", C.POINTER(_Iface))]


class _Disc(C.Structure):
    _fields_ = [("p", C.c_int), ("r", C.c_int), ("w", C.c_int), ("lmin", C.c_int), ("nq", C.c_int),
                ("nsamples", C.c_int), ("op_tile", C.c_int), ("op_tile3", C.c_int), ("fd_tasks", C.c_int),
                ("full", C.c_int), ("index_host", C.POINTER(C.c_int)), ("nindex", C.c_int),
                ("keep_all", C.c_int)]


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int), ("prm", C.c_double * 4), ("data_dev", C.c_void_p),
                ("n", C.c_int * 3), ("sample_stride", C.c_int64)]


class _Opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("batched", C.c_int), ("tol", C.c_double),
                ("tol_inner", C.c_double), ("maxit", C.c_int), ("max_refine", C.c_int),
                ("workgroups", C.c_int), ("timing", C.c_int), ("continue_cg", C.c_int),
                ("precond", C.c_int), ("learned_iters", C.c_int), ("plain_fd", C.c_int),
                ("schedule", C.c_int)]


class _Report(C.Structure):
    _fields_ = [("ncomp", C.c_int), ("iters", C.POINTER(C.c_int)),
                ("refinements", C.POINTER(C.c_int)), ("relres", C.POINTER(C.c_double)),
                ("prelres", C.POINTER(C.c_double)), ("status", C.POINTER(C.c_int)),
                ("total_iters", C.c_int), ("sweeps", C.c_int), ("kernel_ms", C.c_double * 4),
                ("precision", C.c_int), ("lam_ratio", C.c_double), ("phase_us", C.c_double * 6)]


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_plans = None  # live plans (weak references), released before interpreter teardown


def _release_plans():
    """atexit: destroy every live plan (graphs, events) while the HIP runtime
    is still up; a destructor run from interpreter or library teardown would
    call into an already finalised runtime (or profiler)."""
    if _plans is None:
        return
    try:
        import torch
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for p in list(_plans):
        try:
            if getattr(p, "h", None):
                _lib.iga_sg_destroy(p.h)
                p.h = None
        except Exception:
            pass


def lib():
    """Load libigasg.so (raises if it has not been built).

    torch is imported first: it ships its own HIP runtime under the same
    soname (libamdhip64.so.7), so loading torch first makes the dynamic
    loader bind this library to torch's runtime; loading this library
    first would leave two HIP runtimes in the process.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401  (see docstring)
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1707_09598_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.iga_sg_plan_create.argtypes = [C.POINTER(_Geometry), C.POINTER(_Disc), C.POINTER(vp)]
        L.iga_sg_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.iga_sg_plan_stats.argtypes = [vp, _ip, _ip, _ip, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.iga_sg_bind.argtypes = [vp, vp, C.c_size_t, vp]
        L.iga_sg_bind_static.argtypes = [vp, vp]
        L.iga_sg_components.argtypes = [vp, _ip, _ip, C.POINTER(C.c_int64), _dp]
        L.iga_sg_assemble.argtypes = [vp, C.POINTER(_Field), C.POINTER(_Field), C.POINTER(_Field)]
        L.iga_sg_solve.argtypes = [vp, C.POINTER(_Opts), C.POINTER(_Report)]
        L.iga_sg_solve_twolevel.argtypes = [vp, vp, C.POINTER(_Opts), C.POINTER(_Opts), C.c_int,
                                            C.POINTER(_Report)]
        L.iga_sg_prolongation.argtypes = [vp, C.c_int, C.c_int, _ip, _ip, _dp]
        L.iga_sg_detail_norms.argtypes = [vp, vp, vp, C.c_int64, vp, vp]
        L.iga_sg_quad_points.argtypes = [vp, vp, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.iga_sg_combine.argtypes = [vp, vp, vp, C.c_int64, vp, vp]
        L.iga_sg_eval.argtypes = [vp, C.c_int, vp, vp, C.c_int64, vp, vp]
        L.iga_sg_coeffs.argtypes = [vp, C.c_int, vp]
        L.iga_sg_coeffs_full.argtypes = [vp, C.c_int, vp]
        L.iga_sg_apply.argtypes = [vp, C.c_int, C.c_int, vp, vp]
        L.iga_sg_rhs.argtypes = [vp, C.c_int, vp]
        L.iga_sg_set_rhs.argtypes = [vp, C.c_int, vp]
        L.iga_sg_fd_factor.argtypes = [vp, C.c_int, C.c_int, _ip, _dp, _dp]
        L.iga_sg_matrices_1d.argtypes = [vp, C.c_int, C.c_int, _ip, _dp, _dp]
        L.iga_sg_graph_capture.argtypes = [vp, C.POINTER(_Field), C.POINTER(_Field), C.POINTER(_Opts)]
        L.iga_sg_graph_launch.argtypes = [vp]
        L.iga_sg_destroy.argtypes = [vp]
        L.iga_sg_destroy.restype = None
        L.iga_sg_last_error.restype = C.c_char_p
        L.iga_sg_version.restype = C.c_char_p
        L.iga_sg_loga.argtypes = [vp, C.c_int, vp]
        L.iga_sg_set_network.argtypes = [vp, _ip, C.c_int, vp, C.c_int]
        L.iga_nn_param_count.argtypes = [_ip, C.c_int]
        L.iga_nn_param_count.restype = C.c_int64
        L.iga_nn_init.argtypes = [_ip, C.c_int, C.c_uint64, C.POINTER(C.c_float)]
        L.iga_nn_save.argtypes = [C.c_char_p, _ip, C.c_int, C.c_int, C.POINTER(C.c_float)]
        L.iga_nn_load.argtypes = [C.c_char_p, _ip, _ip, _ip, C.POINTER(C.c_float), C.c_int64]
        L.iga_nn_forward.argtypes = [_ip, C.c_int, vp, C.c_int, _ip, vp, vp, vp, vp]
        L.iga_nn_backward.argtypes = [_ip, C.c_int, vp, C.c_int, _ip, vp, vp, vp, vp, C.c_int, C.c_double, vp,
                                      vp, vp, vp]
        L.iga_nn_adam.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float,
                                  C.c_int, vp]
        L.iga_nn_pair.argtypes = [vp, vp, vp, vp, vp, C.c_int64, C.c_int, vp, vp, vp]
        _lib = L
        global _plans
        import atexit
        import weakref
        _plans = weakref.WeakSet()
        # registered after torch's import, so it runs before torch's own exit handlers
        atexit.register(_release_plans)
    return _lib


def _check(code: int) -> None:
    if code != 0:
        raise IgaError(code, lib().iga_sg_last_error().decode())


def _arr(x, dtype=np.float64) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


def _ptr(a: Optional[np.ndarray]):
    return _dp() if a is None else a.ctypes.data_as(_dp)


class Plan:
    """One plan of the solver for a workload dictionary (see ``workloads``).

    Host-side methods (components, fd_factor, matrices_1d) need no GPU.
    ``bind`` allocates the device workspace with torch on the current device.
    ``nsamples`` > 1 plans that many problems differing in their field data
    (a grid3d coefficient given as [nsamples, n3, n2, n1]); component c of
    sample s is instance s * ncomp + c, combine returns [nsamples, n].
    ``shape`` sets the launch shape: {"op_tile", "op_tile3", "fd_tasks"}
    (missing or 0: library default; see ``tune.autotune``).
    ``full`` plans the single full tensor-product grid at level w in every
    direction (standard IGA) instead of the combination technique;
    ``index_set`` ([n, d] absolute levels, downward closed) the combination
    over that set instead of the sparse-grid set of level w; ``keep_all``
    gives every index of the set a grid (also those with coefficient 0), for
    ``detail_norms``.
    """

    def __init__(self, wl: Dict[str, Any], nsamples: int = 1, shape: Optional[Dict[str, int]] = None,
                 full: bool = False, index_set=None, keep_all: bool = False):
        self.wl = wl
        self.dim = d = int(wl["dim"])
        self._keep = []
        pats = wl["patches"]
        parr = (_Patch * len(pats))()
        gpp = wl.get("grading_per_patch") or [wl["grading"]] * len(pats)
        for i, pt in enumerate(pats):
            for k in range(d):
                kv = _arr(pt["knots"][k])
                self._keep.append(kv)
                parr[i].degree[k] = int(pt["degree"][k])
                parr[i].nknots[k] = len(kv)
                parr[i].knots_host[k] = _ptr(kv)
                kind, gam = gpp[i][k]
                parr[i].grading[k] = GRADE[kind]
                parr[i].gamma[k] = float(gam)
            ctrl = _arr(pt["ctrl"]).reshape(-1)
            self._keep.append(ctrl)
            parr[i].ctrl_host = _ptr(ctrl)
            if pt.get("weights") is not None:
                wt = _arr(pt["weights"]).reshape(-1)
                self._keep.append(wt)
                parr[i].weights_host = _ptr(wt)
            else:
                parr[i].weights_host = _dp()
        self._keep.append(parr)
        ifs = wl.get("interfaces") or []
        iarr = (_Iface * max(1, len(ifs)))()
        for i, (pa, sa, pb, sb) in enumerate(ifs):
            iarr[i].patch_a, iarr[i].side_a, iarr[i].patch_b, iarr[i].side_b = pa, sa, pb, sb
        self._keep.append(iarr)
        G = _Geometry(d, len(pats), C.cast(parr, C.POINTER(_Patch)), len(ifs),
                      C.cast(iarr, C.POINTER(_Iface)))
        self.nsamples = int(nsamples)
        self.shape = dict(shape or {})
        D = _Disc(int(wl["p"]), int(wl["r"]), int(wl["w"]), int(wl["lmin"]), 0, self.nsamples,
                  int(self.shape.get("op_tile", 0)), int(self.shape.get("op_tile3", 0)),
                  int(self.shape.get("fd_tasks", 0)), int(full))
        if index_set is not None:
            iset = np.ascontiguousarray(np.asarray(index_set, dtype=np.int32).reshape(-1, d))
            self._keep.append(iset)
            D.index_host = iset.ctypes.data_as(_ip)
            D.nindex = len(iset)
            D.keep_all = int(keep_all)
        h = C.c_void_p()
        _check(lib().iga_sg_plan_create(C.byref(G), C.byref(D), C.byref(h)))
        self.h = h
        _plans.add(self)
        self.ws = None
        self.stream = None
        n = C.c_int()
        _check(lib().iga_sg_components(self.h, C.byref(n), _ip(), C.POINTER(C.c_int64)(), _dp()))
        self.ncomp = n.value
        lv = np.zeros((self.ncomp, d), dtype=np.int32)
        nd = np.zeros(self.ncomp, dtype=np.int64)
        cf = np.zeros(self.ncomp)
        _check(lib().iga_sg_components(self.h, C.byref(n), lv.ctypes.data_as(_ip),
                                       nd.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(cf)))
        self.levels, self.ndof, self.coef = lv, nd, cf
        self.ninst = self.ncomp * self.nsamples

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().iga_sg_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # ---- host queries ----------------------------------------------------
    def workspace_bytes(self) -> int:
        b = C.c_size_t()
        _check(lib().iga_sg_workspace_bytes(self.h, C.byref(b)))
        return b.value

    def fd_factor(self, direction: int, level: int):
        n = C.c_int()
        _check(lib().iga_sg_fd_factor(self.h, direction, level, C.byref(n), _dp(), _dp()))
        U = np.zeros((n.value, n.value))
        lam = np.zeros(n.value)
        _check(lib().iga_sg_fd_factor(self.h, direction, level, C.byref(n), _ptr(U), _ptr(lam)))
        return U, lam

    def stats(self) -> Dict[str, int]:
        """Task counts of a batched solve and the LDS bytes per workgroup."""
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        n, m = C.c_size_t(), C.c_size_t()
        _check(lib().iga_sg_plan_stats(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(n), C.byref(m)))
        return {"op_tasks": a.value, "fd_tasks_fp64": b.value, "fd_tasks_lowp": c.value, "lds_bytes": n.value,
                "lds_plain_bytes": m.value}

    def matrices_1d(self, direction: int, level: int):
        n = C.c_int()
        _check(lib().iga_sg_matrices_1d(self.h, direction, level, C.byref(n), _dp(), _dp()))
        K = np.zeros((n.value, n.value))
        M = np.zeros((n.value, n.value))
        _check(lib().iga_sg_matrices_1d(self.h, direction, level, C.byref(n), _ptr(K), _ptr(M)))
        return K, M

    # ---- device ------------------------------------------------------------
    def bind(self, device=None, stream=None) -> None:
        import torch
        dev = torch.device(device if device is not None else "cuda")
        nbytes = self.workspace_bytes()
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-raw.data_ptr()) % 256
        self.ws = raw
        self.ws_ptr = raw.data_ptr() + off
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        _check(lib().iga_sg_bind(self.h, C.c_void_p(self.ws_ptr), C.c_size_t(nbytes),
                                 C.c_void_p(self.stream.cuda_stream)))

    def bind_static(self, device=None, stream=None) -> None:
        """Bind to the library's static workspace of the device (no device
        allocation; see iga_sg_bind_static)."""
        import torch
        dev = torch.device(device if device is not None else "cuda")
        self.ws = None
        self.ws_ptr = None
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        with torch.cuda.device(dev):
            _check(lib().iga_sg_bind_static(self.h, C.c_void_p(self.stream.cuda_stream)))

    def _field(self, spec, keep):
        F = _Field()
        if spec is None:
            F.kind = -1
            return F
        F.kind = FIELD[spec["kind"]]
        for i, v in enumerate((list(spec.get("params") or []) + [0.0] * 4)[:4]):
            F.prm[i] = float(v)
        data = spec.get("data")
        if data is not None:
            import torch
            t = data if isinstance(data, torch.Tensor) else torch.as_tensor(np.ascontiguousarray(data))
            t = t.to(device=self.device, dtype=torch.float64).contiguous()
            keep.append(t)
            F.data_dev = t.data_ptr()
            if spec["kind"] != "qp_samples":  # a gridded field: [samples,] n3, n2, n1
                shp = tuple(t.shape)[::-1]
                for k in range(3):
                    F.n[k] = int(shp[k])
                if t.dim() == 4:  # one field per sample
                    F.sample_stride = int(shp[0] * shp[1] * shp[2])
        return F

    def assemble(self, f=None, a=None, g=None) -> None:
        wl = self.wl
        keep = []
        Ff = self._field(f if f is not None else wl["f"], keep)
        Fa = self._field(a if a is not None else wl["a"], keep)
        Fg = self._field(g if g is not None else wl.get("g"), keep)
        self._fields = keep
        _check(lib().iga_sg_assemble(self.h, C.byref(Ff), C.byref(Fa),
                                     C.byref(Fg) if Fg.kind >= 0 else C.POINTER(_Field)()))

    def solve(self, precision: str = "fp64", tol: float = 1e-11, tol_inner: float = 1e-4,
              maxit: int = 500, max_refine: int = 0, batched: bool = True, workgroups: int = 0,
              timing: bool = False, check: bool = True, continue_cg: bool = False,
              learned: bool = False, learned_iters: int = 0, scaled: bool = True,
              schedule: str = "auto") -> Dict[str, Any]:
        o = _Opts(PREC[precision], int(batched), tol, tol_inner, maxit, max_refine, workgroups,
                  int(timing), int(continue_cg), int(learned), int(learned_iters), int(not scaled),
                  SCHED[schedule])
        it = np.zeros(self.ninst, dtype=np.int32)
        rf = np.zeros(self.ninst, dtype=np.int32)
        rr = np.zeros(self.ninst)
        pr = np.zeros(self.ninst)
        stt = np.zeros(self.ninst, dtype=np.int32)
        R = _Report(self.ninst, it.ctypes.data_as(_ip), rf.ctypes.data_as(_ip), _ptr(rr), _ptr(pr),
                    stt.ctypes.data_as(_ip), 0, 0)
        code = lib().iga_sg_solve(self.h, C.byref(o), C.byref(R))
        rep = {"code": code, "iters": it, "refinements": rf, "relres": rr, "prelres": pr,
               "status": stt, "total_iters": R.total_iters, "kernel_ms": list(R.kernel_ms),
               "sweeps": R.sweeps, "phase_us": list(R.phase_us),
               "precision": {v: k for k, v in PREC.items()}.get(R.precision, R.precision),
               "lam_ratio": R.lam_ratio}
        if check:
            _check(code)
        return rep

    def solve_twolevel(self, sg: "Plan", tol: float = 1e-11, maxit: int = 500, max_refine: int = 3,
                       inner_tol: float = 1e-6, inner_precision: str = "fp64", inner_maxit: int = 500,
                       coarse_every: int = 1, timing: bool = False, check: bool = True) -> Dict[str, Any]:
        """Flexible CG on this full tensor plan with the sparse-grid plan
        ``sg`` as the coarse level of a two-level preconditioner
        (iga_sg_solve_twolevel)."""
        o = _Opts(PREC["fp64"], 1, tol, 0.0, maxit, max_refine, 0, int(timing), 0, 0, 0, 0, 0)
        oi = _Opts(PREC[inner_precision], 1, inner_tol, 1e-4, inner_maxit, 0, 0, 0,
                   int(inner_precision != "fp64"), 0, 0, 0, 0)
        it = np.zeros(1, dtype=np.int32)
        rf = np.zeros(1, dtype=np.int32)
        rr = np.zeros(1)
        pr = np.zeros(1)
        stt = np.zeros(1, dtype=np.int32)
        R = _Report(1, it.ctypes.data_as(_ip), rf.ctypes.data_as(_ip), _ptr(rr), _ptr(pr),
                    stt.ctypes.data_as(_ip), 0, 0)
        code = lib().iga_sg_solve_twolevel(self.h, sg.h, C.byref(o), C.byref(oi), int(coarse_every), C.byref(R))
        rep = {"code": code, "iters": int(it[0]), "restarts": int(rf[0]), "relres": float(rr[0]),
               "prelres": float(pr[0]), "status": int(stt[0]), "inner_iters": R.sweeps,
               "kernel_ms": list(R.kernel_ms)}
        if check:
            _check(code)
        return rep

    def prolongation(self, direction: int, level: int) -> np.ndarray:
        """1D prolongation of a full tensor plan from ``level`` to its own
        level (interior unknowns, [n_fine, n_coarse]; host tables only)."""
        nf = C.c_int(0)
        nc = C.c_int(0)
        _check(lib().iga_sg_prolongation(self.h, direction, level, C.byref(nf), C.byref(nc), _dp()))
        T = np.zeros((nf.value, nc.value))
        _check(lib().iga_sg_prolongation(self.h, direction, level, C.byref(nf), C.byref(nc), _ptr(T)))
        return T

    def solve_async(self, precision: str = "fp64", tol: float = 1e-11, tol_inner: float = 1e-4,
                    maxit: int = 500, max_refine: int = 0, batched: bool = True,
                    workgroups: int = 0, continue_cg: bool = False, learned: bool = False,
                    learned_iters: int = 0, scaled: bool = True, schedule: str = "auto") -> None:
        """Enqueue a solve without reading the report back (no host sync)."""
        o = _Opts(PREC[precision], int(batched), tol, tol_inner, maxit, max_refine, workgroups, 0,
                  int(continue_cg), int(learned), int(learned_iters), int(not scaled), SCHED[schedule])
        _check(lib().iga_sg_solve(self.h, C.byref(o), C.POINTER(_Report)()))

    def capture(self, f=None, a=None, precision: str = "fp64", tol: float = 1e-11, tol_inner: float = 1e-4,
                maxit: int = 500, max_refine: int = 0, batched: bool = True, workgroups: int = 0,
                continue_cg: bool = False, learned: bool = False, learned_iters: int = 0,
                scaled: bool = True, schedule: str = "auto") -> None:
        """Record assembly + solve (no report) as a HIP graph; ``replay``
        enqueues it.  The fields' device data is kept alive by the plan.  The
        plan must be bound to a created stream (``bind(stream=...)``), made
        torch's current stream wherever torch reads the plan's outputs."""
        wl = self.wl
        keep = []
        Ff = self._field(f if f is not None else wl["f"], keep)
        Fa = self._field(a if a is not None else wl["a"], keep)
        o = _Opts(PREC[precision], int(batched), tol, tol_inner, maxit, max_refine, workgroups, 0,
                  int(continue_cg), int(learned), int(learned_iters), int(not scaled), SCHED[schedule])
        _check(lib().iga_sg_graph_capture(self.h, C.byref(Ff), C.byref(Fa), C.byref(o)))
        self._graph_fields = keep

    def replay(self) -> None:
        """Enqueue the captured step on the plan's stream."""
        _check(lib().iga_sg_graph_launch(self.h))

    def combine(self, xi, patch=None, grad: bool = False):
        """u_sg at parametric points xi [n, d] ([nsamples, n] for several
        samples); with grad also its physical gradient ([.., n, d])."""
        import torch
        xi = torch.as_tensor(xi, dtype=torch.float64, device=self.device).contiguous()
        n = xi.shape[0]
        u = torch.empty(self.nsamples * n, dtype=torch.float64, device=self.device)
        g = torch.empty((self.nsamples * n, self.dim), dtype=torch.float64, device=self.device) if grad else None
        pid = None if patch is None else torch.as_tensor(patch, dtype=torch.int32,
                                                         device=self.device).contiguous()
        _check(lib().iga_sg_combine(self.h, C.c_void_p(xi.data_ptr()),
                                    C.c_void_p(pid.data_ptr() if pid is not None else 0), n,
                                    C.c_void_p(u.data_ptr()), C.c_void_p(g.data_ptr() if grad else 0)))
        if self.nsamples > 1:
            u = u.view(self.nsamples, n)
            g = g.view(self.nsamples, n, self.dim) if grad else None
        return (u, g) if grad else u

    def quad_points(self, weights: bool = False):
        """Physical Gauss points of every grid ([nqp_total, d], device), and
        with ``weights`` the weights w |det DF| (iga_sg_quad_points): where a
        QP_SAMPLES field (``{"kind": "qp_samples", "data": values}``) is
        sampled."""
        import torch
        n = C.c_int64(0)
        _check(lib().iga_sg_quad_points(self.h, None, None, 0, C.byref(n)))
        xq = torch.empty((n.value, self.dim), dtype=torch.float64, device=self.device)
        wq = torch.empty(n.value, dtype=torch.float64, device=self.device) if weights else None
        _check(lib().iga_sg_quad_points(self.h, C.c_void_p(xq.data_ptr()),
                                        C.c_void_p(wq.data_ptr() if weights else 0), n.value, C.byref(n)))
        return (xq, wq) if weights else xq

    def detail_norms(self, xi, wq):
        """||Delta_b||_L2 of every grid b under the quadrature (xi [n, d]
        parametric points, wq [n] weights including |det DF|); a plan built
        with keep_all (iga_sg_detail_norms)."""
        import torch
        xi = torch.as_tensor(xi, dtype=torch.float64, device=self.device).contiguous()
        wq = torch.as_tensor(wq, dtype=torch.float64, device=self.device).contiguous()
        n = xi.shape[0]
        vals = torch.empty(self.ncomp * max(n, 1), dtype=torch.float64, device=self.device)
        out = torch.empty(self.ncomp, dtype=torch.float64, device=self.device)
        _check(lib().iga_sg_detail_norms(self.h, C.c_void_p(xi.data_ptr()), C.c_void_p(wq.data_ptr()), n,
                                         C.c_void_p(vals.data_ptr()), C.c_void_p(out.data_ptr())))
        return out.cpu().numpy()

    def eval(self, comp: int, xi, patch=None, grad: bool = False):
        import torch
        xi = torch.as_tensor(xi, dtype=torch.float64, device=self.device).contiguous()
        n = xi.shape[0]
        u = torch.empty(n, dtype=torch.float64, device=self.device)
        g = torch.empty((n, self.dim), dtype=torch.float64, device=self.device) if grad else None
        pid = None if patch is None else torch.as_tensor(patch, dtype=torch.int32,
                                                         device=self.device).contiguous()
        _check(lib().iga_sg_eval(self.h, comp, C.c_void_p(xi.data_ptr()),
                                 C.c_void_p(pid.data_ptr() if pid is not None else 0), n,
                                 C.c_void_p(u.data_ptr()), C.c_void_p(g.data_ptr() if grad else 0)))
        return (u, g) if grad else u

    def coeffs(self, comp: int):
        import torch
        out = torch.empty(int(self.ndof[comp % self.ncomp]), dtype=torch.float64, device=self.device)
        _check(lib().iga_sg_coeffs(self.h, comp, C.c_void_p(out.data_ptr())))
        return out

    def coeffs_full(self, comp: int):
        """Full per-patch coefficient arrays of a component instance
        [npatch, n_d, .., n_1] (unknowns plus Dirichlet lift)."""
        import torch
        lv = self.levels[comp % self.ncomp]
        p, r = int(self.wl["p"]), int(self.wl["r"])
        nb = [p + 1 + (2 ** int(l) - 1) * (p - r) for l in lv]
        npat = len(self.wl["patches"])
        out = torch.empty([npat] + nb[::-1], dtype=torch.float64, device=self.device)
        _check(lib().iga_sg_coeffs_full(self.h, comp, C.c_void_p(out.data_ptr())))
        return out

    def rhs(self, comp: int):
        import torch
        out = torch.empty(int(self.ndof[comp % self.ncomp]), dtype=torch.float64, device=self.device)
        _check(lib().iga_sg_rhs(self.h, comp, C.c_void_p(out.data_ptr())))
        return out

    def set_rhs(self, comp: int, b) -> None:
        import torch
        b = torch.as_tensor(b, dtype=torch.float64, device=self.device).contiguous()
        if b.numel() != int(self.ndof[comp % self.ncomp]):
            raise ValueError("load vector length does not match the component")
        self._rhs_keep = b  # the copy is asynchronous on the plan's stream
        _check(lib().iga_sg_set_rhs(self.h, comp, C.c_void_p(b.data_ptr())))

    def loga(self, comp: int):
        import torch
        out = torch.empty(int(self.ndof[comp % self.ncomp]), dtype=torch.float64, device=self.device)
        _check(lib().iga_sg_loga(self.h, comp, C.c_void_p(out.data_ptr())))
        return out

    def set_network(self, net) -> None:
        """Attach a Network for learned solves (None detaches)."""
        if net is None:
            _check(lib().iga_sg_set_network(self.h, None, 0, None, 0))
            self._net = None
            return
        _check(lib().iga_sg_set_network(self.h, net._ch, net.nl, C.c_void_p(net.params.data_ptr()), net.head))
        self._net = net

    def apply(self, comp: int, which: str, x):
        import torch
        x = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        y = torch.empty_like(x)
        _check(lib().iga_sg_apply(self.h, comp, APPLY[which], C.c_void_p(x.data_ptr()),
                                  C.c_void_p(y.data_ptr())))
        return y


class Network:
    """The learned preconditioner's network: parameters (FP32, device) and Adam
    state; forward, backward and update run in the library's kernels."""

    def __init__(self, channels=(3, 16, 16, 1), params=None, device="cuda:0", stream=None, head: int = 0):
        import torch
        self.head = int(head)
        self.channels = tuple(int(c) for c in channels)
        self._ch = (C.c_int * len(self.channels))(*self.channels)
        self.nl = len(self.channels) - 1
        self.count = int(lib().iga_nn_param_count(self._ch, self.nl))
        if self.count < 0:
            raise ValueError("invalid network description")
        self.device = torch.device(device)
        self.stream = stream
        if params is None:
            params = np.zeros(self.count, dtype=np.float32)
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32), device=self.device).contiguous()
        if self.params.numel() != self.count:
            raise ValueError("parameter count mismatch")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.step = 0

    @staticmethod
    def init_params(channels, seed: int = 0) -> np.ndarray:
        """Seeded initial parameters from the library (iga_nn_init)."""
        ch = (C.c_int * len(channels))(*[int(c) for c in channels])
        n = int(lib().iga_nn_param_count(ch, len(channels) - 1))
        if n < 0:
            raise ValueError("invalid network description")
        out = np.zeros(n, dtype=np.float32)
        _check(lib().iga_nn_init(ch, len(channels) - 1, int(seed), out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def save(self, path: str) -> None:
        """Write the parameters (and the description) to a checked file."""
        p = np.ascontiguousarray(self.params.detach().cpu().numpy(), dtype=np.float32)
        _check(lib().iga_nn_save(path.encode(), self._ch, self.nl, self.head,
                                 p.ctypes.data_as(C.POINTER(C.c_float))))

    @classmethod
    def load(cls, path: str, device="cuda:0", stream=None) -> "Network":
        nl, head = C.c_int(), C.c_int()
        _check(lib().iga_nn_load(path.encode(), None, C.byref(nl), C.byref(head), None, 0))
        ch = (C.c_int * (nl.value + 1))()
        _check(lib().iga_nn_load(path.encode(), ch, C.byref(nl), C.byref(head), None, 0))
        n = int(lib().iga_nn_param_count(ch, nl.value))
        p = np.zeros(n, dtype=np.float32)
        _check(lib().iga_nn_load(path.encode(), ch, C.byref(nl), C.byref(head),
                                 p.ctypes.data_as(C.POINTER(C.c_float)), n))
        return cls(tuple(ch), p, device=device, stream=stream, head=head.value)

    def _s(self):
        import torch
        return C.c_void_p(self.stream.cuda_stream if self.stream is not None
                          else torch.cuda.current_stream(self.device).cuda_stream)

    def forward(self, x, keep: bool = False):
        """x [nb, 3, n3, n2, n1] FP32 device tensor -> y [nb, 1, n3, n2, n1]
        (and the hidden activations when keep)."""
        import torch
        nb, n3, n2, n1 = int(x.shape[0]), int(x.shape[2]), int(x.shape[3]), int(x.shape[4])
        n = (C.c_int * 3)(n1, n2, n3)
        nh = sum(self.channels[1:-1]) * nb * n1 * n2 * n3
        acts = torch.empty(max(nh, 1), dtype=torch.float32, device=self.device)
        y = torch.empty((nb, self.channels[-1], n3, n2, n1), dtype=torch.float32, device=self.device)
        _check(lib().iga_nn_forward(self._ch, self.nl, C.c_void_p(self.params.data_ptr()), nb, n,
                                    C.c_void_p(x.data_ptr()), C.c_void_p(acts.data_ptr()),
                                    C.c_void_p(y.data_ptr()), self._s()))
        return (y, acts) if keep else y

    def gradient(self, x, t):
        """Loss sum (y - t)^2 / (2 count) and its gradient (into self.grads)."""
        import torch
        y, acts = self.forward(x, keep=True)
        nb, n3, n2, n1 = int(x.shape[0]), int(x.shape[2]), int(x.shape[3]), int(x.shape[4])
        n = (C.c_int * 3)(n1, n2, n3)
        scratch = torch.empty(2 * nb * max(self.channels) * n1 * n2 * n3 + 2048, dtype=torch.float32,
                              device=self.device)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        _check(lib().iga_nn_backward(self._ch, self.nl, C.c_void_p(self.params.data_ptr()), nb, n,
                                     C.c_void_p(x.data_ptr()), C.c_void_p(acts.data_ptr()),
                                     C.c_void_p(y.data_ptr()), C.c_void_p(t.data_ptr()), self.head,
                                     float(t.numel()), C.c_void_p(self.grads.data_ptr()),
                                     C.c_void_p(loss.data_ptr()), C.c_void_p(scratch.data_ptr()), self._s()))
        return loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _check(lib().iga_nn_adam(C.c_void_p(self.params.data_ptr()), C.c_void_p(self.grads.data_ptr()),
                                 C.c_void_p(self.m.data_ptr()), C.c_void_p(self.v.data_ptr()), self.count,
                                 lr, beta1, beta2, eps, self.step, self._s()))


def make_pair(r, zfd, loga, xs=None, xk=None, head: int = 0):
    """Network input [3, n] and target [n] of one component (FP32 device
    tensors) from FP64 device vectors."""
    import torch
    n = int(r.numel())
    x = torch.empty((3, n), dtype=torch.float32, device=r.device)
    t = torch.empty(n, dtype=torch.float32, device=r.device)
    ptr = lambda v: C.c_void_p(v.data_ptr()) if v is not None else None
    _check(lib().iga_nn_pair(ptr(r), ptr(zfd), ptr(loga), ptr(xs), ptr(xk), n, int(head), ptr(x), ptr(t),
                             C.c_void_p(torch.cuda.current_stream(r.device).cuda_stream)))
    return x, t


def version() -> str:
    return lib().iga_sg_version().decode()
