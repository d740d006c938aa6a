"""Host-side checks of the GPU library (no GPU needed): the C-ABI exports every
symbol that include/iga_sg.h declares, plan-time host logic matches the
oracle (index set, coefficients, unknown counts, 1D matrices), the
fast-diagonalisation factors solve the generalised eigenproblem (scipy pin),
and invalid arguments are rejected with the documented status codes.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def S():
    import paper_1707_09598_amd as S
    if not os.path.exists(S.LIB_PATH):
        from paper_1707_09598_amd import build as B
        B.build(force=False)
    S.lib()
    return S


def test_exports_every_declared_symbol(S):
    hdr = "".join(open(os.path.join(ROOT, "include", h)).read() for h in ("iga_sg.h", "iga_nn.h"))
    declared = set(re.findall(r"\b(iga_(?:sg|nn)_\w+)\s*\(", hdr))
    assert declared, "no declarations found"
    L = C.CDLL(S.LIB_PATH)
    missing = [name for name in sorted(declared) if not hasattr(L, name)]
    assert not missing, missing
    assert set(S.EXPORTS) == declared


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3", "cfg5"])
def test_components_match_oracle(S, name):
    wl = W.config(name, w=min(W.config(name)["w"], 8))
    P = S.Plan(wl)
    lv, cc = O.Problem(wl).components()
    assert np.array_equal(P.levels, lv)
    assert np.array_equal(P.coef, cc)
    Po = O.Problem(wl)
    for l, n in zip(lv, P.ndof):
        assert n == Po.ndof(l)


@pytest.mark.parametrize("grading,gamma", [("uniform", 1.0), ("radical", 3.0), ("toward0", 3.0)])
@pytest.mark.parametrize("p,r", [(2, 1), (3, 2), (3, 0)])
def test_1d_matrices_match_oracle(S, grading, gamma, p, r):
    wl = W.config("cfg1", p=p, r=r, w=5, grading=[(grading, gamma)] * 2)
    P = S.Plan(wl)
    line = {"degree": [1], "knots": [[0.0, 0.0, 1.0, 1.0]], "ctrl": np.array([[0.0], [1.0]]),
            "weights": None}
    P1 = O.Problem(W.workload("1d", 1, [line], p=p, r=r, w=0, lmin=0,
                              f={"kind": "const", "params": [1, 0, 0, 0], "data": None},
                              grading=[(grading, gamma)]))
    for lev in range(0, 6):
        K, M = P.matrices_1d(0, lev)
        Ko, _ = P1.assemble_dense([lev], 0)
        Mo, _ = P1.assemble_dense([lev], O.MASS)
        assert np.allclose(K, Ko, rtol=0, atol=1e-11 * np.abs(Ko).max())
        assert np.allclose(M, Mo, rtol=0, atol=1e-15)


@pytest.mark.parametrize("lev", [0, 1, 2, 5, 8])
def test_fd_factors_solve_generalised_eigenproblem(S, lev):
    P = S.Plan(W.config("cfg2", w=8))
    K, M = P.matrices_1d(1, lev)
    U, lam = P.fd_factor(1, lev)
    n = len(lam)
    assert np.abs(U.T @ M @ U - np.eye(n)).max() < 1e-12
    assert np.abs(U.T @ K @ U - np.diag(lam)).max() < 1e-12 * lam.max()
    ref = sl.eigh(K, M, eigvals_only=True)
    assert np.allclose(lam, ref, rtol=1e-12, atol=1e-12 * ref.max())
    assert np.all(np.diff(lam) >= 0)


def test_invalid_arguments_are_rejected(S):
    wl = W.config("cfg1")
    with pytest.raises(S.IgaError) as e:
        S.Plan(dict(wl, p=9))
    assert e.value.code == 1
    with pytest.raises(S.IgaError) as e:
        S.Plan(dict(wl, r=2))
    assert e.value.code == 1
    bad = dict(wl)
    bad["patches"] = [dict(wl["patches"][0], knots=[[0.0, 0.5, 1.0, 1.0], [0.0, 0.0, 1.0, 1.0]])]
    with pytest.raises(S.IgaError) as e:
        S.Plan(bad)
    assert e.value.code == 2


def test_degree_one_plans_are_deterministic(S):
    """Degree 1 at level 0 leaves no interior unknowns: a plan whose combination
    uses such a grid is rejected with the same error every time (the 1D factor
    cache keeps failures as failures), and one whose levels start at 1 builds
    every time, its unused level-0 tables empty."""
    for _ in range(2):
        with pytest.raises(S.IgaError) as e:
            S.Plan(W.config("cfg1", w=4, p=1, r=0))
        assert e.value.code == 1 and "no interior unknowns" in str(e.value)
    for _ in range(2):
        P = S.Plan(W.config("cfg3", w=5, p=1, r=0))
        assert P.ncomp == 10 and int(P.ndof.min()) >= 1


def test_call_order_state_errors(S):
    P = S.Plan(W.config("cfg1"))
    L = S.lib()
    # assemble / solve / combine before bind must report IGA_ERR_STATE
    f = S._Field()
    f.kind = 0
    assert L.iga_sg_assemble(P.h, C.byref(f), C.byref(f), None) == 7
    o = S._Opts(0, 1, 1e-12, 1e-4, 100, 0, 0, 0, 0, 0, 0, 0, 0)
    assert L.iga_sg_solve(P.h, C.byref(o), None) == 7
    assert L.iga_sg_combine(P.h, C.c_void_p(8), None, 1, C.c_void_p(8), None) == 7
    assert b"before" in L.iga_sg_last_error()
    # the graph of a step: capture before bind, launch before capture
    assert L.iga_sg_graph_capture(P.h, C.byref(f), C.byref(f), C.byref(o)) == 7
    assert L.iga_sg_graph_launch(P.h) == 7
    assert b"before" in L.iga_sg_last_error()


def test_workspace_and_tiles_cover_every_unknown(S):
    P = S.Plan(W.config("cfg2"))
    assert P.workspace_bytes() > 0
    assert int(P.ndof.sum()) == 22545


def test_bind_rejects_small_null_or_misaligned_workspace(S):
    """Checked on the host before any device call."""
    import ctypes as C
    P = S.Plan(W.config("cfg1"))
    need = P.workspace_bytes()
    L = S.lib()
    assert L.iga_sg_bind(P.h, C.c_void_p(4096), C.c_size_t(need - 1), None) == 3
    assert "too small" in L.iga_sg_last_error().decode()
    assert L.iga_sg_bind(P.h, None, C.c_size_t(need), None) == 1
    assert L.iga_sg_bind(P.h, C.c_void_p(4096 + 8), C.c_size_t(need), None) == 1
    assert "aligned" in L.iga_sg_last_error().decode()


def test_batched_plan_scales_tasks_and_workspace(S):
    one = S.Plan(W.config("cfg5", w=5))
    many = S.Plan(W.config("cfg5", w=5), nsamples=4)
    assert many.ncomp == one.ncomp and many.ninst == 4 * one.ncomp
    s1, s4 = one.stats(), many.stats()
    assert s4["op_tasks"] == 4 * s1["op_tasks"] and s4["fd_tasks_fp64"] == 4 * s1["fd_tasks_fp64"]
    assert many.workspace_bytes() > 3 * one.workspace_bytes()
    with pytest.raises(S.IgaError):
        S.Plan(W.config("cfg5", w=5), nsamples=-1)


def test_launch_shape_options(S):
    base = S.Plan(W.config("cfg2")).stats()
    small = S.Plan(W.config("cfg2"), shape={"op_tile": 64}).stats()
    nofit = S.Plan(W.config("cfg2"), shape={"fd_tasks": 1 << 20}).stats()
    assert small["op_tasks"] > base["op_tasks"]
    assert nofit["fd_tasks_lowp"] > base["fd_tasks_lowp"]  # long directions kept in blocks
    t3 = S.Plan(W.config("cfg5", w=5), shape={"op_tile3": 64}).stats()
    assert t3["op_tasks"] > S.Plan(W.config("cfg5", w=5)).stats()["op_tasks"]


def test_index_set_plan(S):
    """A caller's downward-closed index set: the plan keeps the multi-indices
    with nonzero coefficient, in lexicographic order, with the coefficients
    of the general form (checked against the oracle's); a set that is not
    downward closed is rejected."""
    import oracle as O
    I = [b for b in np.ndindex(6, 11) if 2 * b[0] + b[1] <= 10]
    P = S.Plan(W.config("cfg2", w=10), index_set=I)
    c = O.combination_coefficients(I)
    want = sorted((b, v) for b, v in c.items() if v != 0)
    got = [(tuple(int(x) for x in l), float(v)) for l, v in zip(P.levels.tolist(), P.coef.tolist())]
    assert got == [(b, float(v)) for b, v in want]
    with pytest.raises(S.IgaError) as e:
        S.Plan(W.config("cfg2", w=10), index_set=[(0, 0), (2, 0)])
    assert e.value.code == 1


def test_network_init_save_load_roundtrip(tmp_path):
    """Seeded initialisation is deterministic (same seed, same parameters;
    another seed, others), He-scaled with a zero last layer; a saved network
    loads back bit for bit; a corrupted byte or a truncated file is refused
    (checksum and size checks)."""
    import ctypes as C
    import numpy as np
    import paper_1707_09598_amd as S
    L = S.lib()
    ch = (3, 32, 48, 1)
    a = S.Network.init_params(ch, seed=0)
    assert a.size == 3 * 32 * 27 + 32 + 32 * 48 * 27 + 48 + 48 * 27 + 1 == 45441
    assert np.array_equal(a, S.Network.init_params(ch, seed=0))
    assert not np.array_equal(a, S.Network.init_params(ch, seed=1))
    w1 = a[:3 * 32 * 27]
    assert abs(w1.std() - np.sqrt(2.0 / 81)) < 0.02 and abs(w1.mean()) < 0.02
    assert np.all(a[-(48 * 27 + 1):] == 0)
    cha = (C.c_int * 4)(*ch)
    path = str(tmp_path / "net.bin")
    p = np.random.default_rng(3).standard_normal(a.size).astype(np.float32)
    assert L.iga_nn_save(path.encode(), cha, 3, 1, p.ctypes.data_as(C.POINTER(C.c_float))) == 0
    nl, hd = C.c_int(), C.c_int()
    out = np.zeros_like(p)
    chb = (C.c_int * 4)()
    assert L.iga_nn_load(path.encode(), chb, C.byref(nl), C.byref(hd), out.ctypes.data_as(C.POINTER(C.c_float)),
                         out.size) == 0
    assert nl.value == 3 and hd.value == 1 and tuple(chb) == ch and np.array_equal(out, p)
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 0x10
    open(path, "wb").write(bytes(raw))
    assert L.iga_nn_load(path.encode(), chb, C.byref(nl), C.byref(hd), None, 0) == 1
    open(path, "wb").write(bytes(raw[:-9]))
    assert L.iga_nn_load(path.encode(), chb, C.byref(nl), C.byref(hd), None, 0) == 1
