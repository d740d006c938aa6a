"""Several coefficient samples planned, assembled and solved in one launch
(through the C-ABI): every instance must equal the single-sample solve of its
sample bit for bit (each grid's arithmetic is fixed-order and independent of
which workgroup runs it), and the combination returns one row per sample."""
import sys

import numpy as np
import pytest

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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_samples_equal_single_sample_solves(S, precision):
    import torch
    ns, w = 3, 4
    log(f"case batched cfg5 w={w} samples={ns} {precision}")
    fields = W.grf_samples(ns, n=24)
    kw = dict(precision=precision, tol=1e-11, maxit=400, max_refine=3 if precision == "fp64" else 8,
              continue_cg=precision != "fp64")
    xi, _ = W.eval_points(3, 1024, lattice=4, seed=3)
    wl = W.config("cfg5", w=w, a=W._field("grid3d", data=fields[0]))
    B = S.Plan(wl, nsamples=ns)
    assert B.ninst == ns * B.ncomp
    B.bind()
    a_all = torch.as_tensor(fields, device="cuda")
    B.assemble(a=W._field("grid3d", data=a_all))
    rep = B.solve(**kw)
    assert len(rep["iters"]) == ns * B.ncomp and np.all(rep["status"] == 0)
    ub = B.combine(xi).cpu().numpy()
    assert ub.shape == (ns, len(xi))
    for s in range(ns):
        P = S.Plan(W.config("cfg5", w=w, a=W._field("grid3d", data=fields[s])))
        P.bind()
        P.assemble()
        r1 = P.solve(**kw)
        for c in range(P.ncomp):
            assert np.array_equal(P.rhs(c).cpu().numpy(), B.rhs(s * B.ncomp + c).cpu().numpy()), (s, c)
            assert np.array_equal(P.loga(c).cpu().numpy(), B.loga(s * B.ncomp + c).cpu().numpy()), (s, c)
        for c in range(P.ncomp):
            x1 = P.coeffs(c).cpu().numpy()
            xb = B.coeffs(s * B.ncomp + c).cpu().numpy()
            assert np.array_equal(x1, xb), (s, c)
        assert np.array_equal(r1["iters"], rep["iters"][s * B.ncomp:(s + 1) * B.ncomp])
        assert np.array_equal(P.combine(xi).cpu().numpy(), ub[s])
        c = P.ncomp // 2
        assert np.array_equal(P.eval(c, xi).cpu().numpy(), B.eval(s * B.ncomp + c, xi).cpu().numpy())
    log(f"  {ns} samples x {B.ncomp} grids: iterations {int(rep['total_iters'])}")


@pytest.mark.parametrize("name,precision,ns", [("cfg5", "fp64", 6), ("cfg5", "fp32", 6), ("cfg2", "fp32", 1)])
def test_static_and_dynamic_schedules_agree_bitwise(S, name, precision, ns):
    """The persistent solve's two task schedules (round robin over the launch's
    tasks; round robin over per-sweep lists of the grids still iterating) give
    the same coefficients, iteration counts and statuses bit for bit: each
    task writes its own partial sums in a fixed order."""
    import torch
    w = 4 if name == "cfg5" else 7
    log(f"case schedules {name} w={w} samples={ns} {precision}")
    if name == "cfg5":
        fields = W.grf_samples(ns, n=24)
        P = S.Plan(W.config("cfg5", w=w, a=W._field("grid3d", data=fields[0])), nsamples=ns)
        P.bind()
        P.assemble(a=W._field("grid3d", data=torch.as_tensor(fields, device="cuda")))
    else:
        P = S.Plan(W.config(name, w=w))
        P.bind()
        P.assemble()
    kw = dict(precision=precision, tol=1e-11, maxit=400, max_refine=3 if precision == "fp64" else 8,
              continue_cg=precision != "fp64")
    out = {}
    for sched in ("static", "lists"):
        rep = P.solve(schedule=sched, **kw)
        assert np.all(rep["status"] == 0), sched
        out[sched] = (rep, [P.coeffs(c).cpu().numpy() for c in range(P.ninst)])
    (ra, xa), (rb, xb) = out["static"], out["lists"]
    assert np.array_equal(ra["iters"], rb["iters"])
    assert np.array_equal(ra["refinements"], rb["refinements"])
    assert np.array_equal(ra["relres"], rb["relres"])
    for c in range(P.ninst):
        assert np.array_equal(xa[c], xb[c]), c


@pytest.mark.parametrize("name,precision,ns,batched", [("cfg2", "fp32", 1, True), ("cfg2", "fp64", 1, False),
                                                        ("cfg5", "fp32", 3, True)])
def test_graph_replays_equal_direct_calls(S, name, precision, ns, batched):
    """Assembly + solve captured as one HIP graph (the persistent solve as a
    cooperative node): three replays, with eager work of the program between
    them (a different solve, a device copy, a synchronisation), each give the
    coefficients of the direct calls bit for bit."""
    import torch
    w = 4 if name == "cfg5" else 7
    log(f"case graph {name} w={w} samples={ns} {precision} batched={batched}")
    kw = dict(precision=precision, tol=1e-11, maxit=400, max_refine=3 if precision == "fp64" else 8,
              continue_cg=precision != "fp64", batched=batched)
    # a created stream (the legacy default stream cannot be captured), made
    # torch's current stream so that torch's reads follow the library's work
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        if name == "cfg5":
            fields = W.grf_samples(ns, n=24)
            P = S.Plan(W.config("cfg5", w=w, a=W._field("grid3d", data=fields[0])), nsamples=ns)
            fa = W._field("grid3d", data=torch.as_tensor(fields, device="cuda"))
        else:
            P = S.Plan(W.config(name, w=w))
            fa = None
        P.bind(stream=st)
        P.assemble(a=fa)
        rep = P.solve(**kw)
        assert np.all(rep["status"] == 0)
        ref = [P.coeffs(c).cpu().numpy() for c in range(P.ninst)]
        P.capture(a=fa, **kw)
        other = dict(kw, precision="fp64" if precision != "fp64" else "fp32", max_refine=8)
        for k in range(3):
            # eager work between replays: another solve overwrites the solution
            P.assemble(a=fa)
            P.solve(**other)
            junk = torch.arange(1 << 16, device="cuda", dtype=torch.float64) * (k + 1)
            junk2 = junk.clone()
            torch.cuda.synchronize()
            P.replay()
            torch.cuda.synchronize()
            for c in range(P.ninst):
                assert np.array_equal(P.coeffs(c).cpu().numpy(), ref[c]), (k, c)
            del junk, junk2


def test_narrow_build_parity_with_oracle(S):
    """A 3D launch with more tasks than workgroups runs the 256-thread build of
    the solve (whose reductions group the wavefronts differently): every
    sample's coefficients equal the oracle's direct solve (FP64, relative
    1e-10), checked on the first and last samples."""
    import torch
    import oracle as O
    ns, w = 16, 4
    log(f"case narrow build cfg5 w={w} samples={ns}")
    fields = W.grf_samples(ns, n=24)
    P = S.Plan(W.config("cfg5", w=w, a=W._field("grid3d", data=fields[0])), nsamples=ns)
    assert P.stats()["op_tasks"] > 256
    P.bind()
    P.assemble(a=W._field("grid3d", data=torch.as_tensor(fields, device="cuda")))
    rep = P.solve(precision="fp64", tol=1e-12, maxit=400, max_refine=3, schedule="lists")
    assert np.all(rep["status"] == 0)
    for s in (0, ns - 1):
        Po = O.Problem(W.config("cfg5", w=w, a=W._field("grid3d", data=fields[s])))
        ref = Po.split(Po.solve_all())
        for c in range(P.ncomp):
            nb = Po.nbasis(P.levels[c])
            x = P.coeffs(s * P.ncomp + c).cpu().numpy()
            r = ref[c][0][tuple(slice(1, -1) for _ in nb)].ravel()
            assert np.linalg.norm(x - r) <= 1e-10 * np.linalg.norm(r), (s, c)


def test_graph_released_by_rebind_and_network_change(S):
    """A captured step records the workspace (and network) addresses of its
    capture: binding the plan again, or attaching another network, releases
    it, and a replay is then refused (IGA_ERR_STATE) instead of touching the
    old memory."""
    import torch
    log("case graph released by rebind cfg2 w=6")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        P = S.Plan(W.config("cfg2", w=6))
        P.bind(stream=st)
        P.assemble()
        P.capture(precision="fp64", tol=1e-11, max_refine=3)
        P.replay()
        torch.cuda.synchronize()
        P.bind(stream=st)
        with pytest.raises(S.IgaError) as e:
            P.replay()
        assert e.value.code == 7
    log("case graph released by a network change cfg5 w=3")
    with torch.cuda.stream(st):
        P = S.Plan(W.config("cfg5", w=3, a=W._field("grid3d", data=W.grf_samples(1, n=24)[0])))
        P.bind(stream=st)
        P.assemble()
        net = S.Network((3, 4, 4, 1), device="cuda", stream=st)
        P.set_network(net)
        P.capture(precision="fp64", tol=1e-11, max_refine=3, learned=True)
        P.replay()
        torch.cuda.synchronize()
        P.set_network(S.Network((3, 4, 4, 1), device="cuda", stream=st))
        with pytest.raises(S.IgaError) as e:
            P.replay()
        assert e.value.code == 7
        torch.cuda.synchronize()


@pytest.mark.parametrize("name,precision,ns,w", [("cfg5", "fp64", 12, 4), ("cfg5", "fp32", 12, 4),
                                                  ("cfg5", "fp32", 2, 7), ("cfg3", "fp64", 1, 6),
                                                  ("cfg3", "bf16fd", 1, 6), ("cfg1", "fp64", 1, 6),
                                                  ("cfg2", "fp64", 1, 6), ("cfg2", "fp32", 1, 6)])
def test_whole_grid_solve_parity(S, name, precision, ns, w):
    """The whole-grid solve (one workgroup per grid, schedule 3) against the
    oracle's direct solves of the first and last samples (relative 1e-10 in
    FP64, 1e-9 in the mixed modes) and against the cooperative solve of the
    same launch (schedule 2: the same iteration, iteration counts within one)."""
    import torch
    import oracle as O
    log(f"case whole-grid {name} w={w} samples={ns} {precision}")
    kw = dict(precision=precision, tol=1e-12 if precision == "fp64" else 1e-11, tol_inner=1e-5, maxit=600,
              max_refine=3 if precision == "fp64" else 12, continue_cg=precision != "fp64")
    if name == "cfg5":
        fields = W.grf_samples(ns, n=24)
        wl0 = lambda s: W.config("cfg5", w=w, a=W._field("grid3d", data=fields[s]))
        P = S.Plan(wl0(0), nsamples=ns)
        P.bind()
        P.assemble(a=W._field("grid3d", data=torch.as_tensor(fields, device="cuda")))
    else:
        wl0 = lambda s: W.config(name, w=w)
        P = S.Plan(wl0(0))
        P.bind()
        P.assemble()
    rg = P.solve(schedule="grid", **kw)
    assert np.all(rg["status"] == 0)
    xg = [P.coeffs(c).cpu().numpy() for c in range(P.ninst)]
    rl = P.solve(schedule="lists", **kw)
    assert np.all(np.abs(rg["iters"] - rl["iters"]) <= 1)
    bar = 1e-10 if precision == "fp64" else 1e-9
    for c in range(P.ninst):
        xl = P.coeffs(c).cpu().numpy()
        assert np.linalg.norm(xg[c] - xl) <= bar * np.linalg.norm(xl), c
    for s in sorted({0, ns - 1}):
        Po = O.Problem(wl0(s))
        ref = Po.split(Po.solve_all())
        for c in range(P.ncomp):
            nb = Po.nbasis(P.levels[c])
            r = ref[c][0][tuple(slice(1, -1) for _ in nb)].ravel()
            x = xg[s * P.ncomp + c]
            assert np.linalg.norm(x - r) <= bar * np.linalg.norm(r), (s, c)
    log(f"  iterations grid {int(rg['total_iters'])} lists {int(rl['total_iters'])}")
