"""iga_sg_bind_static (the entry point that allocates nothing) against
iga_sg_bind: the same plan bound to the library's static workspace gives the
same coefficients and combined values, on two bindings in a row, the second
with a smaller plan; a plan whose static binding was taken over by another
plan is refused, and a plan larger than the static workspace is rejected."""
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


def _run(S, wl, static, precision, xi):
    P = S.Plan(wl)
    if static:
        P.bind_static()
    else:
        P.bind()
    P.assemble()
    rep = P.solve(precision=precision, tol=1e-11, tol_inner=1e-5, max_refine=8,
                  continue_cg=precision != "fp64")
    u = P.combine(xi).cpu().numpy()
    x = [P.coeffs(c).cpu().numpy() for c in range(P.ncomp)]
    return P, rep, u, x


def _compare(ref, got):
    _, r0, u0, x0 = ref
    _, r1, u1, x1 = got
    assert np.array_equal(r0["iters"], r1["iters"])
    assert np.all(r1["status"] == 0)
    for c, (a, b) in enumerate(zip(x0, x1)):
        err = np.linalg.norm(a - b) / max(np.linalg.norm(a), 1e-300)
        assert err <= 1e-12, (c, err)
    err = np.linalg.norm(u0 - u1) / np.linalg.norm(u0)
    assert err <= 1e-12, err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_binding_equals_workspace_binding(S, precision):
    xi, _ = W.eval_points(2, 4096, lattice=16, seed=7)
    big = W.config("cfg2", w=9)
    small = W.config("cfg2", w=6)
    log(f"case cfg2 w=9 {precision}: workspace binding, then static binding")
    ref_big = _run(S, big, False, precision, xi)
    got_big = _run(S, big, True, precision, xi)
    _compare(ref_big, got_big)
    log(f"case cfg2 w=6 {precision}: second static binding, smaller plan")
    ref_small = _run(S, small, False, precision, xi)
    got_small = _run(S, small, True, precision, xi)
    _compare(ref_small, got_small)
    # the first static plan lost the array to the second one
    with pytest.raises(S.IgaError) as e:
        got_big[0].combine(xi)
    assert e.value.code == 7
    # rebinding it takes the array back and reproduces its solve
    log(f"case cfg2 w=9 {precision}: rebinding the first static plan")
    P = got_big[0]
    P.bind_static()
    P.assemble()
    P.solve(precision=precision, tol=1e-11, tol_inner=1e-5, max_refine=8, continue_cg=precision != "fp64")
    assert np.array_equal(P.combine(xi).cpu().numpy(), got_big[2])


def test_static_binding_3d(S):
    xi, _ = W.eval_points(3, 2048, lattice=4, seed=9)
    wl = W.config("cfg5", w=5, a=W._field("grid3d", data=W.grf_samples(1, n=24)[0]))
    log("case cfg5 w=5 fp64: workspace binding, then static binding")
    _compare(_run(S, wl, False, "fp64", xi), _run(S, wl, True, "fp64", xi))


def test_static_binding_rejects_large_plan(S):
    P = S.Plan(W.config("cfg5", w=7), nsamples=4)
    assert P.workspace_bytes() > 128 << 20
    log("case cfg5 w=7 x 4 samples: static binding refused (workspace beyond 128 MiB)")
    with pytest.raises(S.IgaError) as e:
        P.bind_static()
    assert e.value.code == 3
