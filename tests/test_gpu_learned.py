"""GPU checks of the learned preconditioner (through the C-ABI) against the
CPU oracle in oracle/learned.py.

  - network forward pass, loss and parameter gradients (both output heads)
    element by element against the oracle's FP64 loops: FP32 kernels, so
    1e-5 relative for the forward pass and 1e-4 for the gradients;
  - one Adam step against its closed-form update;
  - the training-pair features against the oracle's feature map;
  - k iterations of the in-kernel flexible CG against the oracle's flexible
    CG built only from oracle matrices (dense Galerkin operator, Kronecker
    pencil of the oracle's 1D matrices, oracle network and features);
  - the converged learned solve against the oracle's direct solves (1e-9),
    non-finite network weights falling back to the plain preconditioner,
    training by the library's kernels lowering the loss, and a report of the
    iterations and time of the learned and plain solves on held-out
    coefficient samples.
"""
import sys
import time

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import learned as OL

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


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _params(ch, seed, last_scale=0.1):
    """He-initialised layers with a random (not zero) last layer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for li, (cin, cout) in enumerate(zip(ch[:-1], ch[1:])):
        std = np.sqrt(2.0 / (27 * cin)) if li + 2 < len(ch) else last_scale
        out.append(rng.standard_normal(cout * cin * 27) * std)
        out.append(rng.standard_normal(cout) * 0.05)
    return np.concatenate(out).astype(np.float32)


@pytest.mark.parametrize("ch,nb,shape", [((3, 4, 5, 1), 2, (3, 4, 5)), ((3, 16, 16, 1), 3, (9, 7, 13))])
@pytest.mark.parametrize("head", [0, 1])
def test_network_forward_and_gradient(S, ch, nb, shape, head):
    import torch
    log(f"case nn ch={ch} nb={nb} shape={shape} head={head}")
    flat = _params(ch, seed=3)
    rng = np.random.Generator(np.random.PCG64(11))
    x = rng.standard_normal((nb, ch[0]) + shape).astype(np.float32)
    t = rng.standard_normal((nb, 1) + shape).astype(np.float32)
    net = S.Network(ch, flat, head=head)
    X = torch.as_tensor(x, device="cuda")
    T = torch.as_tensor(t, device="cuda")
    y = net.forward(X).cpu().numpy()
    onet = OL.Net.from_flat(ch, flat.astype(np.float64))
    yo = np.stack([onet.forward(x[b].astype(np.float64))[0] for b in range(nb)])
    assert rel(y, yo) < 1e-5
    loss = float(net.gradient(X, T).item())
    g = net.grads.cpu().numpy()
    lo, go = 0.0, None
    for b in range(nb):
        l, gr = onet.loss_and_grad(x[b].astype(np.float64), t[b].astype(np.float64), t.size, head)
        lo += l
        f = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in gr])
        go = f if go is None else go + f
    log(f"  forward rel {rel(y, yo):.2e} loss {loss:.6e} / {lo:.6e} grad rel {rel(g, go):.2e}")
    assert abs(loss - lo) < 1e-5 * abs(lo)
    assert rel(g, go) < 1e-4


def test_adam_step_closed_form(S):
    import torch
    log("case adam")
    rng = np.random.Generator(np.random.PCG64(5))
    ch = (3, 4, 1)
    p0 = rng.standard_normal(S.Network(ch).count).astype(np.float32)
    net = S.Network(ch, p0)
    m = np.zeros(p0.size)
    v = np.zeros(p0.size)
    p = p0.astype(np.float64)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    for step in range(1, 4):
        g = rng.standard_normal(p0.size).astype(np.float32)
        net.grads.copy_(torch.as_tensor(g, device="cuda"))
        net.adam(lr=lr, beta1=b1, beta2=b2, eps=eps)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g.astype(np.float64) ** 2
        p = p - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    assert rel(net.params.cpu().numpy(), p) < 1e-5


@pytest.mark.parametrize("head", [0, 1])
def test_pair_features(S, head):
    import torch
    log(f"case pair head={head}")
    rng = np.random.Generator(np.random.PCG64(8))
    n = 700
    r, zfd, la, xs, xk = (rng.standard_normal(n) for _ in range(5))
    dev = lambda a: torch.as_tensor(a, device="cuda")
    x, t = S.make_pair(dev(r), dev(zfd), dev(la), dev(xs), dev(xk), head=head)
    xo, s = OL.features(r, zfd, la)
    e = xs - xk
    to = (e - zfd) / s if head == 0 else e / s
    assert rel(x.cpu().numpy(), xo) < 1e-6
    assert rel(t.cpu().numpy(), to) < 1e-6


# ---------------------------------------------------------------------------
# learned solves on the random-field cube


def _cube(w, sample=0, nsamples=1):
    a = W.grf_samples(nsamples, n=24)[sample]
    return W.config("cfg5", w=w, a=W._field("grid3d", data=a))


def _oracle_perm(nb):
    """GPU interior lexicographic index -> index of the oracle's dense
    assembly (directions ordered by basis count, first one fastest)."""
    d = len(nb)
    ni = [n - 2 for n in nb]
    order = list(range(d))
    for a in range(d):
        for b in range(a + 1, d):
            if nb[order[b]] < nb[order[a]]:
                order[a], order[b] = order[b], order[a]
    idx = np.arange(int(np.prod(ni)))
    ik = [idx % ni[0], (idx // ni[0]) % ni[1], idx // (ni[0] * ni[1])]
    out, mult = np.zeros_like(idx), 1
    for k in order:
        out += ik[k] * mult
        mult *= ni[k]
    return out


def _oracle_1d(p, r, lev):
    line = {"degree": [1], "knots": [[0.0, 0.0, 1.0, 1.0]], "ctrl": np.array([[0.0], [1.0]]),
            "weights": None}
    P1 = O.Problem(W.workload("1d", 1, [line], p=p, r=r, w=0, lmin=0,
                              f={"kind": "const", "params": [1, 0, 0, 0], "data": None},
                              grading=[("uniform", 1.0)]))
    K, _ = P1.assemble_dense([lev], 0)
    M, _ = P1.assemble_dense([lev], O.MASS)
    return K, M


def _oracle_loga(Po, lv):
    """log a at the Greville points of the interior unknowns (identity
    geometry), GPU order (direction 1 fastest)."""
    p, r = int(Po.wl["p"]), int(Po.wl["r"])
    gre = []
    for lev in lv:
        kn = O.knots(p, r, int(lev))
        nbas = len(kn) - p - 1
        gre.append(np.array([np.mean(kn[i + 1:i + p + 1]) for i in range(1, nbas - 1)]))
    out = np.zeros((len(gre[2]), len(gre[1]), len(gre[0])))
    for i3, z in enumerate(gre[2]):
        for i2, y in enumerate(gre[1]):
            for i1, x in enumerate(gre[0]):
                out[i3, i2, i1] = np.log(Po.field("a", np.array([x, y, z])))
    return out.reshape(-1)


def test_learned_fcg_iterates_match_oracle(S):
    """x_k of the in-kernel flexible CG equals the oracle's flexible CG with
    the oracle network (plain preconditioner on the initial residual).  The
    solve infers in BF16 (features, weights and activations rounded to BF16,
    FP32 accumulation on the matrix cores); the oracle rounds the same
    quantities to BF16 and sums exactly, so the two differ by the FP32
    accumulation and the rare BF16 rounding it flips (bar 1e-3)."""
    wl = _cube(3)
    log("case learned fcg iterates cfg5 w=3")
    P = S.Plan(wl)
    P.bind()
    P.assemble()
    ch = (3, 32, 48, 1)
    flat = _params(ch, seed=21, last_scale=0.02)
    net = S.Network(ch, flat)
    P.set_network(net)
    onet = OL.Net.from_flat(ch, flat.astype(np.float64))
    Po = O.Problem(wl)
    p, r = int(wl["p"]), int(wl["r"])
    checked = 0
    for c, lv in enumerate(P.levels):
        nb = Po.nbasis(lv)
        ni = [n - 2 for n in nb]
        if int(np.prod(ni)) < 8:
            continue
        A, b = Po.assemble_dense(lv)
        perm = _oracle_perm(nb)
        Ag, bg = A[np.ix_(perm, perm)], b[perm]
        KM = [_oracle_1d(p, r, int(lv[k])) for k in range(3)]
        (K1, M1), (K2, M2), (K3, M3) = KM
        Pk = np.kron(M3, np.kron(M2, K1)) + np.kron(M3, np.kron(K2, M1)) + np.kron(K3, np.kron(M2, M1))
        la = _oracle_loga(Po, lv)
        assert rel(P.loga(c).cpu().numpy(), la) < 1e-12
        shp = (ni[2], ni[1], ni[0])

        def prec(res):
            zfd = np.linalg.solve(Pk, res)
            return OL.precondition(onet, res.reshape(shp), zfd.reshape(shp), la.reshape(shp), bf16=True).reshape(-1)

        for k in (1, 2, 4):
            xo, _, _ = OL.fcg(Ag, bg, prec, 1e-30, k, prec0=lambda res: np.linalg.solve(Pk, res))
            P.solve(precision="fp64", tol=1e-30, maxit=k, max_refine=1, learned=True, check=False,
                    scaled=False)
            xg = P.coeffs(c).cpu().numpy()
            e = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
            log(f"  comp {c} {lv.tolist()} k={k} rel {e:.2e}")
            assert e < 1e-3, (c, k, e)
        checked += 1
        if checked == 4:
            break
    assert checked == 4


def _solve_vs_oracle(P, wl, learned, tol, learned_iters=0, precision="fp64"):
    mixed = precision != "fp64"
    rep = P.solve(precision=precision, tol=1e-11, maxit=600, max_refine=12 if mixed else 4, learned=learned,
                  learned_iters=learned_iters, continue_cg=mixed, check=False)
    assert rep["code"] == 0 and np.all(rep["status"] == 0), rep["code"]
    Po = O.Problem(wl)
    coefs = Po.solve_all()
    worst = 0.0
    for c, (lv, co) in enumerate(zip(P.levels, Po.split(coefs))):
        ref = co[0][(slice(1, -1),) * 3].reshape(-1)
        worst = max(worst, np.linalg.norm(P.coeffs(c).cpu().numpy() - ref) / np.linalg.norm(ref))
    xi, _ = W.eval_points(3, 2048, lattice=8, seed=12345)
    u = P.combine(xi).cpu().numpy()
    u_ref = Po.sg_eval(coefs, xi)
    e_sg = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    log(f"  learned={learned} iters {rep['total_iters']} worst coef rel {worst:.2e} u_sg rel {e_sg:.2e}")
    assert worst < tol and e_sg < tol
    return rep


def test_learned_solve_parity_and_fallback(S):
    wl = _cube(4)
    log("case learned solve parity cfg5 w=4")
    P = S.Plan(wl)
    P.bind()
    P.assemble()
    ch = (3, 32, 48, 1)
    net = S.Network(ch, _params(ch, seed=4, last_scale=0.02))
    P.set_network(net)
    rep_plain = _solve_vs_oracle(P, wl, False, 1e-10)
    # an untrained (random) network: the correction acts on the first ten
    # preconditionings of each solve, plain fast diagonalisation after them
    _solve_vs_oracle(P, wl, True, 1e-9, learned_iters=10)
    # FP32 inner solves with the correction, FP64 refinement judged by the
    # plain preconditioner; a milder random correction (a large random one
    # can stall FP32 flexible CG into p.Ap <= 0, a breakdown)
    P.set_network(S.Network(ch, _params(ch, seed=4, last_scale=0.005)))
    _solve_vs_oracle(P, wl, True, 1e-9, learned_iters=10, precision="fp32")
    P.set_network(net)
    # non-finite weights: every learned step is rejected, the plain
    # preconditioner takes over and the iteration is the plain one
    bad = S.Network(ch, np.full(net.count, np.nan, dtype=np.float32))
    P.set_network(bad)
    rep_nan = _solve_vs_oracle(P, wl, True, 1e-10)
    d = np.abs(rep_nan["iters"] - rep_plain["iters"])
    assert d.max() <= 1, (rep_nan["iters"], rep_plain["iters"])
    P.set_network(None)
    with pytest.raises(S.IgaError):
        P.solve(precision="fp64", learned=True)


def test_training_lowers_loss_and_report_gain(S):
    """Train on the library's kernels (pairs from the plain PCG on training
    samples), then solve held-out samples with the trained correction on
    every iteration of flexible CG: every grid converges (status 0), the
    solutions equal the oracle's direct solves (1e-9), at w=5 and, with the
    same network, at w=7 on a 64^3 field.  Iterations and time of the
    learned and plain solves are reported; the gain is not asserted (on
    these problems the trained correction costs iterations against the
    diagonally scaled fast diagonalisation alone)."""
    import torch
    from paper_1707_09598_amd import learn
    w, ntr, nte = 5, 6, 2
    log(f"case learned training cfg5 w={w} train {ntr} held-out {nte}")
    fields = W.grf_samples(ntr + nte, n=24)

    def plan_for(a, level=w):
        P = S.Plan(W.config("cfg5", w=level, a=W._field("grid3d", data=a)))
        P.bind()
        P.assemble()
        return P

    pairs, P0 = {}, None
    for s in range(ntr):
        P = plan_for(fields[s])
        learn.collect_pairs(P, pairs=pairs)
        P0 = P0 or P
    shapes = {c: learn.grid_shape(P0, c) for c in range(P0.ncomp)}
    ch = (3, 32, 48, 1)
    net = S.Network(ch, learn.init_params(ch, seed=0))
    assert net.count == 45441
    before = learn.evaluate(net, pairs, shapes)
    learn.train(net, pairs, shapes, steps=600, lr=2e-3, batch=16, seed=1)
    after = learn.evaluate(net, pairs, shapes)
    log(f"  training loss over all pairs: before {before:.4e} after {after:.4e}")
    assert after < before

    def held_out(P, wl, tag):
        P.set_network(net)
        res = {}
        for key, mode, k in (("plain", False, 0), ("learned", True, 0), ("learned-10", True, 10)):
            P.assemble()
            rep = P.solve(precision="fp64", tol=1e-11, maxit=600, max_refine=4, learned=mode,
                          learned_iters=k, check=False)
            assert rep["code"] == 0 and np.all(rep["status"] == 0), (tag, key, rep["status"])
            if key == "learned":
                Po = O.Problem(wl)
                xi, _ = W.eval_points(3, 2048, lattice=8, seed=12345)
                u = P.combine(xi).cpu().numpy()
                u_ref = Po.sg_eval(Po.solve_all(), xi)
                e = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
                log(f"  {tag} learned on every iteration: u_sg rel {e:.2e} against the oracle")
                assert e <= 1e-9
            P.assemble()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.solve_async(precision="fp64", tol=1e-11, maxit=600, max_refine=4, learned=mode, learned_iters=k)
            torch.cuda.synchronize()
            res[key] = (rep["total_iters"], 1e3 * (time.perf_counter() - t0))
        log(f"  {tag}: " + " | ".join(f"{k} {v[0]} iterations {v[1]:.2f} ms" for k, v in res.items()))

    for s in range(ntr, ntr + nte):
        held_out(plan_for(fields[s]), W.config("cfg5", w=w, a=W._field("grid3d", data=fields[s])), f"sample {s} w={w}")
    a7 = W.grf_samples(1, n=64, first_seed=ntr)[0]
    held_out(plan_for(a7, 7), W.config("cfg5", w=7, a=W._field("grid3d", data=a7)), "sample 6 w=7 64^3 field")
