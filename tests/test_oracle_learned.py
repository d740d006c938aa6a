"""Pins of the learned-preconditioner oracle (CPU): convolution against
brute-force loops and exact identities, gradients against central
differences, flexible CG against exactly known behaviour."""
import itertools

import numpy as np
import pytest

from oracle import learned as L


def _rng(seed=0):
    return np.random.Generator(np.random.PCG64(seed))


def test_shift_matches_index_definition():
    x = _rng(1).standard_normal((2, 3, 4, 5))
    for d3, d2, d1 in itertools.product((-1, 0, 1), repeat=3):
        y = L.shift(x, d3, d2, d1)
        for i3, i2, i1 in itertools.product(range(3), range(4), range(5)):
            j3, j2, j1 = i3 + d3, i2 + d2, i1 + d1
            want = x[:, j3, j2, j1] if (0 <= j3 < 3 and 0 <= j2 < 4 and 0 <= j1 < 5) else 0.0
            assert np.all(y[:, i3, i2, i1] == want)


def test_conv_brute_force_loops():
    rng = _rng(2)
    x = rng.standard_normal((2, 3, 4, 5))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    y = L.conv3d(x, w, b)
    n3, n2, n1 = x.shape[1:]
    for co in range(3):
        for i3, i2, i1 in itertools.product(range(n3), range(n2), range(n1)):
            s = b[co]
            for ci, t3, t2, t1 in itertools.product(range(2), range(3), range(3), range(3)):
                j3, j2, j1 = i3 + t3 - 1, i2 + t2 - 1, i1 + t1 - 1
                if 0 <= j3 < n3 and 0 <= j2 < n2 and 0 <= j1 < n1:
                    s += w[co, ci, t3, t2, t1] * x[ci, j3, j2, j1]
            assert abs(y[co, i3, i2, i1] - s) < 1e-12


def test_delta_kernels_identity_and_shift():
    x = _rng(3).standard_normal((1, 4, 5, 6))
    w = np.zeros((1, 1, 3, 3, 3))
    w[0, 0, 1, 1, 1] = 1.0
    assert np.array_equal(L.conv3d(x, w, np.zeros(1)), x)
    w[:] = 0.0
    w[0, 0, 1, 1, 2] = 1.0  # neighbour +1 in direction 1
    y = L.conv3d(x, w, np.zeros(1))
    assert np.array_equal(y[0, :, :, :-1], x[0, :, :, 1:]) and np.all(y[0, :, :, -1] == 0.0)


def test_adjoint_identity():
    rng = _rng(4)
    x = rng.standard_normal((3, 4, 3, 5))
    y = rng.standard_normal((2, 4, 3, 5))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    lhs = np.sum(L.conv3d(x, w, np.zeros(2)) * y)
    rhs = np.sum(x * L.conv3d_adjoint(y, w))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


@pytest.mark.parametrize("head", [0, 1])
def test_gradients_central_differences(head):
    rng = _rng(5)
    net = L.Net([3, 4, 4, 1], seed=7)
    x = rng.standard_normal((3, 3, 4, 5))
    t = rng.standard_normal((1, 3, 4, 5))
    count = t.size
    _, grads = net.loss_and_grad(x, t, count, head)
    h = 1e-6
    for li in range(3):
        w, b = net.layers[li]
        for idx in [tuple(rng.integers(0, s) for s in w.shape) for _ in range(6)]:
            w0 = w[idx]
            w[idx] = w0 + h
            lp, _ = net.loss_and_grad(x, t, count, head)
            w[idx] = w0 - h
            lm, _ = net.loss_and_grad(x, t, count, head)
            w[idx] = w0
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[li][0][idx]) < 1e-6 * max(1.0, abs(fd)), (li, idx)
        for k in range(b.shape[0]):
            b0 = b[k]
            b[k] = b0 + h
            lp, _ = net.loss_and_grad(x, t, count, head)
            b[k] = b0 - h
            lm, _ = net.loss_and_grad(x, t, count, head)
            b[k] = b0
            assert abs((lp - lm) / (2 * h) - grads[li][1][k]) < 1e-6


def test_flat_roundtrip_and_count():
    net = L.Net([3, 16, 16, 1], seed=0)
    f = net.flat()
    assert f.size == 3 * 16 * 27 + 16 + 16 * 16 * 27 + 16 + 16 * 27 + 1
    net2 = L.Net.from_flat([3, 16, 16, 1], f)
    for (w, b), (w2, b2) in zip(net.layers, net2.layers):
        assert np.array_equal(w, w2) and np.array_equal(b, b2)


def _spd(n, seed):
    rng = _rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return q @ np.diag(np.linspace(1.0, 300.0, n)) @ q.T


def test_fcg_exact_preconditioner_one_step():
    A = _spd(30, 6)
    b = _rng(7).standard_normal(30)
    x, it, _ = L.fcg(A, b, lambda r: np.linalg.solve(A, r), 1e-12, 50)
    assert it == 1 and np.linalg.norm(A @ x - b) < 1e-10 * np.linalg.norm(b)


def test_fcg_first_step_uses_prec0():
    """The first direction comes from prec0: with the exact inverse there and
    a useless prec afterwards, one step solves the system."""
    A = _spd(25, 13)
    b = _rng(14).standard_normal(25)
    x, it, _ = L.fcg(A, b, lambda r: r * 0.0 + r, 1e-12, 50, prec0=lambda r: np.linalg.solve(A, r))
    assert it == 1 and np.linalg.norm(A @ x - b) < 1e-10 * np.linalg.norm(b)


def test_fcg_with_linear_spd_preconditioner_equals_pcg():
    """For a fixed SPD preconditioner z.r_old = 0 in exact arithmetic, so the
    flexible iteration reproduces plain PCG (Fletcher-Reeves beta)."""
    A = _spd(40, 8)
    M = np.diag(np.diag(A))
    b = _rng(9).standard_normal(40)
    prec = lambda r: np.linalg.solve(M, r)
    _, it_f, hist_f = L.fcg(A, b, prec, 1e-10, 200)
    # plain PCG
    x = np.zeros(40)
    r = b.copy()
    z = prec(r)
    p = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r)]
    for k in range(200):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        hist.append(np.linalg.norm(r))
        if hist[-1] <= 1e-10 * np.linalg.norm(b):
            break
        z = prec(r)
        rzn = r @ z
        p = z + (rzn / rz) * p
        rz = rzn
    assert it_f == len(hist) - 1
    np.testing.assert_allclose(hist_f, hist, rtol=1e-6, atol=1e-12 * np.linalg.norm(b))


@pytest.mark.parametrize("head", [0, 1])
def test_preconditioner_scale_equivariant(head):
    rng = _rng(10)
    net = L.Net([3, 4, 4, 1], seed=3)
    r = rng.standard_normal((3, 4, 5))
    zfd = r + 0.1 * rng.standard_normal((3, 4, 5))
    la = rng.standard_normal((3, 4, 5))
    z1 = L.precondition(net, r, zfd, la, head)
    z2 = L.precondition(net, 7.5 * r, 7.5 * zfd, la, head)
    np.testing.assert_allclose(z2, 7.5 * z1, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("head", [0, 1])
def test_untrained_last_layer_gives_fd(head):
    """A zero last layer makes the correction vanish: z = z_FD exactly."""
    rng = _rng(11)
    net = L.Net([3, 4, 4, 1], seed=3)
    w, b = net.layers[-1]
    w[:] = 0.0
    b[:] = 0.0
    r = rng.standard_normal((3, 4, 5))
    zfd = rng.standard_normal((3, 4, 5))
    zfd *= np.sign(np.sum(r * zfd)) or 1.0
    assert np.array_equal(L.precondition(net, r, zfd, rng.standard_normal((3, 4, 5)), head), zfd)


def test_rejected_correction_falls_back_to_fd():
    """A correction that turns z against r (r.z <= 0) is discarded."""
    rng = _rng(12)
    net = L.Net([3, 1], seed=0)
    w, b = net.layers[0]
    w[:] = 0.0
    b[:] = -1e3  # additive head: z = z_FD - 1e3 s, r.z < 0 for r = z_FD > 0
    zfd = np.abs(rng.standard_normal((2, 3, 4))) + 0.1
    r = zfd.copy()
    assert np.array_equal(L.precondition(net, r, zfd, np.zeros_like(r), 0), zfd)


def test_to_bf16_rounding():
    """Rounding to bfloat16: torch's own conversion (round to nearest even)
    on random values, exact values kept, halfway cases to the even
    neighbour, and the relative error within half a unit of the last of
    its 8 significand bits (2^-8)."""
    import torch
    rng = _rng(21)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 8, 10000), [1.0, -2.5, 0.0]])
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = L.to_bf16(x)
    assert np.array_equal(got, want)
    assert L.to_bf16(1.0) == 1.0 and L.to_bf16(-2.5) == -2.5
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: to the even significand (1)
    assert L.to_bf16(1.0 + 2.0 ** -8) == 1.0
    assert L.to_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    nz = x != 0
    assert np.max(np.abs(got[nz] - x[nz]) / np.abs(x[nz])) <= 2.0 ** -8 * (1 + 1e-6)


def test_bf16_inference_close_to_exact():
    """The network in BF16 inference precision stays within the BF16 error
    of the exact forward pass (relative 2e-2 on the output of a random
    network), and equals it for weights and inputs that BF16 holds exactly
    and activations that stay exact (integer data, small sums)."""
    rng = _rng(22)
    net = L.Net((3, 8, 8, 1), seed=5)
    x = rng.standard_normal((3, 4, 5, 6))
    y = net.forward(x)[0]
    yb = net.infer_bf16(x)
    assert np.linalg.norm(yb - y) <= 2e-2 * np.linalg.norm(y)
    net2 = L.Net((3, 2, 2, 1), seed=0)
    net2.layers = [(rng.integers(-2, 3, w.shape).astype(float), rng.integers(-2, 3, b.shape).astype(float))
                   for w, b in net2.layers]
    xi = rng.integers(-2, 3, (3, 3, 3, 3)).astype(float)
    assert np.array_equal(net2.infer_bf16(xi), net2.forward(xi)[0])
