"""Plain CPU reference (numpy, FP64) for the learned preconditioner.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library shares no code with it.

A small convolutional network acts on the tensor grid of one component: three
3x3x3 convolutions with zero padding ("same" size), ReLU between them.  Its
input channels are the normalised residual, the normalised fast-diagonalisation
output and the centred log-coefficient at the unknowns; its output y corrects
the fast-diagonalisation output z_FD, either additively (head 0:
z = z_FD + s y, s = ||z_FD||) or as a pointwise log-scale (head 1:
z = z_FD exp(y)).  A corrected z that is not a descent direction (r.z <= 0) is
replaced by z_FD.  The network is trained by minimising the mean squared error
of the predicted z / s against e / s on pairs (r, e) with A e = r taken from
the iterates of the plain preconditioned CG.  Flexible CG (Polak-Ribiere beta)
uses it as a variable preconditioner.

Tensors are [channels, n3, n2, n1] (direction 1 fastest), weights
[c_out, c_in, 3, 3, 3] indexed [.., t3, t2, t1] with tap t acting on the
neighbour at offset t - 1.  Parity unpinned: none (the pins are in
tests/test_oracle_learned.py).
"""
from __future__ import annotations

from typing import Callable, List, Sequence, Tuple

import numpy as np


def to_bf16(x) -> np.ndarray:
    """x rounded to bfloat16 (8 significand bits; nearest, ties to even)
    through float32, as FP32 values are converted on the GPU; returned as
    float64 (finite inputs)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(x: np.ndarray, d3: int, d2: int, d1: int) -> np.ndarray:
    """y[..., i3, i2, i1] = x[..., i3 + d3, i2 + d2, i1 + d1], zero outside."""
    y = np.zeros_like(x)
    n3, n2, n1 = x.shape[-3:]

    def rng(d, n):
        lo, hi = max(0, -d), min(n, n - d)
        return slice(lo, hi), slice(lo + d, hi + d)

    (a3, b3), (a2, b2), (a1, b1) = rng(d3, n3), rng(d2, n2), rng(d1, n1)
    y[..., a3, a2, a1] = x[..., b3, b2, b1]
    return y


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[co] = b[co] + sum_ci sum_taps w[co, ci, t3, t2, t1] x[ci](i + t - 1)."""
    cout = w.shape[0]
    y = np.zeros((cout,) + x.shape[1:])
    for t3 in range(3):
        for t2 in range(3):
            for t1 in range(3):
                xs = shift(x, t3 - 1, t2 - 1, t1 - 1)
                y += np.einsum("oc,c...->o...", w[:, :, t3, t2, t1], xs)
    return y + b[:, None, None, None]


def conv3d_adjoint(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of x -> conv3d(x, w, 0): dx[ci] = sum_co sum_taps w[co, ci, t] dy[co](i - t + 1)."""
    cin = w.shape[1]
    dx = np.zeros((cin,) + dy.shape[1:])
    for t3 in range(3):
        for t2 in range(3):
            for t1 in range(3):
                ys = shift(dy, 1 - t3, 1 - t2, 1 - t1)
                dx += np.einsum("oc,o...->c...", w[:, :, t3, t2, t1], ys)
    return dx


def conv3d_weight_grad(x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """dL/dw[co, ci, t] = sum_i dy[co](i) x[ci](i + t - 1)."""
    g = np.zeros((dy.shape[0], x.shape[0], 3, 3, 3))
    for t3 in range(3):
        for t2 in range(3):
            for t1 in range(3):
                xs = shift(x, t3 - 1, t2 - 1, t1 - 1)
                g[:, :, t3, t2, t1] = np.einsum("oijk,cijk->oc", dy, xs)
    return g


class Net:
    """Parameters of the network: list of (w, b) per layer."""

    def __init__(self, channels: Sequence[int], seed: int = 0):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.layers: List[Tuple[np.ndarray, np.ndarray]] = []
        for cin, cout in zip(channels[:-1], channels[1:]):
            std = np.sqrt(2.0 / (27 * cin))  # He initialisation
            self.layers.append((rng.standard_normal((cout, cin, 3, 3, 3)) * std, np.zeros(cout)))

    @staticmethod
    def from_flat(channels: Sequence[int], flat: np.ndarray) -> "Net":
        net = Net.__new__(Net)
        net.layers = []
        off = 0
        for cin, cout in zip(channels[:-1], channels[1:]):
            nw = cout * cin * 27
            w = flat[off:off + nw].reshape(cout, cin, 3, 3, 3).astype(np.float64)
            off += nw
            b = flat[off:off + cout].astype(np.float64)
            off += cout
            net.layers.append((w, b))
        return net

    def flat(self) -> np.ndarray:
        return np.concatenate([np.concatenate([w.ravel(), b]) for w, b in self.layers])

    def forward(self, x: np.ndarray):
        """Output and the activations needed by the backward pass."""
        acts = [x]
        h = x
        for li, (w, b) in enumerate(self.layers):
            h = conv3d(h, w, b)
            if li + 1 < len(self.layers):
                h = np.maximum(h, 0.0)
            acts.append(h)
        return h, acts

    def infer_bf16(self, x: np.ndarray) -> np.ndarray:
        """Output in the solve's inference precision: the input features, the
        weights and every hidden activation rounded to BF16 (the activations
        after bias and ReLU, through FP32), the sums formed exactly (FP64),
        the output rounded to FP32."""
        h = to_bf16(x)
        for li, (w, b) in enumerate(self.layers):
            h = conv3d(h, to_bf16(w), b).astype(np.float32).astype(np.float64)
            if li + 1 < len(self.layers):
                h = to_bf16(np.maximum(h, 0.0))
        return h

    def loss_and_grad(self, x: np.ndarray, t: np.ndarray, count: int, head: int = 0):
        """L = sum (pred - t)^2 / (2 count) and its gradients (list of (dw, db));
        pred = y (head 0) or x[1] exp(y) (head 1)."""
        y, acts = self.forward(x)
        if head == 0:
            pred, dpred = y, 1.0
        else:
            pred = x[1:2] * np.exp(y)
            dpred = pred  # d pred / d y
        d = (pred - t) * dpred / count
        loss = 0.5 * float(np.sum((pred - t) ** 2)) / count
        grads = [None] * len(self.layers)
        for li in range(len(self.layers) - 1, -1, -1):
            w, b = self.layers[li]
            xin = acts[li]
            grads[li] = (conv3d_weight_grad(xin, d), d.sum(axis=(1, 2, 3)))
            if li > 0:
                d = conv3d_adjoint(d, w) * (acts[li] > 0.0)
        return loss, grads


def features(r: np.ndarray, zfd: np.ndarray, loga: np.ndarray) -> Tuple[np.ndarray, float]:
    """Network input [3, n3, n2, n1] and the scale s = ||z_FD||."""
    sr = float(np.linalg.norm(r))
    sr = sr if sr > 0 else 1.0
    s = float(np.linalg.norm(zfd))
    s = s if s > 0 else 1.0
    la = loga - loga.mean()
    return np.stack([r / sr, zfd / s, la]), s


def precondition(net: Net, r: np.ndarray, zfd: np.ndarray, loga: np.ndarray, head: int = 0,
                 bf16: bool = False) -> np.ndarray:
    """z = z_FD + s y (head 0) or z_FD exp(y) (head 1) with
    y = N(r / ||r||, z_FD / s, log a - mean), s = ||z_FD||; z_FD itself when
    the corrected z is not a descent direction.  bf16: the network in the
    solve's inference precision (Net.infer_bf16)."""
    x, s = features(r, zfd, loga)
    y = net.infer_bf16(x) if bf16 else net.forward(x)[0]
    z = zfd + s * y[0] if head == 0 else zfd * np.exp(y[0])
    rz = float(np.sum(r * z))
    return z if (rz > 0.0 and np.isfinite(rz)) else zfd


def fcg(A: np.ndarray, b: np.ndarray, prec: Callable[[np.ndarray], np.ndarray], tol: float,
        maxit: int, prec0: Callable[[np.ndarray], np.ndarray] = None) -> Tuple[np.ndarray, int, List[float]]:
    """Flexible CG with the Polak-Ribiere beta: beta = z_k.(r_k - r_{k-1}) / (z_{k-1}.r_{k-1}).
    The initial residual is preconditioned by prec0 (default prec): the
    learned solve keeps the plain preconditioner for it.  Stops when
    ||r|| <= tol ||b||.  Returns x, iterations, residual history."""
    x = np.zeros_like(b)
    r = b.copy()
    z = (prec0 or prec)(r)
    p = z.copy()
    rz = float(r @ z)
    hist = [float(np.linalg.norm(r))]
    nb = float(np.linalg.norm(b))
    for k in range(1, maxit + 1):
        q = A @ p
        alpha = rz / float(p @ q)
        x += alpha * p
        r_old = r
        r = r - alpha * q
        hist.append(float(np.linalg.norm(r)))
        if hist[-1] <= tol * nb:
            return x, k, hist
        z = prec(r)
        rz_new = float(r @ z)
        beta = (rz_new - float(z @ r_old)) / rz
        p = z + beta * p
        rz = rz_new
    return x, maxit, hist
