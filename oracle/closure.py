"""Oracle of the learned closure (test infrastructure only).

A plain FP64 numpy statement of the network that include/closure.h defines:
L periodic 3 x 3 cross-correlations (wrap-around at the grid edges), ReLU
between them, input channels (u_x, u_y, conditions), output added to u:

    X_1 = [u, cond],  Z_l[p][o] = sum_{tap, c} X_l[p + off(tap)][c] W_l[tap][c][o] + b_l[o],
    X_{l+1} = relu(Z_l),  pred = u + Z_L,

with off(tap) = (tap mod 3 - 1, floor(tap / 3) - 1) as (dx, dy).  The loss is
the mean of (pred - target)^2 over every value; the gradients are those of
that loss, by the chain rule written out layer by layer.  The network is
defined with BF16 weights and activations as the operands of its
convolutions (FP32-or-better sums): with bf16_ops=True the operands are
rounded to BF16 (nearest, ties to even) at exactly those points - the weights
and activations entering a convolution, and the output gradient entering an
input-gradient convolution - and every sum is FP64; with bf16_ops=False it is
the same network in plain FP64, which bounds what the BF16 operands cost.  Adam follows
Kingma & Ba (ICLR 2015), Algorithm 1.
"""
from __future__ import annotations

import numpy as np


def bf16(a):
    """Round to the nearest BF16 value (8 significant bits, ties to even)."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def shapes(c_in: int, width: int, layers: int):
    """(c_in, c_out) of every convolution."""
    return [(c_in if l == 0 else width, 2 if l == layers - 1 else width) for l in range(layers)]


def param_count(c_in: int, width: int, layers: int) -> int:
    return sum(9 * ci * co + co for ci, co in shapes(c_in, width, layers))


def unpack(params, c_in: int, width: int, layers: int):
    """[(W[9][ci][co], b[co]), ...] views of the flat parameter vector."""
    out, off = [], 0
    for ci, co in shapes(c_in, width, layers):
        W = np.asarray(params[off:off + 9 * ci * co], dtype=np.float64).reshape(9, ci, co)
        off += 9 * ci * co
        b = np.asarray(params[off:off + co], dtype=np.float64)
        off += co
        out.append((W, b))
    return out


def _shift(X, tap, sign):
    """Y[b, y, x] = X[b, (y + sign dy) mod M, (x + sign dx) mod M] for the tap's (dx, dy)."""
    dy, dx = tap // 3 - 1, tap % 3 - 1
    return np.roll(X, shift=(-sign * dy, -sign * dx), axis=(1, 2))


def conv(X, W, b):
    """Periodic 3 x 3 cross-correlation of X[B][M][M][ci] with W[9][ci][co], plus b."""
    Z = np.zeros(X.shape[:3] + (W.shape[2],))
    for tap in range(9):
        Z += _shift(X, tap, +1) @ W[tap]
    return Z + b


def forward(params, u, cond, c_in: int, width: int, layers: int, bf16_ops: bool = True):
    """pred [B][M][M][2] and the activations X_1 .. X_L."""
    u = np.asarray(u, dtype=np.float64)
    B, M = u.shape[0], u.shape[1]
    cond = np.asarray(cond, dtype=np.float64).reshape(B, c_in - 2)
    X = np.concatenate([u, np.broadcast_to(cond[:, None, None, :], (B, M, M, c_in - 2))], axis=3)
    rnd = bf16 if bf16_ops else (lambda a: a)
    X = rnd(X)
    acts = []
    layers_p = unpack(params, c_in, width, layers)
    for l, (W, b) in enumerate(layers_p):
        acts.append(X)
        Z = conv(X, rnd(W), b)
        if l < layers - 1:
            X = rnd(np.maximum(Z, 0.0))
        else:
            return u + Z, acts
    raise AssertionError("unreachable")


def loss_and_gradient(params, u, cond, target, c_in: int, width: int, layers: int,
                      bf16_ops: bool = True):
    """(loss, gradient in the parameter layout)."""
    pred, acts = forward(params, u, cond, c_in, width, layers, bf16_ops)
    d = pred - np.asarray(target, dtype=np.float64)
    n = d.size
    loss = float((d * d).sum() / n)
    rnd = bf16 if bf16_ops else (lambda a: a)
    layers_p = unpack(params, c_in, width, layers)
    grads = [None] * layers
    dZ = 2.0 * d / n
    for l in range(layers - 1, -1, -1):
        W, _ = layers_p[l]
        X = acts[l]
        gW = np.stack([np.einsum("bhwc,bhwo->co", _shift(X, tap, +1), dZ) for tap in range(9)])
        gb = dZ.sum(axis=(0, 1, 2))
        grads[l] = (gW, gb)
        if l > 0:
            dZr, Wr = rnd(dZ), rnd(W)
            dX = np.zeros(X.shape)
            for tap in range(9):
                dX += _shift(dZr, tap, -1) @ Wr[tap].T
            dZ = dX * (X > 0)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam(w, m, v, g, t: int, lr: float, b1: float, b2: float, eps: float):
    """One Adam step at step count t (>= 1); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
