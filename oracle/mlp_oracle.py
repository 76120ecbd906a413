"""CPU FP64 oracle of the learned Front2VOF surrogate.

TEST INFRASTRUCTURE: only tests, the smoke check and the CPU-baseline leg of
the benchmark use it.

The surrogate is not part of the paper: it approximates the volume fraction
that Front2VOF (paper sec. 2.5) computes for a cell from the cell's own
description: the 12 edge-marker fractions (0 where an edge carries none;
edge id 4e + oA + 2 oB along axis e with offsets oA, oB on the two other axes
A < B) and the 8 corner colours (corner k = ox + 2 oy + 4 oz).

Network (READING of the stated design): 20 -> 128 -> 128 -> 1,
    z1 = x W1 + b1,  h1 = relu(z1)
    z2 = h1 W2 + b2, h2 = relu(z2)
    z3 = h2 . w3 + b3, y = sigmoid(z3)
loss = mean over the batch of (y - c)^2; Adam (beta1 0.9, beta2 0.999,
eps 1e-8) with bias correction.

Parameter vector (float32 master copy on the GPU), in this order:
W1 (20 x 128, row-major in x out), b1 (128), W2 (128 x 128), b2 (128),
w3 (128), b3 (1): 19329 numbers.

With ``bf16=True`` the functions round to bfloat16 (round to nearest even)
at the points where the GPU kernels do: the inputs, W1, W2, h1 before the
second product, and in the backward pass dz2 and dz1 before their products.
"""
from __future__ import annotations

import numpy as np

NIN, NH = 20, 128
SIZES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SIZES:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) through float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(a, on):
    return bf16(a) if on else a


def forward(theta, X, bf16_mode=False, keep=False):
    """y for rows X (m x 20)."""
    p = unpack(theta)
    X = _r(np.asarray(X, dtype=np.float64), bf16_mode)
    W1, W2 = _r(p["W1"], bf16_mode), _r(p["W2"], bf16_mode)
    z1 = X @ W1 + p["b1"]
    h1 = np.maximum(z1, 0.0)
    h1r = _r(h1, bf16_mode)
    z2 = h1r @ W2 + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["w3"] + p["b3"][0]
    y = 1.0 / (1.0 + np.exp(-z3))
    if keep:
        return y, dict(X=X, W1=W1, W2=W2, z1=z1, h1r=h1r, z2=z2, h2=h2, y=y)
    return y


def loss_and_grad(theta, X, c, bf16_mode=False):
    """Mean squared error and its gradient with respect to theta."""
    m = X.shape[0]
    p = unpack(theta)
    y, t = forward(theta, X, bf16_mode, keep=True)
    c = np.asarray(c, dtype=np.float64)
    loss = np.mean((y - c) ** 2)
    dz3 = (2.0 / m) * (y - c) * y * (1.0 - y)
    g = {}
    g["w3"] = t["h2"].T @ dz3
    g["b3"] = np.array([dz3.sum()])
    dz2 = np.outer(dz3, p["w3"]) * (t["z2"] > 0)
    g["b2"] = dz2.sum(axis=0)
    dz2r = _r(dz2, bf16_mode)
    g["W2"] = t["h1r"].T @ dz2r
    dh1 = dz2r @ t["W2"].T
    dz1 = dh1 * (t["z1"] > 0)
    g["b1"] = dz1.sum(axis=0)
    dz1r = _r(dz1, bf16_mode)
    g["W1"] = t["X"].T @ dz1r
    return loss, pack(g)


class Adam:
    """Adam with bias correction (Kingma and Ba)."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def cell_features(flags, s, cells):
    """Surrogate inputs of the cells (flat node indices) of a state given as
    numpy arrays (n,n,n): 12 marker fractions (0 without marker) then 8
    corner colours."""
    n = flags.shape[0]
    f = flags.ravel()
    sv = [x.ravel() for x in s]
    cells = np.asarray(cells, dtype=np.int64)
    x = cells % n
    y = (cells // n) % n
    z = cells // (n * n)
    X = np.zeros((len(cells), NIN))
    for e in range(3):
        others = [a for a in range(3) if a != e]
        for oB in (0, 1):
            for oA in (0, 1):
                off = [0, 0, 0]
                off[others[0]] = oA
                off[others[1]] = oB
                q = (x + off[0]) % n + n * (((y + off[1]) % n) + n * ((z + off[2]) % n))
                has = (f[q] >> (4 + e)) & 1
                X[:, 4 * e + oA + 2 * oB] = np.where(has == 1, sv[e][q], 0.0)
    for k in range(8):
        ox, oy, oz = k & 1, (k >> 1) & 1, (k >> 2) & 1
        q = (x + ox) % n + n * (((y + oy) % n) + n * ((z + oz) % n))
        X[:, 12 + k] = f[q] & 1
    return X
