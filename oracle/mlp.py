"""Float64 reference of the schedule selector (test infrastructure).

The sparsity features are their plain definitions over pos/crd; the network
is 7 -> 64 -> 64 -> K with ReLU, inputs standardized as (x - mu) * istd; the
loss is the mean squared error over the batch and the K outputs; the
gradient is the chain rule written out layer by layer; the optimizer is
Adam (Kingma and Ba, ICLR 2015) with bias correction.  Parameters use the
same flat layout as the GPU library: W1[64][7], b1[64], W2[64][64], b2[64],
W3[K][64], b3[K].
"""
from __future__ import annotations

import numpy as np

IN, HID = 7, 64


def features(pos, crd, m):
    """The seven features of a CSR matrix (n rows, m columns)."""
    pos = np.asarray(pos, dtype=np.int64)
    crd = np.asarray(crd, dtype=np.int64)
    n = len(pos) - 1
    deg = np.diff(pos).astype(np.float64)
    rows = max(n, 1)
    nnz = deg.sum()
    mean = nnz / rows
    var = max(0.0, float((deg * deg).sum() / rows - mean * mean))
    bw = 0.0
    span = 0.0
    empty = 0
    for i in range(n):
        if pos[i + 1] > pos[i]:
            first, last = crd[pos[i]], crd[pos[i + 1] - 1]
            bw = max(bw, abs(first - i), abs(last - i))
            span += last - first + 1
        else:
            empty += 1
    nonempty = max(1, rows - empty)
    return np.array([np.log2(rows), np.log2(nnz + 1), mean, np.log2(1 + var),
                     np.log2(1 + (deg.max() if n else 0.0)), np.log2(1 + bw),
                     span / nonempty / max(m, 1)])


def unpack(P, K):
    P = np.asarray(P, dtype=np.float64)
    o = 0
    out = []
    for shape in ((HID, IN), (HID,), (HID, HID), (HID,), (K, HID), (K,)):
        size = int(np.prod(shape))
        out.append(P[o:o + size].reshape(shape))
        o += size
    assert o == len(P), (o, len(P))
    return out


def param_count(K):
    return HID * IN + HID + HID * HID + HID + K * HID + K


def forward(P, K, X, norm=None):
    """Returns Y (B x K) and the activations (x, z1, h1, z2, h2)."""
    W1, b1, W2, b2, W3, b3 = unpack(P, K)
    x = np.asarray(X, dtype=np.float64)
    if norm is not None:
        norm = np.asarray(norm, dtype=np.float64)
        x = (x - norm[:IN]) * norm[IN:]
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    Y = h2 @ W3.T + b3
    return Y, (x, z1, h1, z2, h2)


def loss_and_grad(P, K, X, T, norm=None):
    """Mean squared error and its gradient with respect to P (flat)."""
    W1, b1, W2, b2, W3, b3 = unpack(P, K)
    Y, (x, z1, h1, z2, h2) = forward(P, K, X, norm)
    T = np.asarray(T, dtype=np.float64)
    B = Y.shape[0]
    E = Y - T
    loss = float(np.mean(E * E))
    dY = 2.0 * E / (B * K)
    gW3 = dY.T @ h2
    gb3 = dY.sum(0)
    dh2 = dY @ W3
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam(P, m, v, g, lr, b1, b2, eps, step):
    """One Adam step; returns new (P, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return P - lr * mh / (np.sqrt(vh) + eps), m, v
