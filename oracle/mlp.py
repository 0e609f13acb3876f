"""CPU oracle, part 5: the root-scoring MLP in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network is a project addition, not part of the paper (parity of what it
learns is unpinned by the paper; its arithmetic is pinned here).
16 inputs -> 64 -> 64 -> 1 with ReLU; parameter vector layout
    W1[64][16] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3      (5313 values).
The GPU keeps FP32 master weights and computes with their BF16 rounding
(round to nearest, ties to even) and FP32 accumulation.  This oracle applies
the same BF16 rounding to the weights and then works in FP64 throughout:
forward pass, the weighted logistic loss
    loss = (1/B) sum_i c_i (softplus(z_i) - y_i z_i),  c_i = pos_weight if y_i else 1,
its gradient by backpropagation, and one Adam step (beta1 0.9, beta2 0.999,
eps 1e-8, bias corrected).
"""
from __future__ import annotations

import numpy as np

NFEAT = 16
HID = 64
NPARAM = HID * NFEAT + HID + HID * HID + HID + HID + 1


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32.  bfloat16 keeps the upper 16 bits of the float32 pattern, so
    rounding adds half an ulp of the kept part (0x7fff, plus 1 when the kept
    part is odd) and clears the low 16 bits.  Inf and NaN pass unchanged."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    special = (b & 0x7F800000) == 0x7F800000
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    r = np.where(special, b, r).astype(np.uint32)
    return r.view(np.float32)


def unpack(w):
    """Split a parameter vector into (W1, b1, W2, b2, W3, b3), float64."""
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    assert w.size == NPARAM
    o = 0
    W1 = w[o:o + HID * NFEAT].reshape(HID, NFEAT); o += HID * NFEAT
    b1 = w[o:o + HID]; o += HID
    W2 = w[o:o + HID * HID].reshape(HID, HID); o += HID * HID
    b2 = w[o:o + HID]; o += HID
    W3 = w[o:o + HID]; o += HID
    b3 = w[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(W3),
                           np.atleast_1d(b3)]).astype(np.float64)


def effective(w32) -> np.ndarray:
    """The weights the kernels compute with: BF16 rounding of the FP32
    master weights, as float64."""
    return bf16_round(np.asarray(w32, dtype=np.float32)).astype(np.float64)


def forward(w, X):
    """Logits of the rows of X (float64 math on the given weights)."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ W3 + b3


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def loss(w, X, y, pos_weight=1.0) -> float:
    z = forward(w, X)
    y = np.asarray(y, dtype=np.float64)
    c = np.where(y > 0, pos_weight, 1.0)
    return float(np.mean(c * (softplus(z) - y * z)))


def loss_and_grad(w, X, y, pos_weight=1.0):
    """Loss and its gradient with respect to the parameter vector w, by
    backpropagation through the two ReLU layers."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    B = X.shape[0]
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3 + b3
    c = np.where(y > 0, pos_weight, 1.0)
    L = float(np.mean(c * (softplus(z) - y * z)))
    dz = c * (1.0 / (1.0 + np.exp(-z)) - y) / B          # d loss / d z_i
    gW3 = h2.T @ dz
    gb3 = dz.sum()
    d2 = np.outer(dz, W3) * (a2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (a1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    return L, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
