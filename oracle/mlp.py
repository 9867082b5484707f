"""Reference of the scoring network used by the learned rewrite proposal.

TEST INFRASTRUCTURE ONLY (imported by ``tests/``).

The paper fixes no proposal policy (its rewriting is the greedy rule
application of the appendix "Stabilizer decompositions"); the network here
is this project's reading: score(x) = w2 . relu(W1^T x + b1) + b2 with the
inputs x and the weights W1, w2 rounded to bf16 (round to nearest even)
before use.  Everything after the rounding is float64 here, so the HIP
kernels (fp32 sums) are compared with a tolerance.

Parameter vector layout (fp32 master): W1[16][256] (input major) | b1[256] |
w2[256] | b2.
"""
from __future__ import annotations

import numpy as np

IN, HID = 16, 256
P_W1, P_B1 = 0, IN * HID
P_W2 = P_B1 + HID
P_B2 = P_W2 + HID
NPARAM = P_B2 + 1


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bf16 value (ties to even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16_bits_to_float(h) -> np.ndarray:
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def unpack(param):
    p = np.asarray(param, dtype=np.float32)
    W1 = p[P_W1:P_B1].reshape(IN, HID)
    return W1, p[P_B1:P_W2], p[P_W2:P_B2], float(p[P_B2])


def forward(param, X, round_weights: bool = True):
    """Scores (float64) of the rows of X (rows x 16; float32 values or bf16
    bit patterns as uint16).  Also returns the pre-activations."""
    W1, b1, w2, b2 = unpack(param)
    X = np.asarray(X)
    Xf = bf16_bits_to_float(X) if X.dtype == np.uint16 else bf16_round(X)
    if round_weights:
        W1, w2 = bf16_round(W1), bf16_round(w2)
    pre = Xf.astype(np.float64) @ W1.astype(np.float64) + b1.astype(np.float64)
    h = np.maximum(pre, 0.0)
    return h @ w2.astype(np.float64) + b2, pre


def loss_and_dscore(score, cost, seg_off):
    """Softmax cross-entropy per segment toward its least-cost present rows:
    the target spreads evenly over every present row of least cost (rows
    with cost < 0 absent).  dscore = (softmax - target) / n_seg.  Returns
    (loss per segment, dscore)."""
    score = np.asarray(score, dtype=np.float64)
    cost = np.asarray(cost)
    n_seg = len(seg_off) - 1
    loss = np.zeros(n_seg)
    ds = np.zeros_like(score)
    for i in range(n_seg):
        a, b = int(seg_off[i]), int(seg_off[i + 1])
        rows = [r for r in range(a, b) if cost[r] >= 0]
        if not rows:
            continue
        best = min(cost[r] for r in rows)
        tgt = [r for r in rows if cost[r] == best]
        s = np.array([score[r] for r in rows])
        mx = s.max()
        e = np.exp(s - mx)
        z = e.sum()
        loss[i] = np.log(z) + mx - sum(score[r] for r in tgt) / len(tgt)
        for r, ei in zip(rows, e):
            ds[r] = (ei / z - (1.0 / len(tgt) if r in tgt else 0.0)) / n_seg
    return loss, ds


def backward(param, X, dscore):
    """Gradient of sum_r dscore[r] * score[r] with respect to the parameter
    vector, the bf16 rounding of W1 and w2 taken as the identity."""
    W1, b1, w2, b2 = unpack(param)
    X = np.asarray(X)
    Xf = (bf16_bits_to_float(X) if X.dtype == np.uint16 else bf16_round(X)).astype(np.float64)
    w2r = bf16_round(w2).astype(np.float64)
    _, pre = forward(param, X)
    h = np.maximum(pre, 0.0)
    d = np.asarray(dscore, dtype=np.float64)
    g = np.zeros(NPARAM)
    g[P_W2:P_B2] = h.T @ d
    g[P_B2] = d.sum()
    dpre = np.where(pre > 0.0, np.outer(d, w2r), 0.0)
    g[P_B1:P_W2] = dpre.sum(axis=0)
    g[P_W1:P_B1] = (Xf.T @ dpre).reshape(-1)
    return g


def adam(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (float64): returns (param, m, v)."""
    p = np.asarray(param, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
