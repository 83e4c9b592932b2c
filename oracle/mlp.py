"""FP64 reference of the learned-restart network and its trajectory
features -- TEST INFRASTRUCTURE (see oracle/__init__.py for the rules).

Network: 32 -> 128 -> 128 -> 1, ReLU, sigmoid output, mean binary
cross-entropy; parameters in one vector ordered W1 [128][32], b1 [128],
W2 [128][128], b2 [128], w3 [128], b3.  Written from the definitions
(matrix products, chain rule); pinned by finite differences and closed forms
in tests/test_oracle_mlp.py.  forward_bf16 / grad_bf16 are the same network
with each hidden layer's input rounded to bf16 (the operand precision of the
matrix cores), differentiated straight through the roundings; pinned by their
reduction to forward / grad where every rounding is exact and by a case
rounded by hand.

Features (per replica and checkpoint), about the first component x_{p,1}
(the one the anneal keeps and the readout reads): its Rayleigh quotient per
spin -(x_1^T J x_1) / (n x_1^T x_1), the Ising energy per spin of the sign
readout, its share of the squared norm, and the fraction of signs flipped
since the previous checkpoint -- written from those definitions with the
oracle's pinned energy and readout routines.  Standardization within each
pump's batch of runs and the top-k selection of the restart policy are
written out from their definitions too.
"""
from __future__ import annotations

import numpy as np

import oracle

F, H1, H2 = 32, 128, 128
SHAPES = (("W1", (H1, F)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)), ("w3", (H2,)), ("b3", (1,)))
PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    out, off = {}, 0
    for name, shp in SHAPES:
        size = int(np.prod(shp))
        out[name] = w[off:off + size].reshape(shp)
        off += size
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(x, w):
    """logit [B], h1 [B][128], h2 [B][128] (post-ReLU)."""
    p = unpack(w)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.maximum(x @ p["W1"].T + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    z = h2 @ p["w3"] + p["b3"][0]
    return z, h1, h2


def forward_bf16(x, w):
    """The network as the matrix cores evaluate it: each hidden layer's input
    (the features, then the first layer's activations) rounded to bf16, the
    rest exact.  Returns logit [B], the rounded h1 [B][128] and h2 [B][128]."""
    p = unpack(w)
    x = bf16_round(x)
    h1 = bf16_round(np.maximum(x @ p["W1"].T + p["b1"], 0.0))
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    z = h2 @ p["w3"] + p["b3"][0]
    return z, h1, h2


def _bce(z, y):
    return float(np.mean(np.logaddexp(0.0, z) - np.asarray(y, dtype=np.float64) * z))


def loss(x, y, w):
    """Mean binary cross-entropy of sigmoid(logit) against labels y."""
    return _bce(forward(x, w)[0], y)


def loss_bf16(x, y, w):
    """The mean binary cross-entropy of forward_bf16's logits."""
    return _bce(forward_bf16(x, w)[0], y)


def grad(x, y, w):
    """Gradient of the mean BCE by the chain rule."""
    x = np.asarray(x, dtype=np.float64)
    return _chain(x, y, unpack(w), *forward(x, w))


def grad_bf16(x, y, w):
    """The chain rule through forward_bf16 with each rounding taken as the
    identity (its derivative almost everywhere is zero, so this is the
    straight-through gradient): the weight gradients of a layer use its
    rounded input."""
    return _chain(bf16_round(x), y, unpack(w), *forward_bf16(x, w))


def _chain(x, y, p, z, h1, h2):
    """Gradient of the mean BCE given the layer inputs x, h1 and the
    activations h2 and logits z of a forward pass."""
    y = np.asarray(y, dtype=np.float64)
    b = x.shape[0]
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / b
    g = {"w3": h2.T @ dz, "b3": np.array([dz.sum()])}
    d2 = np.outer(dz, p["w3"]) * (h2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (h1 > 0)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(axis=0)
    return pack(g)


def adam(w, m, v, g, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba): returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round float32 values to bf16 (nearest even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    bits = a32.view(np.uint32).astype(np.uint64)
    rb = ((bits + (((bits >> 16) & 1) + 0x7FFF)) >> 16).astype(np.uint32) << 16
    return rb.astype(np.uint32).view(np.float32).astype(np.float64)


def features(J, x, prev_sigma):
    """The four checkpoint features of every replica of x [n, r, d] and the
    new signs; prev_sigma [r][n] are the signs of the previous checkpoint."""
    x = np.asarray(x, dtype=np.float64)
    J = np.asarray(J, dtype=np.float64)
    n, r, _ = x.shape
    sig = oracle.readout(x)
    x1 = x[:, :, 0]
    s1 = (x1 * x1).sum(axis=0)
    sall = (x * x).sum(axis=(0, 2))
    quad = np.array([x1[:, i] @ J @ x1[:, i] for i in range(r)])
    rq = np.where(s1 > 0, -quad / (n * np.where(s1 > 0, s1, 1.0)), 0.0)
    eis = oracle.ising_energy(J, sig) / n
    share = np.where(sall > 0, s1 / np.where(sall > 0, sall, 1.0), 0.0)
    flips = (sig != prev_sigma).mean(axis=1)
    return np.stack([rq, eis, share, flips], axis=1), sig


def standardize(F, group):
    """Each column of F [groups * group][k] as (f - mean) / sd within each
    group of `group` consecutive rows (population sd; 0 where sd = 0)."""
    F = np.asarray(F, dtype=np.float64)
    out = np.empty_like(F)
    for g in range(F.shape[0] // group):
        blk = F[g * group:(g + 1) * group]
        mu = blk.mean(axis=0)
        sd = np.sqrt(((blk - mu) ** 2).mean(axis=0))
        out[g * group:(g + 1) * group] = np.where(sd > 0, (blk - mu) / np.where(sd > 0, sd, 1.0), 0.0)
    return out


def select_top(score, group, keep):
    """Global indices [groups][keep] of the keep highest scores of each group
    of consecutive scores, ascending; equal scores: lower index first; NaN
    lowest."""
    score = np.asarray(score, dtype=np.float64)
    out = []
    for g in range(score.shape[0] // group):
        s = score[g * group:(g + 1) * group]
        key = np.where(np.isnan(s), -np.inf, s)
        order = sorted(range(group), key=lambda i: (-key[i], i))  # highest first, then lowest index
        out.append(sorted(g * group + i for i in order[:keep]))
    return np.array(out, dtype=np.int64)
