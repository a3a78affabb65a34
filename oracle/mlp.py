"""FP64 oracle of the learned refinement indicator (TEST INFRASTRUCTURE ONLY).

The indicator is not part of the paper; the paper's gradient-based criterion
(Sec. 3.3, eq. lohner-simple) provides its training labels and stays its
fallback.  Definitions (written in the design notes):

Features, 16 per block: with r0 = max over interior cells of |grad rho|/rho
and r1 = max |grad p|/p (undivided central differences, norm over axes),
  f0 = log(1 + r0), f1 = log(1 + r1), f2 = level / L_max,
  f(3+2k), f(4+2k) = log(1 + r0), log(1 + r1) of the face neighbour(s) across
  face k = -x, +x, -y, +y, -z, +z (maximum over a finer group), 0 if absent,
  f15 = 0.
Network: 16 -> 64 ReLU -> 64 ReLU -> 3 logits (classes -1, 0, +1).  With
emulate=True every matrix-product operand (inputs, activations, weights,
back-propagated errors) is rounded to BF16 (round to nearest even, via FP32)
as the GPU's MFMA operands are; products and sums are FP64 here (FP32 on the
GPU).  Biases stay unrounded.  Loss: class-weighted cross-entropy,
sum_s w_c(s) CE_s / sum_s w_c(s).  Adam (lr 1e-3, beta 0.9 / 0.999, eps 1e-8).
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 16, 64, 3
SIZES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NOUT)),
         ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(w):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(w[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(x):
    """Round to BF16 (nearest even) through FP32, returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, emulate):
    return bf16(x) if emulate else np.asarray(x, dtype=np.float64)


def init_weights(seed=0):
    """He-style uniform initialisation from the seeded generator."""
    import synth
    w = {}
    u = synth.uniform_pm1(seed, NPARAM)
    o = 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        scale = np.sqrt(6.0 / shape[0]) if name.startswith("W") else 0.0
        w[name] = (u[o:o + n] * scale).reshape(shape)
        o += n
    return pack(w)


def forward(w, X, emulate=True):
    p = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    z1 = _r(X, emulate) @ _r(p["W1"], emulate) + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = _r(h1, emulate) @ _r(p["W2"], emulate) + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = _r(h2, emulate) @ _r(p["W3"], emulate) + p["b3"]
    return dict(z1=z1, h1=h1, z2=z2, h2=h2, z3=z3)


def softmax(z):
    e = np.exp(z - z.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grad(w, X, labels, class_w, emulate=True):
    """Weighted mean cross-entropy and its gradient (flat, like w).  labels
    in {-1, 0, +1} are classes 0, 1, 2."""
    p = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    c = np.asarray(labels).astype(np.int64) + 1
    cw = np.asarray(class_w, dtype=np.float64)[c]
    norm = 1.0 / cw.sum()
    f = forward(w, X, emulate)
    P = softmax(f["z3"])
    loss = float(np.sum(cw * -np.log(P[np.arange(len(c)), c])) * norm)
    onehot = np.zeros_like(P)
    onehot[np.arange(len(c)), c] = 1.0
    dz3 = (P - onehot) * (cw * norm)[:, None]
    g = {}
    g["W3"] = _r(f["h2"], emulate).T @ _r(dz3, emulate)
    g["b3"] = dz3.sum(axis=0)
    dh2 = _r(dz3, emulate) @ _r(p["W3"], emulate).T
    dz2 = dh2 * (f["z2"] > 0)
    g["W2"] = _r(f["h1"], emulate).T @ _r(dz2, emulate)
    g["b2"] = dz2.sum(axis=0)
    dh1 = _r(dz2, emulate) @ _r(p["W2"], emulate).T
    dz1 = dh1 * (f["z1"] > 0)
    g["W1"] = _r(X, emulate).T @ _r(dz1, emulate)
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def features(forest, raw, lmax, ndim):
    """[nb][16] features from per-block raw maxima (see module docstring)."""
    nb = forest.nb
    lr = np.log1p(np.asarray(raw, dtype=np.float64))
    F = np.zeros((nb, 16))
    F[:, 0:2] = lr
    F[:, 2] = np.array([l for l, _ in forest.leaves], dtype=np.float64) / lmax
    for n in range(nb):
        for f in range(2 * ndim):
            kind = forest.face_neighbours(n, f)
            if kind[0] in ("srl", "coarse"):
                F[n, 3 + 2 * f:5 + 2 * f] = lr[kind[1]]
            elif kind[0] == "fine":
                F[n, 3 + 2 * f:5 + 2 * f] = np.max(lr[[q for q, _ in kind[1]]], axis=0)
    return F


def predict_flags(w, X, lohner=None, threshold=0.5, emulate=True):
    """argmax class as a flag in {-1, 0, +1}; where the largest softmax
    probability is below threshold (or no weights), the Lohner flag."""
    P = softmax(forward(w, X, emulate)["z3"])
    flags = P.argmax(axis=1) - 1
    if lohner is not None:
        low = P.max(axis=1) < threshold
        flags = np.where(low, lohner, flags)
    return flags.astype(np.int8), P
