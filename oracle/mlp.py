"""Oracle for the learned start proposal's network (test infrastructure only).

Plain NumPy in float64: a multilayer perceptron 5 -> 64 -> 64 -> 2 with ReLU
hidden layers and a linear output, the mean-squared-error loss and its
gradient by backpropagation (textbook chain rule), Adam, and an emulation of
bfloat16 rounding (round to nearest even on the top 16 bits of a float32)
for checking a forward pass that feeds bfloat16 operands to matrix cores.

Parameter layout (shared with the library's C interface): one float32
vector, in order W1 (5 x 64, row-major: input-major), b1 (64), W2 (64 x 64),
b2 (64), W3 (64 x 2), b3 (2): 4,674 numbers.  A layer computes
h_out = act(h_in @ W + b).
"""
from __future__ import annotations

import numpy as np

SIZES = (5, 64, 64, 2)


def n_params(sizes=SIZES) -> int:
    return sum(sizes[i] * sizes[i + 1] + sizes[i + 1] for i in range(len(sizes) - 1))


def unpack(p: np.ndarray, sizes=SIZES):
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for i in range(len(sizes) - 1):
        a, b = sizes[i], sizes[i + 1]
        W = p[o:o + a * b].reshape(a, b)
        o += a * b
        bb = p[o:o + b]
        o += b
        out.append((W, bb))
    assert o == p.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, X, bf16_operands: bool = False):
    """Returns the output and the list of pre-activations / activations.
    With bf16_operands the inputs of every matrix product (activations and
    weights) are rounded to bfloat16 and the products accumulate in float64
    (the matrix cores accumulate in float32; the difference is far below the
    bfloat16 rounding)."""
    layers = unpack(p)
    h = np.asarray(X, dtype=np.float64)
    cache = [h]
    for i, (W, b) in enumerate(layers):
        hin, Win = (bf16(h), bf16(W)) if bf16_operands else (h, W)
        z = hin @ Win + b
        h = np.maximum(z, 0.0) if i < len(layers) - 1 else z
        cache.append(z)
        cache.append(h)
    return h, cache


def loss(p, X, Y) -> float:
    out, _ = forward(p, X)
    return float(np.mean(np.sum((out - Y) ** 2, axis=1)))


def grad(p, X, Y) -> np.ndarray:
    """Gradient of loss = mean over samples of |out - Y|^2."""
    layers = unpack(p)
    out, cache = forward(p, X)
    m = X.shape[0]
    delta = 2.0 * (out - Y) / m                      # dL/d(out)
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        h_in = cache[2 * i]
        gW = h_in.T @ delta
        gb = delta.sum(axis=0)
        grads.append((gW, gb))
        if i > 0:
            z_prev = cache[2 * i - 1]
            delta = (delta @ W.T) * (z_prev > 0.0)
    return pack(grads[::-1])


def adam(p, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def he_uniform(seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    layers = []
    for i in range(len(SIZES) - 1):
        a, b = SIZES[i], SIZES[i + 1]
        lim = np.sqrt(6.0 / a)
        layers.append((rng.uniform(-lim, lim, (a, b)), np.zeros(b)))
    return pack(layers).astype(np.float32)
