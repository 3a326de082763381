"""CPU reference of the pair-scoring MLP -- test infrastructure only.

The network is the learned proposal's scorer (not part of the paper, which has
no MLP; its results are therefore "parity unpinned" against the paper and pinned
instead by finite differences on this reference).  Input x = [a XOR b, a AND b]
of two 4,096-bit signatures, layers 8192 -> 512 -> 256 -> 1 with ReLU, logit
output, BCE-with-logits loss with a positive-class weight, Adam.

With `bf16=True` the reference rounds the same values the GPU kernels round to
BF16 (weights W1 and W2, the layer-1 activations, the layer-2 and layer-1
input gradients) with round-to-nearest-even, and accumulates in float64;
with `bf16=False` everything is float64 (used for the finite-difference check).
"""
from __future__ import annotations

import numpy as np

SHAPES = (("W1", (512, 8192)), ("b1", (512,)), ("W2", (256, 512)), ("b2", (256,)),
          ("w3", (256,)), ("b3", (1,)))


def unflatten(flat):
    out, at = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[at:at + n], dtype=np.float64).reshape(shape)
        at += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round float32 values to bfloat16 (round to nearest even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def pair_inputs(sig, pairs):
    """x[m] = [bits of sig_a XOR sig_b, bits of sig_a AND sig_b] as float64 0/1."""
    sig = np.asarray(sig, dtype=np.uint64)
    pairs = np.asarray(pairs, dtype=np.uint64)
    a = sig[(pairs >> np.uint64(32)).astype(np.int64)]
    b = sig[(pairs & np.uint64(0xFFFFFFFF)).astype(np.int64)]

    def bits(words):
        by = words.view(np.uint8).reshape(len(words), -1)
        return np.unpackbits(by, axis=1, bitorder="little").astype(np.float64)

    return np.concatenate([bits(a ^ b), bits(a & b)], axis=1)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(p, X, bf16_on=True):
    W1, W2 = _r(p["W1"], bf16_on), _r(p["W2"], bf16_on)
    a1 = np.maximum(X @ W1.T + p["b1"], 0.0)
    a1s = _r(a1, bf16_on)
    a2 = np.maximum(a1s @ W2.T + p["b2"], 0.0)
    z = a2 @ p["w3"] + p["b3"][0]
    return {"a1": a1, "a1s": a1s, "a2": a2, "z": z, "W1": W1, "W2": W2}


def loss_and_grads(p, X, y, pos_weight, bf16_on=True):
    f = forward(p, X, bf16_on)
    z, M = f["z"], len(y)
    sp_pos = np.maximum(z, 0) + np.log1p(np.exp(-np.abs(z)))  # softplus(z) = -log(1 - s(z))
    sp_neg = sp_pos - z                                       # softplus(-z) = -log s(z)
    loss = float(np.mean(pos_weight * y * sp_neg + (1 - y) * sp_pos))
    s = 1.0 / (1.0 + np.exp(-z))
    dz = (s * (pos_weight * y + 1 - y) - pos_weight * y) / M
    g = {"w3": f["a2"].T @ dz, "b3": np.array([dz.sum()])}
    dh2 = np.outer(dz, p["w3"]) * (f["a2"] > 0)
    g["b2"] = dh2.sum(0)
    dh2s = _r(dh2, bf16_on)
    g["W2"] = dh2s.T @ f["a1s"]
    dh1 = (dh2s @ f["W2"]) * (f["a1s"] > 0)
    g["b1"] = dh1.sum(0)
    g["W1"] = _r(dh1, bf16_on).T @ X
    return loss, g, f


def adam(p_flat, g_flat, m1, m2, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns (params, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g_flat
    m2 = b2 * m2 + (1 - b2) * g_flat * g_flat
    c1, c2 = 1 - b1 ** step, 1 - b2 ** step
    return p_flat - lr * (m1 / c1) / (np.sqrt(m2 / c2) + eps), m1, m2
