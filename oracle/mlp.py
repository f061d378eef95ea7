"""CPU oracle of the surrogate fitness model (not part of the paper's method).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

A 3-layer MLP over learned column embeddings, in float64:

    x    = [ (1/L) sum_t E[c_t] + Z[L] ;
             (1/(L-1)) sum_{t<L-1} F[c_t] * T[c_{t+1}]  (0 when L = 1) ]
    z1   = W1 r(x) + b1,   h1 = relu(z1)
    z2   = W2 r(h1) + b2,  h2 = relu(z2)
    y    = w3 . r(h2) + b3
    loss = mean (y - t)^2

``r`` rounds to bfloat16 (round to nearest even) when ``bf16=True``, the
precision the GPU feeds its matrix units; the backward pass rounds the
propagated gradients at the same points (dz2 before dW2 and dh1, dz1 before
dW1 and dx) and treats every rounding as the identity (straight-through).
With ``bf16=False`` the model is a plain float64 MLP, which the tests pin
against central finite differences.

Z [M+1][D] is a learned embedding of the series length L.  Parameters are
one flat vector: E, F, T [M][D] each, Z [M+1][D], W1 [H][2D], b1 [H],
W2 [H][H], b2 [H], w3 [H], b3 [1].
"""
from __future__ import annotations

import numpy as np


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32.  NaN stays NaN."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


def split(params, M, D, H):
    p = np.asarray(params, dtype=np.float64)
    i = 0
    out = {}
    for name, shape in (("E", (M, D)), ("F", (M, D)), ("T", (M, D)), ("Z", (M + 1, D)),
                        ("W1", (H, 2 * D)),
                        ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))):
        n = int(np.prod(shape))
        out[name] = p[i:i + n].reshape(shape)
        i += n
    assert i == p.size
    return out


def n_params(M, D, H):
    return 3 * M * D + (M + 1) * D + H * 2 * D + H + H * H + H + H + 1


def _r(x, on):
    if not on:
        return np.asarray(x, dtype=np.float64)
    return bf16_round(np.asarray(x, dtype=np.float32)).astype(np.float64)


def forward(params, offsets, cols, M, D, H, bf16=True):
    P = split(params, M, D, H)
    offsets = np.asarray(offsets)
    B = len(offsets) - 1
    x = np.zeros((B, 2 * D))
    for b in range(B):
        s = cols[offsets[b]:offsets[b + 1]]
        x[b, :D] = P["E"][s].sum(axis=0) / len(s) + P["Z"][len(s)]
        if len(s) > 1:
            x[b, D:] = (P["F"][s[:-1]] * P["T"][s[1:]]).sum(axis=0) / (len(s) - 1)
    xr = _r(x, bf16)
    W1, W2, w3 = _r(P["W1"], bf16), _r(P["W2"], bf16), _r(P["w3"], bf16)
    z1 = xr @ W1.T + P["b1"]
    h1r = _r(np.maximum(z1, 0.0), bf16)
    z2 = h1r @ W2.T + P["b2"]
    h2r = _r(np.maximum(z2, 0.0), bf16)
    y = h2r @ w3 + P["b3"][0]
    return y, dict(x=x, xr=xr, z1=z1, h1r=h1r, z2=z2, h2r=h2r, W1=W1, W2=W2, w3=w3, P=P)


def loss_and_grad(params, offsets, cols, target, M, D, H, bf16=True):
    offsets = np.asarray(offsets)
    cols = np.asarray(cols)
    B = len(offsets) - 1
    y, c = forward(params, offsets, cols, M, D, H, bf16)
    t = np.asarray(target, dtype=np.float64)
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / B
    g_w3 = c["h2r"].T @ dy
    g_b3 = np.array([dy.sum()])
    dz2 = np.outer(dy, c["w3"]) * (c["z2"] > 0)
    g_b2 = dz2.sum(axis=0)
    dz2r = _r(dz2, bf16)
    g_W2 = dz2r.T @ c["h1r"]
    dz1 = (dz2r @ c["W2"]) * (c["z1"] > 0)
    g_b1 = dz1.sum(axis=0)
    dz1r = _r(dz1, bf16)
    g_W1 = dz1r.T @ c["xr"]
    dx = dz1r @ c["W1"]
    P = c["P"]
    g_E, g_F, g_T = np.zeros((M, D)), np.zeros((M, D)), np.zeros((M, D))
    g_Z = np.zeros((M + 1, D))
    for b in range(B):
        s = cols[offsets[b]:offsets[b + 1]]
        np.add.at(g_E, s, dx[b, :D] / len(s))
        g_Z[len(s)] += dx[b, :D]
        if len(s) > 1:
            np.add.at(g_F, s[:-1], dx[b, D:] * P["T"][s[1:]] / (len(s) - 1))
            np.add.at(g_T, s[1:], dx[b, D:] * P["F"][s[:-1]] / (len(s) - 1))
    grad = np.concatenate([g_E.ravel(), g_F.ravel(), g_T.ravel(), g_Z.ravel(), g_W1.ravel(), g_b1,
                           g_W2.ravel(), g_b2, g_w3, g_b3])
    return loss, grad, y


def adam_step(params, grad, m1, m2, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m1, m2)."""
    m1 = beta1 * m1 + (1 - beta1) * grad
    m2 = beta2 * m2 + (1 - beta2) * grad * grad
    c1 = 1 - beta1 ** step
    c2 = 1 - beta2 ** step
    return params - lr * (m1 / c1) / (np.sqrt(m2 / c2) + eps), m1, m2
