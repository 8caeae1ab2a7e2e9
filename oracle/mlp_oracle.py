"""FP64 reference of the surrogate network (TEST INFRASTRUCTURE ONLY).

MLP 6 -> 64 -> 64 -> 3 with ReLU; parameter vector W1[64][6], b1[64],
W2[64][64], b2[64], W3[3][64], b3[3].  With ``bf16=True`` the values that the
device rounds to bfloat16 (round to nearest even) are rounded here too: the
normalised inputs, the three weight matrices, the first-layer bias (it rides
on a constant-one input), both hidden activations after ReLU, and in the
backward pass the output gradient and both hidden-layer gradients.  Products
are accumulated in float64.  Loss: 0.5/B sum ||f(x) - y/out_scale||^2.
"""
from __future__ import annotations

import numpy as np

N_PARAM = 4803
SLICES = {"W1": (0, 384, (64, 6)), "b1": (384, 448, (64,)), "W2": (448, 4544, (64, 64)),
          "b2": (4544, 4608, (64,)), "W3": (4608, 4800, (3, 64)), "b3": (4800, 4803, (3,))}


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return {k: p[a:b].reshape(s) for k, (a, b, s) in SLICES.items()}


def pack(d):
    out = np.zeros(N_PARAM)
    for k, (a, b, s) in SLICES.items():
        out[a:b] = np.asarray(d[k], dtype=np.float64).reshape(-1)
    return out


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def _id(x):
    return np.asarray(x, dtype=np.float64)


def forward(params, X, in_mean, in_scale, bf16_round=True):
    r = bf16 if bf16_round else _id
    P = unpack(params)
    x = r((np.asarray(X, np.float64) - np.asarray(in_mean, np.float64)) / np.asarray(in_scale, np.float64))
    a1 = x @ r(P["W1"]).T + r(P["b1"])
    h1 = r(np.maximum(a1, 0.0))
    a2 = h1 @ r(P["W2"]).T + P["b2"]
    h2 = r(np.maximum(a2, 0.0))
    y = h2 @ r(P["W3"]).T + P["b3"]
    return y, (x, h1, h2)


def predict(params, X, in_mean, in_scale, out_scale, bf16_round=True):
    """Changes (alpha_s, alpha_m, beta): network outputs times out_scale."""
    return forward(params, X, in_mean, in_scale, bf16_round)[0] * np.asarray(out_scale, np.float64)


def loss_and_grad(params, X, Y, in_mean, in_scale, out_scale, bf16_round=True):
    r = bf16 if bf16_round else _id
    P = unpack(params)
    B = X.shape[0]
    y, (x, h1, h2) = forward(params, X, in_mean, in_scale, bf16_round)
    res = y - np.asarray(Y, np.float64) / np.asarray(out_scale, np.float64)
    loss = 0.5 * np.sum(res * res) / B
    dy = r(res / B)
    dh2 = r((dy @ r(P["W3"])) * (h2 > 0))
    dh1 = r((dh2 @ r(P["W2"])) * (h1 > 0))
    g = {"W3": dy.T @ h2, "b3": dy.sum(0), "W2": dh2.T @ h1, "b2": dh2.sum(0),
         "W1": dh1.T @ x, "b1": dh1.sum(0)}
    return loss, pack(g)
