"""Pins of the FP64 network reference: its gradient equals central finite
differences of its loss, closed-form special cases, bf16 rounding.  CPU only."""
import numpy as np
import pytest

import workload
from oracle import mlp_oracle as M


def _data(B=37, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (B, 6)) * [100, 100, 0.5, 0.3, 0.3, 0.3] + [600, 600, -13, 0.3, 0.4, 0.3]
    Y = rng.normal(0, 1e-6, (B, 3))
    mean = np.array([600, 600, -13, 0.3, 0.4, 0.3])
    scale = np.array([100, 100, 0.5, 0.3, 0.3, 0.3])
    osc = np.array([1e-6, 1e-6, 1e-6])
    return X, Y, mean, scale, osc


def test_gradient_matches_finite_differences():
    X, Y, mean, scale, osc = _data()
    p = workload.mlp_init_params(3).astype(np.float64)
    p[M.SLICES["b2"][0]:M.SLICES["b2"][1]] = 0.05  # keep ReLUs away from their kink
    loss, g = M.loss_and_grad(p, X, Y, mean, scale, osc, bf16_round=False)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(np.arange(a, b), min(12, b - a), replace=False)
                          for (a, b, _) in M.SLICES.values()])
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (M.loss_and_grad(pp, X, Y, mean, scale, osc, False)[0] -
              M.loss_and_grad(pm, X, Y, mean, scale, osc, False)[0]) / (2 * eps)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_closed_form_special_cases():
    X, Y, mean, scale, osc = _data(B=5)
    d = {k: np.zeros(s) for k, (_, _, s) in M.SLICES.items()}
    d["b3"] = np.array([0.25, -0.5, 1.0])
    y, _ = M.forward(M.pack(d), X, mean, scale, bf16_round=False)
    assert np.all(y == d["b3"])
    # a single path: y0 = w3 * relu(w2 * relu(w1 * x0n + b1) + b2) + b3
    d["W1"][0, 0] = 0.5; d["b1"][0] = 0.1; d["W2"][0, 0] = 2.0; d["b2"][0] = -0.05; d["W3"][0, 0] = 3.0
    y, _ = M.forward(M.pack(d), X, mean, scale, bf16_round=False)
    x0 = (X[:, 0] - mean[0]) / scale[0]
    want = 3.0 * np.maximum(2.0 * np.maximum(0.5 * x0 + 0.1, 0) - 0.05, 0) + 0.25
    assert np.allclose(y[:, 0], want, rtol=1e-15, atol=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 3.0e-5])
    r = M.bf16(vals)
    assert r[0] == 1.0 and r[4] == -2.5 and r[5] == 0.0
    # spacing at 1 is 2^-7; halfway cases round to the even neighbour
    assert M.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0            # tie -> even (1.0)
    assert M.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6  # tie -> even
    assert M.bf16(np.array([1.0 + 2 ** -7]))[0] == 1.0 + 2 ** -7      # representable
    assert np.all(np.abs(r - vals) <= np.abs(vals) * 2 ** -8 + 1e-45)
