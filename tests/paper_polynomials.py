"""The paper's exp / ln method of Sec. 3.3 written out in numpy from its
equations (eqs. exp_algorithm_1 - exp_algorithm_3, eq. ln_approx) with the
coefficients of Table tab:coefficients_approx_correction, for measuring its
accuracy against the C library: test helper, not product code."""
import json
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_exp_ln_coefficients.json")


def coefficients():
    with open(GOLD) as f:
        d = json.load(f)
    return np.array(d["a"]), np.array(d["b"])


def k_exp(yf, a):
    return np.polyval(a[::-1], yf)


def k_ln(m, b):
    return np.polyval(b[::-1], m)


def exp2(y, a):
    """2^y: the double with bits int64(2^52 (y - K_exp(y - floor y)) + 2^52 1023)."""
    y = np.asarray(y, dtype=np.float64)
    yf = y - np.floor(y)
    bits = (2.0 ** 52 * (y - k_exp(yf, a)) + 2.0 ** 52 * 1023.0).astype(np.int64)
    return bits.view(np.float64)


def log2(x, b):
    """log2 x = (p - bias) + K_ln(m) from the exponent and mantissa fields (normal x > 0)."""
    x = np.asarray(x, dtype=np.float64)
    bits = x.view(np.int64)
    e = ((bits >> 52) & 0x7FF) - 1023
    m = (bits & ((1 << 52) - 1)).astype(np.float64) / 2.0 ** 52
    return e + k_ln(m, b)


def error_bounds(n=400_001):
    """(max relative error of exp2 on [-60, 60], max absolute error of log2
    on [2^-80, 2^80]) of the method with the printed coefficients."""
    a, b = coefficients()
    y = np.linspace(-60.0, 60.0, n)
    e_exp = float(np.abs(exp2(y, a) / np.exp2(y) - 1.0).max())
    x = np.exp2(np.linspace(-80.0, 80.0, n))
    e_log = float(np.abs(log2(x, b) - np.log2(x)).max())
    return e_exp, e_log
