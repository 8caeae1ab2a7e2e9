"""Accuracy of the paper's exp / ln method (Sec. 3.3, Table
tab:coefficients_approx_correction) against the C library, on the CPU.  The
GPU float64 mode MSTRUCT_F64_PAPER implements the same method; its parity
bar against the oracle (tests/test_gpu_f64.py) is derived from these
bounds.  The table prints twelve coefficients of K_ln while the text speaks
of degree 10: the twelve (degree 11) reach 3e-8, the first eleven only
2.5e-3, so the table is taken as it is printed."""
import numpy as np

from paper_polynomials import coefficients, error_bounds, exp2, k_exp, k_ln, log2


def test_k_exp_fits_its_definition():
    a, _ = coefficients()
    y = np.linspace(0.0, 1.0, 100_001)[:-1]
    err = np.abs(k_exp(y, a) - (1.0 + y - np.exp2(y))).max()
    assert 1e-11 < err < 2e-10  # a least-squares fit of degree 7: ~1.6e-10
    assert len(a) == 8


def test_k_ln_fits_its_definition_with_all_printed_coefficients():
    _, b = coefficients()
    m = np.linspace(0.0, 1.0, 100_001)[:-1]
    err = np.abs(k_ln(m, b) - np.log2(1.0 + m)).max()
    assert 1e-9 < err < 3.1e-8
    # the text's "degree 10" (b_0 .. b_10) fits far worse
    assert np.abs(k_ln(m, b[:11]) - np.log2(1.0 + m)).max() > 1e-3


def test_bit_synthesis_exp2_and_log2():
    a, b = coefficients()
    # exact powers of two at integer arguments up to K_exp(0) = a_0 (1.2e-10 relative)
    y = np.arange(-50, 51, dtype=np.float64)
    assert np.abs(exp2(y, a) / np.exp2(y) - 1.0).max() < 2e-10
    x = np.exp2(y)
    assert np.abs(log2(x, b) - y).max() < 2e-10
    e_exp, e_log = error_bounds()
    assert e_exp < 2e-10 and e_log < 3.1e-8
    # 2^y 2^-y = 1 and log2 of a product: consistent to the bounds
    yy = np.linspace(-30, 30, 10001)
    assert np.abs(exp2(yy, a) * exp2(-yy, a) - 1.0).max() < 4 * e_exp
    xs = np.exp2(np.linspace(-20, 20, 1001))
    assert np.abs(log2(xs * 3.0, b) - log2(xs, b) - np.log2(3.0)).max() < 2.1 * e_log
