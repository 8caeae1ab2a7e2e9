"""Pins of the oracle's analytic temperature (moving point source on a
semi-infinite body) against direct quadrature of the instantaneous-source
integral, its Rosenthal limit and special cases.  CPU only."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import workload

K, ALPHA, Q, V = 7.0, 3e-6, 70.0, 1.0
RHOC = K / ALPHA


def quad_T(x, y, z, tau_lo, tau_hi, P0=(0.0, 0.0, 0.0), u=(1.0, 0.0), t_on=0.0, t=None):
    """Temperature rise at (x, y, z) from the source that was on during source
    ages [tau_lo, tau_hi] before time t (numerical quadrature, image factor 2)."""
    def f(s):  # s = age of the heat pulse
        ts = t - s - t_on
        xs, ys = P0[0] + V * ts * u[0], P0[1] + V * ts * u[1]
        r2 = (x - xs) ** 2 + (y - ys) ** 2 + (z - P0[2]) ** 2
        return 2 * Q / RHOC * (4 * math.pi * ALPHA * s) ** -1.5 * math.exp(-r2 / (4 * ALPHA * s))
    pts = None
    return integrate.quad(f, tau_lo, tau_hi, limit=500, epsabs=0, epsrel=1e-11, points=pts)[0]


def test_erfcx_matches_library(orc):
    for y in np.concatenate([np.linspace(0, 30, 301), [24.999, 25.0, 25.001, 60.0, 1e3]]):
        assert orc.erfcx(y) == pytest.approx(special.erfcx(y), rel=2e-14)


def test_source_matches_quadrature_golden(orc):
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "derived_values.json")))
    tr = np.array([0, 0, 0, 1, 0, 0, 1.0, Q, V])
    for xi, rho, tau, want in d["temperature_quadrature"]["cases"]:
        F = orc.source_F(tr, tau, K, ALPHA, (V * tau + xi, rho, 0.0))
        assert F == pytest.approx(want, rel=d["temperature_quadrature"]["rtol"])


def test_source_matches_quadrature_random(orc):
    rng = np.random.default_rng(3)
    ux, uy = math.cos(0.7), math.sin(0.7)
    tr = np.array([1e-4, -2e-4, 0.0, ux, uy, 0.0, 1.0, Q, V])
    for _ in range(25):
        tau = 10 ** rng.uniform(-5, -2)
        p = np.array([1e-4, -2e-4, 0.0]) + rng.normal(0, 4e-4, 3)
        p[2] = -abs(p[2])
        F = orc.source_F(tr, tau, K, ALPHA, p)
        ref = quad_T(*p, 0.0, tau, P0=tr[:3], u=(ux, uy), t=tau)
        assert F == pytest.approx(ref, rel=1e-8, abs=1e-12)


def test_rosenthal_limit(orc):
    tr = np.array([0, 0, 0, 1, 0, 0, 10.0, Q, V])
    for xi, rho in ((-1e-4, 2e-5), (5e-5, 3e-5), (-3e-4, 1e-4)):
        tau = 0.5
        R = math.hypot(xi, rho)
        ros = Q / (2 * math.pi * K * R) * math.exp(-V * (xi + R) / (2 * ALPHA))
        F = orc.source_F(tr, tau, K, ALPHA, (V * tau + xi, rho, 0.0))
        assert F == pytest.approx(ros, rel=1e-6)


def test_track_start_is_not_quasi_steady(orc):
    # 200 us after switch-on, 200 um behind the start point the transient
    # solution is cold whereas Rosenthal's quasi-steady field is not
    tr = np.array([0, 0, 0, 1, 0, 0, 1.0, Q, V])
    tau = 200e-6
    x = -200e-6
    F = orc.source_F(tr, tau, K, ALPHA, (x, 0.0, 0.0))
    R = V * tau - x
    ros = Q / (2 * math.pi * K * R) * math.exp(-V * (-R + R) / (2 * ALPHA))
    assert F < 1e-3 and ros > 3000


def _scan(rows, window=2):
    return workload.Scan(np.array(rows, dtype=np.float64), K, ALPHA, 300.0, 1928.0, window)


def test_switched_off_track_matches_quadrature(orc):
    dur = 300e-6
    sc = _scan([[0, 0, 0, 1, 0, 0.0, dur, Q, V]], window=1)
    for t, p in ((500e-6, (250e-6, 40e-6, -20e-6)), (2e-3, (100e-6, 0.0, -50e-6)),
                 (350e-6, (320e-6, 30e-6, 0.0)), (900e-6, (150e-6, 60e-6, -40e-6))):
        T = orc.temperature(sc, np.array(p), t)[0]
        ref = min(1928.0, 300.0 + quad_T(*p, t - dur, t, t=t))
        assert T == pytest.approx(ref, rel=1e-9)


def test_switched_off_track_is_smooth_at_its_virtual_position(orc):
    # after switch-off the closed form is a difference of two sources with a
    # common (virtual) current position; the field there is finite, matches
    # the quadrature of the pulses actually emitted, and is not clamped
    dur = 300e-6
    sc = _scan([[0, 0, 0, 1, 0, 0.0, dur, Q, V]], window=1)
    for t in (330e-6, 340e-6, 350e-6, 400e-6):
        p = (V * t, 0.0, 0.0)
        T = orc.temperature(sc, np.array(p), t)[0]
        ref = 300.0 + quad_T(*p, t - dur, t, t=t)
        assert 300.0 < T < 1928.0
        assert T - 300.0 == pytest.approx(ref - 300.0, rel=2e-3), (t, T, ref)


def test_window_superposition_and_clamp(orc):
    rows = [[0, 0, 0, 1, 0, 0.0, 200e-6, Q, V],
            [2e-4, 1e-4, 0, -1, 0, 200e-6, 200e-6, Q, V],
            [0, 2e-4, 0, 1, 0, 400e-6, 200e-6, Q, V]]
    p = np.array([[0.0, 1e-4, -5e-5]])
    t = 500e-6
    single = [orc.temperature(_scan([r], 1), p, t)[0] - 300.0 for r in rows]
    assert min(single) > 0.01 and 300.0 + sum(single) < 1928.0
    T2 = orc.temperature(_scan(rows, 2), p, t)[0]
    T3 = orc.temperature(_scan(rows, 3), p, t)[0]
    assert T2 == pytest.approx(300.0 + single[1] + single[2], rel=1e-12)
    assert T3 == pytest.approx(300.0 + sum(single), rel=1e-12)
    # before the first switch-on only the far field remains
    assert orc.temperature(_scan(rows, 2), p, 0.0)[0] == 300.0
    # right at the source the clamp applies; everywhere T <= T_clamp
    assert orc.temperature(_scan(rows, 2), np.array([[V * 100e-6, 1e-4, 0.0]]), 300e-6)[0] == 1928.0
    g = np.stack(np.meshgrid(np.linspace(0, 3e-4, 13), np.linspace(0, 3e-4, 13), [0.0, -1e-5]), -1).reshape(-1, 3)
    assert np.all(orc.temperature(_scan(rows, 3), g, 450e-6) <= 1928.0)


def test_workload_tables_are_ordered_and_in_range():
    for wl in (workload.single_track(), workload.multilayer_block(),
               workload.island_scan(128, 96, 32, 3, 20e-6, 500, 2e-6, 11)):
        tr = wl.scan.tracks
        assert tr.shape[1] == workload.N_TRACK_COLS
        assert np.all(np.diff(tr[:, 5]) > 0)
        assert np.all(tr[:, 6] > 0)
        assert np.allclose(np.hypot(tr[:, 3], tr[:, 4]), 1.0)
        # every track ends before the next starts (one laser)
        assert np.all(tr[:-1, 5] + tr[:-1, 6] <= tr[1:, 5] + 1e-15)
