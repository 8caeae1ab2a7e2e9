"""Pins of the oracle's two switchable readings of the paper against values
its formulas fix.  CPU only.

- A3, the temperature of the explicit correction g: T^{n+1} as eq.
  explicit_correction writes it (default), or the T^n that Algorithm 2
  passes.  With T^n, g acts one step late: a quench forms its martensite in
  the step after the one that reaches the cold temperature.
- A4, the martensite formation law (eq. inst_martensite_formation, with the
  pseudo-equilibrium of eqs. equilibrium_phase_am0 / equilibrium_phase_am):
  "max" never lowers alpha_m (default); the literal "=" sets alpha_m to
  X_am,0^eq(T) (0.9 - X_as) / 0.9 below the martensite start, which lowers
  it on reheating.

The implicit scheme corrects at T^{n+1} by eq. implicit_correction in either
reading of A3."""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _one(orc, b, a, m):
    return orc.State(np.array([b]), np.array([a]), np.array([m]))


def test_readings_default_and_reset(orc):
    assert orc.lib().orc_get_readings() == 0
    with orc.readings(correction_T="prev", martensite="assign"):
        assert orc.lib().orc_get_readings() == 3
    assert orc.lib().orc_get_readings() == 0


def test_assign_lowers_martensite_on_reheating(orc):
    """X_as = 0 (the tempering rate carries X_as^p, so it vanishes) and
    X_am = 0.6 held at 700 K: "=" sets X_am to X_am,0^eq(700) = 0.458926,
    "max" keeps 0.6."""
    want = _gold("derived_values.json")["am0_eq_700K"]
    with orc.readings(martensite="assign"):
        st = _one(orc, 0.4, 0.0, 0.6)
        orc.step(st, 700.0, 700.0, 1e-6)
        assert st.alpha_s[0] < 1e-20  # only the closed-form start of beta -> alpha_s acts
        assert st.alpha_m[0] == pytest.approx(want["value"], rel=want["rtol"])
        assert st.beta[0] == pytest.approx(1.0 - want["value"], rel=1e-12)
        # the implicit scheme takes the same correction
        st = _one(orc, 0.4, 0.0, 0.6)
        orc.step_implicit(st, 700.0, 700.0, 1e-3)
        assert st.alpha_m[0] == pytest.approx(want["value"], rel=1e-9)
    st = _one(orc, 0.4, 0.0, 0.6)
    orc.step(st, 700.0, 700.0, 1e-6)
    assert st.alpha_m[0] == 0.6


def test_assign_and_max_agree_where_martensite_forms(orc):
    """Below the pseudo-equilibrium both readings raise X_am to
    X_am,0^eq(T) (0.9 - X_as) / 0.9, bit for bit."""
    out = []
    for mode in ("max", "assign"):
        with orc.readings(martensite=mode):
            st = _one(orc, 0.45, 0.45, 0.1)
            orc.step(st, 700.0, 700.0, 1e-6)
            out.append((st.alpha_s[0], st.alpha_m[0], st.beta[0]))
    assert out[0] == out[1]
    a = out[0][0]
    assert out[0][1] == pytest.approx(orc.am0_eq(700.0) * (0.9 - a) / 0.9, rel=1e-12)
    assert out[0][1] == pytest.approx(0.5 * _gold("derived_values.json")["am0_eq_700K"]["value"], rel=1e-8)


def test_prev_correction_lags_a_quench_by_one_step(orc):
    """Pure beta, 1400 K -> 300 K in one step: with g at T^{n+1} the step
    forms X_am,0^eq(300) = 0.897121; with g at T^n (1400 K, above the
    martensite start) nothing forms until the next step at 300 K."""
    want = _gold("derived_values.json")["am0_eq_300K"]
    st = _one(orc, 1.0, 0.0, 0.0)
    orc.step(st, 1400.0, 300.0, 1e-6)
    assert st.alpha_m[0] == pytest.approx(want["value"], rel=want["rtol"])
    with orc.readings(correction_T="prev"):
        st = _one(orc, 1.0, 0.0, 0.0)
        orc.step(st, 1400.0, 300.0, 1e-6)
        assert st.alpha_m[0] == 0.0 and st.beta[0] == 1.0
        orc.step(st, 300.0, 300.0, 1e-6)
        assert st.alpha_m[0] == pytest.approx(want["value"], rel=1e-9)


def test_prev_correction_lags_heating(orc):
    """Stable alpha heated 300 K -> 1400 K in one step: g at T^{n+1} leaves
    only beta (above T_as_start + T_reg = 1373 K); g at T^n = 300 K leaves
    the state, and the next step at 1400 K dissolves it."""
    st = _one(orc, 0.1, 0.9, 0.0)
    orc.step(st, 300.0, 1400.0, 1e-6)
    assert st.alpha_s[0] == 0.0 and st.beta[0] == 1.0
    with orc.readings(correction_T="prev"):
        st = _one(orc, 0.1, 0.9, 0.0)
        orc.step(st, 300.0, 1400.0, 1e-6)
        assert st.alpha_s[0] == 0.9 and st.beta[0] == pytest.approx(0.1, abs=1e-15)
        orc.step(st, 1400.0, 1400.0, 1e-6)
        assert st.alpha_s[0] == 0.0 and st.beta[0] == 1.0


def test_correction_T_leaves_the_implicit_scheme(orc):
    rng = np.random.default_rng(5)
    n = 500
    a = rng.uniform(0, 0.9, n)
    m = rng.uniform(0, 1, n) * (0.9 - a)
    Tn = rng.uniform(300, 1500, n)
    Tn1 = Tn + rng.uniform(-200, 200, n)
    out = []
    for mode in ("next", "prev"):
        with orc.readings(correction_T=mode):
            st = orc.State(1.0 - a - m, a, m)
            orc.step_implicit(st, Tn, Tn1, 1e-3)
            out.append((st.alpha_s.copy(), st.alpha_m.copy(), st.beta.copy()))
    for x, y in zip(*out):
        assert np.array_equal(x, y)
    # while the explicit scheme differs where g acts
    out = []
    for mode in ("next", "prev"):
        with orc.readings(correction_T=mode):
            st = orc.State(1.0 - a - m, a, m)
            orc.step(st, Tn, Tn1, 1e-3)
            out.append(st.alpha_m.copy())
    assert not np.array_equal(out[0], out[1])
