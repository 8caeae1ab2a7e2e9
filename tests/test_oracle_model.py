"""Pins of the FP64 oracle's phase model against what the paper and the
mathematics fix (constants, printed statements, closed forms, invariants,
limits, convergence).  CPU only."""
import json
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_constants_match_paper_tables(orc):
    want = _gold("paper_constants.json")
    got = orc.constants()
    for k, v in want.items():
        if k.startswith("_"):
            continue
        assert got[k] == v, k


def test_liquid_fraction_shape(orc):
    c = orc.constants()
    assert orc.liquid_fraction(c["T_s"] - 1e-9) == 0.0
    assert orc.liquid_fraction(c["T_l"] + 1e-9) == 1.0
    mid = 0.5 * (c["T_s"] + c["T_l"])
    assert orc.liquid_fraction(mid) == pytest.approx(0.5, abs=1e-15)
    Ts = np.linspace(1800, 2000, 401)
    g = np.array([orc.liquid_fraction(T) for T in Ts])
    assert np.all(np.diff(g) >= 0)


def test_alpha_equilibrium_shape(orc):
    c = orc.constants()
    # continuous at the alpha_s start temperature, flat 0.9 below the end temperature
    assert orc.alpha_eq(c["T_as_start"]) == pytest.approx(0.0, abs=1e-15)
    assert orc.alpha_eq(c["T_as_start"] + 1) == 0.0
    assert orc.alpha_eq(c["T_as_end"] - 1e-9) == 0.9
    Ts = np.linspace(900, 1300, 801)
    x = np.array([orc.alpha_eq(T) for T in Ts])
    assert np.all(np.diff(x) <= 0) and x.max() <= 0.9 and x.min() >= 0.0
    # the Koistinen-Marburger branch lies just below 0.9 at T_as_end (jump < 1e-3)
    assert 0.0 < 0.9 - orc.alpha_eq(c["T_as_end"]) < 1e-3


def test_martensite_pseudo_equilibrium_shape(orc):
    c = orc.constants()
    assert orc.am0_eq(c["T_am_start"]) == pytest.approx(0.0, abs=1e-15)
    assert orc.am0_eq(c["T_am_start"] + 1e-6) == 0.0
    # between the martensite start and the alpha_s start the value is zero (reading R1)
    for T in (900.0, 1000.0, 1200.0):
        assert orc.am0_eq(T) == 0.0
    st = _gold("paper_statements.json")["equilibria_sum_at_T_inf"]
    s = orc.alpha_eq(c["T_inf"]) + orc.am0_eq(c["T_inf"])
    assert abs(s - st["value"]) < st["tol"]


def test_rate_constant_logistic(orc):
    c = orc.constants()
    assert orc.k_as(c["k2"]) == pytest.approx(c["k1"] / 2, rel=1e-15)
    assert orc.k_as(1e5) == pytest.approx(c["k1"], rel=1e-12)
    assert orc.k_as(0.0) < 1e-10
    # k_beta = f * k_as enters the alpha_s -> beta rate linearly
    T = 1100.0
    xeq = orc.alpha_eq(T)
    r1, r2, r3 = orc.rates(0.9, 0.0, 0.2, T)
    pb, qb = 10 / 11, 12 / 11
    assert r3 == pytest.approx(c["f"] * orc.k_as(T) * 0.2 ** pb * (0.9 - xeq) ** qb, rel=1e-13)


def test_zero_rate_states(orc):
    st = _gold("paper_statements.json")
    s = st["zero_rate_state_beta_to_alpha"]
    for T in (950.0, 1000.0, 1200.0):
        r1, r2, r3 = orc.rates(s["alpha_s"], s["alpha_m"], 0.9, T)
        assert (r1, r2, r3) == (0.0, 0.0, 0.0)
    s = st["zero_rate_state_alpha_to_beta"]
    for T in (1000.0, 1200.0, 1260.0):
        r1, r2, r3 = orc.rates(s["alpha_s"], s["alpha_m"], 0.0, T)
        assert (r1, r2, r3) == (0.0, 0.0, 0.0)
    # the start-up forms move both states off zero within one step
    st_b = orc.State(np.array([1.0]), np.array([0.0]), np.array([0.0]))
    orc.step(st_b, 1000.0, 1000.0, 1e-3)
    assert st_b.alpha_s[0] > 0
    st_a = orc.State.initial(1)
    orc.step(st_a, 1200.0, 1200.0, 1e-3)
    assert st_a.xbt[0] > 0


def test_startup_closed_form_values(orc):
    d = _gold("derived_values.json")
    T = 1200.0
    D = 0.9 - orc.alpha_eq(T)
    kb = 3.8 * orc.k_as(T)
    assert orc.logistic_step(0.0, D, D * kb, 11.0, 10.0) == pytest.approx(
        d["startup_beta_1200K_10s"]["value"], rel=d["startup_beta_1200K_10s"]["rtol"])
    T = 1000.0
    D = orc.alpha_eq(T)
    for key, dt in (("startup_alpha_1000K_1us", 1e-6), ("startup_alpha_1000K_1ms", 1e-3),
                    ("startup_alpha_1000K_1s", 1.0)):
        assert orc.logistic_step(0.0, D, D * orc.k_as(T), 2.51, dt) == pytest.approx(
            d[key]["value"], rel=d[key]["rtol"])


@pytest.mark.parametrize("c", [2.51, 11.0])
def test_closed_form_semigroup(orc, c):
    # two half steps equal one full step at constant k~ (the substitution
    # u = (xi/(1-xi))^(1/c) makes u grow linearly in time)
    D, kt = 0.6, 0.8
    for X in (0.0, 1e-12, 1e-4, 0.1, 0.5):
        for dt in (1e-6, 1e-3, 1.0):
            one = orc.logistic_step(X, D, kt, c, dt)
            two = orc.logistic_step(orc.logistic_step(X, D, kt, c, dt / 2), D, kt, c, dt / 2)
            assert two == pytest.approx(one, rel=1e-9, abs=1e-300)


def test_closed_form_solves_the_rate_equation(orc):
    # derivative of the closed form in dt equals the generalised-logistic rate
    D, kt = 0.5, 0.7
    for c in (2.51, 11.0):
        for X in (1e-3, 0.1, 0.3):
            h = 1e-7
            d = (orc.logistic_step(X, D, kt, c, h) - X) / h
            xi = X / D
            rate = D * kt * xi ** ((c - 1) / c) * (1 - xi) ** ((c + 1) / c)
            assert d == pytest.approx(rate, rel=1e-5)


def _run_constant_T(orc, state, T, dt, n):
    for _ in range(n):
        orc.step(state, T, T, dt)
    return state


def test_explicit_converges_to_appendix_solution_alpha_to_beta(orc):
    # Appendix A verification set-up: T = 1200 K from alpha_s = 0.9, beta = 0.1;
    # the closed form is exact at constant T; the explicit scheme (start-up,
    # then Euler on eq. alpha_s_to_beta) must converge to it at first order.
    T, t_end = 1200.0, 10.0
    D = 0.9 - orc.alpha_eq(T)
    exact = orc.logistic_step(0.0, D, D * 3.8 * orc.k_as(T), 11.0, t_end)
    errs = []
    for dt in (4e-3, 2e-3, 1e-3):
        s = _run_constant_T(orc, orc.State.initial(1), T, dt, int(round(t_end / dt)))
        errs.append(abs(s.xbt[0] - exact) / exact)
        assert s.beta[0] == pytest.approx(0.1 + s.xbt[0], abs=1e-15)
    assert errs[-1] < 2e-2
    assert 1.6 < errs[0] / errs[1] < 2.5 and 1.6 < errs[1] / errs[2] < 2.5


def test_explicit_converges_to_startup_solution_beta_to_alpha(orc):
    # same for beta -> alpha_s from pure beta at constant T (reading R7): the
    # Euler steps on eq. beta_to_alpha_s after the first closed-form step
    T, t_end = 1000.0, 3.0
    D = orc.alpha_eq(T)
    exact = orc.logistic_step(0.0, D, D * orc.k_as(T), 2.51, t_end)
    errs = []
    for dt in (4e-3, 2e-3, 1e-3):
        st = orc.State(np.array([1.0]), np.array([0.0]), np.array([0.0]))
        s = _run_constant_T(orc, st, T, dt, int(round(t_end / dt)))
        errs.append(abs(s.alpha_s[0] - exact) / exact)
    assert errs[-1] < 1e-2
    assert 1.6 < errs[0] / errs[1] < 2.6 and 1.6 < errs[1] / errs[2] < 2.6


def test_long_time_equilibrium(orc):
    # at constant T in (T_as_end, T_as_start) pure beta relaxes to X_alpha^eq(T)
    for T in (1000.0, 1100.0):
        st = orc.State(np.array([1.0]), np.array([0.0]), np.array([0.0]))
        _run_constant_T(orc, st, T, 0.05, 20000)
        assert st.alpha_s[0] == pytest.approx(orc.alpha_eq(T), abs=1e-4)
        assert st.alpha_m[0] == 0.0


def test_quench_forms_martensite_from_beta(orc):
    c = orc.constants()
    # one explicit step from 1000 K to T_inf: g uses T^{n+1} (eq. explicit_correction)
    st = orc.State(np.array([1.0]), np.array([0.0]), np.array([0.0]))
    orc.step(st, 1000.0, c["T_inf"], 1e-6)
    want = _gold("paper_statements.json")["room_temperature_beta"]
    assert st.beta[0] == pytest.approx(want["value"], abs=want["tol"])
    assert st.alpha_m[0] + st.alpha_s[0] == pytest.approx(0.9, abs=1e-12)
    # partial stable alpha: martensite only forms from the remaining beta
    st = orc.State(np.array([0.5]), np.array([0.5]), np.array([0.0]))
    orc.step(st, 800.0, 300.0, 1e-6)
    assert 0 < st.alpha_m[0] and st.alpha_s[0] + st.alpha_m[0] <= 0.9
    assert st.alpha_m[0] == pytest.approx(orc.am0_eq(300.0) * (0.9 - st.alpha_s[0]) / 0.9, rel=1e-12)
    # martensite is not dissolved by re-heating below the start temperature (reading R4)
    m0 = st.alpha_m[0]
    orc.step(st, 300.0, 700.0, 1e-6)
    assert st.alpha_m[0] >= m0 - 1e-12


def test_heating_specials(orc):
    c = orc.constants()
    st0 = lambda: orc.State(np.array([0.1]), np.array([0.3]), np.array([0.6]))
    # above T_as_start no martensite remains
    s = st0(); orc.step(s, 1280.0, 1280.0, 1e-6)
    assert s.alpha_m[0] == 0.0
    # regularisation: linear cap 0.9 (1373 - T)/100
    s = orc.State(np.array([0.1]), np.array([0.9]), np.array([0.0]))
    orc.step(s, 1323.0, 1323.0, 1e-9)
    assert s.alpha_s[0] == pytest.approx(0.45, abs=1e-6)
    # at and above T_as_start + T_as_reg only beta remains
    s = st0(); orc.step(s, 1373.0, 1373.0, 1e-6)
    assert s.alpha_s[0] == 0.0 and s.alpha_m[0] == 0.0 and s.beta[0] == 1.0
    # mushy zone: beta = X_sol, liquid above T_l
    T = 1900.0
    s = st0(); orc.step(s, T, T, 1e-6)
    assert s.beta[0] == pytest.approx(1.0 - orc.liquid_fraction(T), abs=1e-15)
    s = st0(); orc.step(s, 2000.0, c["T_l"], 1e-6)
    assert (s.alpha_s[0], s.alpha_m[0], s.beta[0]) == (0.0, 0.0, 0.0)


def test_invariants_random_paths(orc):
    # phase sum equals X_sol(T^{n+1}), fractions in [0, 0.9], beta >= 0.1 when solid
    rng = np.random.default_rng(7)
    n = 4000
    a = rng.uniform(0, 0.9, n)
    m = rng.uniform(0, 1, n) * (0.9 - a)
    st = orc.State(1.0 - a - m, a, m)
    for it in range(200):
        Tn = rng.uniform(300, 2000, n) if it == 0 else T1
        T1 = np.clip(Tn + rng.normal(0, 150, n), 300, 2100)
        dt = float(10 ** rng.uniform(-7, -2))
        orc.step(st, Tn, T1, dt)
        xsol = 1.0 - np.array([orc.liquid_fraction(t) for t in T1])
        assert np.all(st.alpha_s >= 0) and np.all(st.alpha_m >= 0)
        assert np.all(st.alpha_s + st.alpha_m <= 0.9 + 1e-15)
        assert np.allclose(st.alpha_s + st.alpha_m + st.beta, xsol, atol=2e-16, rtol=0)
        solid = T1 < 1878.0
        assert np.all(st.beta[solid] >= 0.1 - 1e-15)
        assert np.all(st.beta <= 1.0) and np.all(st.beta >= 0.0)


def test_first_order_in_time_on_smooth_history(orc):
    # brute force on a tiny set: smooth temperature histories inside the
    # diffusive range (no start-up switch, whose exit test depends on dt) at dt
    # and at a 1000x finer dt; differences shrink linearly in dt
    def T_of(t, ph):
        return 1100.0 + 120.0 * np.sin(30.0 * t + ph)

    a0 = np.array([0.2, 0.5, 0.05, 0.3])
    m0 = np.array([0.3, 0.1, 0.2, 0.0])

    def run(dt):
        n = int(round(0.2 / dt))
        t = np.arange(n + 1) * dt
        st = orc.State(1.0 - a0 - m0, a0, m0)
        orc.history_run(st, np.stack([T_of(t, ph) for ph in (0.0, 1.0, 2.0, 3.0)]), dt)
        return np.concatenate([st.alpha_s, st.alpha_m])

    ref = run(1e-6)
    e = [np.abs(run(dt) - ref).max() for dt in (4e-3, 2e-3, 1e-3)]
    assert e[0] > 1e-6
    assert 1.7 < e[0] / e[1] < 2.3 and 1.7 < e[1] / e[2] < 2.3


def test_alpha_s_to_beta_start_converges_through_the_exit(orc):
    """At constant 1100 K, 10 s from X~beta = 0: the start-up closed form
    runs until X~beta dt > 1e-15, then Euler.  X~beta grows monotonically
    across the switch and its error against the Appendix A closed form over
    the whole hold is first order in dt.  Accumulating alpha_s from the
    start-up increments (near 1e-15 each, rounded at 1.1e-16 in float64)
    instead of setting it from X~beta breaks both."""
    c = orc.constants()
    T = 1100.0
    D = 0.9 - orc.alpha_eq(T)
    exact = orc.logistic_step(0.0, D, c["f"] * orc.k_as(T) * D, c["c_beta"], 10.0)
    errs = []
    for dt in (4e-3, 2e-3, 1e-3):
        st = orc.State.initial(1)
        prev = 0.0
        for _ in range(int(round(10.0 / dt))):
            orc.step(st, T, T, dt)
            assert st.xbt[0] >= prev
            prev = st.xbt[0]
        errs.append(abs(st.xbt[0] - exact) / exact)
    assert errs[-1] < 1e-2
    assert all(1.8 < errs[i] / errs[i + 1] < 2.4 for i in range(2)), errs


# ---- eq. alpha_m_to_alpha_s (tempering of martensite into stable alpha) ----
# At constant T below the alpha_s -> beta end temperature (935 K) the
# equilibrium is X_alpha^eq = 0.9; a state with X_as + X_am = 0.9 then has
# neither beta -> alpha_s nor alpha_s -> beta, and the formation law cannot
# raise alpha_m (X_am,0^eq < 1).  Only the tempering rate acts, and it keeps
# X_as + X_am = 0.9, so X_as' = k_as X_as^p (0.9 - X_as)^q: with xi = X_as/0.9
# this is the Appendix A equation with D = 0.9, k~ = 0.9 k_as(T), c = c_as,
# whose closed form is exact.  A debit of alpha_s instead of a credit, k_beta
# in place of k_as, or swapped exponents all leave this solution.

def _tempering_run(orc, step, T, a0, m0, dt, t_end):
    st = orc.State(np.array([1.0 - a0 - m0]), np.array([a0]), np.array([m0]))
    for _ in range(int(round(t_end / dt))):
        step(st, T, T, dt)
    return st


@pytest.mark.parametrize("key,T,t_end,dts", [
    ("tempering_900K_2s", 900.0, 2.0, (4e-3, 2e-3, 1e-3)),
    ("tempering_700K_20s", 700.0, 20.0, (4e-2, 2e-2, 1e-2)),
])
def test_alpha_m_to_alpha_s_explicit_converges_to_closed_form(orc, key, T, t_end, dts):
    want = _gold("derived_values.json")[key]
    c = orc.constants()
    # the oracle's own closed form agrees with the hand-derived value
    assert orc.logistic_step(0.3, 0.9, 0.9 * orc.k_as(T), c["c_as"], t_end) == pytest.approx(
        want["value"], rel=want["rtol"])
    errs = []
    for dt in dts:
        st = _tempering_run(orc, orc.step, T, 0.3, 0.6, dt, t_end)
        # the transformation conserves the alpha total and leaves beta at 0.1
        assert st.alpha_s[0] + st.alpha_m[0] == pytest.approx(0.9, abs=1e-14)
        assert st.beta[0] == pytest.approx(0.1, abs=1e-14)
        errs.append(abs(st.alpha_s[0] - want["value"]))
    # the hold moves alpha_s by > 0.005; the explicit error is first order
    assert abs(want["value"] - 0.3) > 5e-3
    assert errs[-1] < 1e-4 * (t_end / 2.0)
    assert all(1.8 < errs[i] / errs[i + 1] < 2.2 for i in range(2)), errs


def test_alpha_m_to_alpha_s_rate_value(orc):
    # r2 = k_as X_as^p X_am^q with p = (c-1)/c, q = (c+1)/c, c = c_as; the
    # other two rates vanish at X_alpha = X_alpha^eq = 0.9 (up to the rounding
    # of 0.3 + 0.6 in float64)
    T, a, m = 900.0, 0.3, 0.6
    r1, r2, r3 = orc.rates(a, m, 0.0, T)
    kas = 0.294 / (1.0 + math.exp(-0.0337 * (T - 850.0)))
    p, q = (2.51 - 1) / 2.51, (2.51 + 1) / 2.51
    assert r1 < 1e-20 and r3 == 0.0
    assert r2 == pytest.approx(kas * a ** p * m ** q, rel=1e-13)
    # one small explicit step credits alpha_s with exactly what it takes from alpha_m
    st = orc.State(np.array([0.1]), np.array([a]), np.array([m]))
    orc.step(st, T, T, 1e-6)
    assert st.alpha_s[0] - a == pytest.approx(1e-6 * r2, rel=1e-9)
    assert m - st.alpha_m[0] == pytest.approx(1e-6 * r2, rel=1e-9)
