"""Pins of the oracle's implicit scheme (Crank-Nicolson on the diffusive term,
correction g at T^{n+1}, fixed-point iteration with the WRMS stop, subcycling;
Sec. 3.1).  The scheme's definition is pinned by its order of convergence
against the Appendix A closed forms and against a Richardson-extrapolated
fine explicit integration: second order only holds if both rate evaluations
enter with weight dt/2 at their own temperature.  CPU only."""
import math

import numpy as np
import pytest

TIGHT = dict(eps_abs=1e-30, eps_rel=1e-15, max_iter=200, dt_sub=1e9)


def _run_cn(orc, a, m, T_of_t, t_end, h, **kw):
    n = int(round(t_end / h))
    st = orc.State(np.array([1.0 - a - m]), np.array([a]), np.array([m]))
    for s in range(n):
        bad, _ = orc.step_implicit(st, T_of_t(s * h), T_of_t((s + 1) * h), h, **kw)
        assert bad == 0
    return st


def _order(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_second_order_beta_to_alpha_s_at_constant_T(orc):
    # X_as' = k X^p (X_eq - X)^q with X_am = 0 at 1000 K: Appendix A form with
    # D = X_eq, k~ = k_as D, c = c_as is exact
    T, a0, t_end = 1000.0, 0.2, 2.0
    c = orc.constants()
    D = orc.alpha_eq(T)
    exact = orc.logistic_step(a0, D, orc.k_as(T) * D, c["c_as"], t_end)
    errs = []
    for h in (0.04, 0.02, 0.01):
        st = _run_cn(orc, a0, 0.0, lambda t: T, t_end, h, **TIGHT)
        errs.append(abs(st.alpha_s[0] - exact))
    order = _order(errs)
    assert all(1.85 < o < 2.15 for o in order), (errs, order)
    # the explicit scheme on the same problem is first order
    e_exp = []
    for h in (0.04, 0.02):
        st = orc.State(np.array([1 - a0]), np.array([a0]), np.array([0.0]))
        for _ in range(int(round(t_end / h))):
            orc.step(st, T, T, h)
        e_exp.append(abs(st.alpha_s[0] - exact))
    assert 0.8 < _order(e_exp)[0] < 1.2
    assert errs[0] < e_exp[0] / 5


def test_second_order_alpha_s_to_beta_at_constant_T(orc):
    # X~beta' = k_b X~b^p (D - X~b)^q with D = 0.9 - X_eq at 1200 K
    T, a0, t_end = 1200.0, 0.7, 1.0
    c = orc.constants()
    D = 0.9 - orc.alpha_eq(T)
    kb = c["f"] * orc.k_as(T)
    exact_bt = orc.logistic_step(0.9 - a0, D, kb * D, c["c_beta"], t_end)
    errs = []
    for h in (0.02, 0.01, 0.005):
        st = _run_cn(orc, a0, 0.0, lambda t: T, t_end, h, **TIGHT)
        errs.append(abs((0.9 - st.alpha_s[0]) - exact_bt))
    order = _order(errs)
    assert all(1.8 < o < 2.2 for o in order), (errs, order)


def test_second_order_with_varying_temperature(orc):
    # T rising linearly 1000 -> 1100 K over 1 s; reference: explicit steps of
    # 1e-5 and 2e-5 s Richardson-extrapolated (second order, error ~1e-10)
    a0, t_end = 0.3, 1.0
    T_of_t = lambda t: 1000.0 + 100.0 * t / t_end

    def explicit(h):
        n = int(round(t_end / h))
        hist = T_of_t(np.arange(n + 1) * h)[None, :]
        st = orc.State(np.array([1 - a0]), np.array([a0]), np.array([0.0]))
        orc.history_run(st, hist, h)
        return st.alpha_s[0]

    ref = 2 * explicit(1e-5) - explicit(2e-5)
    errs = []
    for h in (0.05, 0.025, 0.0125):
        st = _run_cn(orc, a0, 0.0, T_of_t, t_end, h, **TIGHT)
        errs.append(abs(st.alpha_s[0] - ref))
    order = _order(errs)
    assert all(1.8 < o < 2.2 for o in order), (errs, order)


def test_paper_tolerances_stay_close_to_the_converged_scheme(orc):
    # the WRMS stop (eps_abs 1e-10, eps_rel 1e-3, mean over N = 2 components)
    # accepts an iterate whose residual is below sqrt(2) (eps_abs + eps_rel |a|)
    # per component; with the fast contraction at these step sizes the
    # distance to the converged scheme stays within twice that
    rng = np.random.default_rng(3)
    n = 400
    am = rng.uniform(0, 0.5, n)
    a = rng.uniform(0.01, 1, n) * (0.9 - am)
    T0 = rng.uniform(900, 1250, n)
    T1 = T0 + rng.normal(0, 20, n)
    for dt in (1e-3, 1e-2):
        s1 = orc.State(1 - a - am, a, am)
        s2 = s1.copy()
        bad1, it1 = orc.step_implicit(s1, T0, T1, dt)
        bad2, it2 = orc.step_implicit(s2, T0, T1, dt, **TIGHT)
        assert bad1 == 0 and bad2 == 0
        d = np.abs(s1.alpha_s - s2.alpha_s)
        assert np.all(d <= 2 * (1e-10 + 1e-3 * np.abs(s2.alpha_s))), float(d.max())
        assert float(d.max()) > 0  # the paper's tolerance does stop early
        assert np.all(it1 >= 1) and np.all(it1 <= it2)


def test_iteration_cap_reports_unconverged(orc):
    rng = np.random.default_rng(4)
    n = 100
    am = rng.uniform(0.1, 0.4, n)
    a = rng.uniform(0.2, 0.9, n) * (0.9 - am)
    # one 1 s step at 1250 K without subcycling: one iteration is not enough
    T = np.full(n, 1250.0)
    st = orc.State(1 - a - am, a, am)
    bad, it = orc.step_implicit(st, T, T, 1.0, dt_sub=10.0, max_iter=1)
    assert bad >= 0.9 * n and np.all(it == 1)
    st = orc.State(1 - a - am, a, am)
    bad, it = orc.step_implicit(st, T, T, 1.0, dt_sub=10.0, max_iter=50)
    assert bad == 0 and it.max() > 1


def test_subcycling_splits_into_equal_substeps(orc):
    assert orc.substeps(0.01) == 1
    assert orc.substeps(0.05) == 5
    assert orc.substeps(0.03) == 3
    assert orc.substeps(0.0100001) == 2
    assert orc.substeps(1e-6) == 1
    rng = np.random.default_rng(5)
    n = 64
    am = rng.uniform(0, 0.4, n)
    a = rng.uniform(0.01, 1, n) * (0.9 - am)
    Tn = rng.uniform(950, 1200, n)
    Tn1 = Tn + rng.uniform(-60, 60, n)
    whole = orc.State(1 - a - am, a, am)
    orc.step_implicit(whole, Tn, Tn1, 0.05)
    parts = orc.State(1 - a - am, a, am)
    for s in range(5):
        orc.step_implicit(parts, Tn + (Tn1 - Tn) * s / 5, Tn + (Tn1 - Tn) * (s + 1) / 5, 0.05 / 5)
    assert np.array_equal(whole.alpha_s, parts.alpha_s)
    assert np.array_equal(whole.alpha_m, parts.alpha_m)


def test_startup_states_take_the_closed_form(orc):
    # pure beta at 1000 K (beta -> alpha_s start) and alpha_s = 0.9 at 1200 K
    # (alpha_s -> beta start): identical to the explicit step, no iteration
    for a0, T in ((0.0, 1000.0), (0.9, 1200.0)):
        s1 = orc.State(np.array([1 - a0]), np.array([a0]), np.array([0.0]))
        s2 = s1.copy()
        bad, it = orc.step_implicit(s1, T, T, 1e-3)
        orc.step(s2, T, T, 1e-3)
        assert bad == 0 and it[0] == 0
        assert s1.alpha_s[0] == s2.alpha_s[0] and s1.xbt[0] == s2.xbt[0]


def test_quench_forms_martensite(orc):
    st = orc.State(np.array([1.0]), np.array([0.0]), np.array([0.0]))
    orc.step_implicit(st, 1300.0, 300.0, 1e-3)
    assert st.alpha_m[0] == pytest.approx(1 - math.exp(-0.00415 * (848 - 300)), rel=1e-12)


def test_invariants_random(orc):
    rng = np.random.default_rng(6)
    n = 2000
    am = rng.uniform(0, 0.9, n)
    a = rng.uniform(0, 1, n) * (0.9 - am)
    st = orc.State(1 - a - am, a, am)
    T = rng.uniform(290, 2000, n)
    for dt in (1e-6, 1e-3, 0.02, 0.1):
        T1 = np.clip(T + rng.normal(0, 150, n), 290, 2000)
        bad, _ = orc.step_implicit(st, T, T1, dt)
        assert bad == 0
        xsol = 1 - np.array([orc.liquid_fraction(t) for t in T1])
        assert np.all(st.alpha_s >= 0) and np.all(st.alpha_m >= 0)
        assert np.all(st.alpha_s + st.alpha_m <= 0.9 + 1e-15)
        assert np.allclose(st.alpha_s + st.alpha_m + st.beta, xsol, atol=1e-14)
        T = T1


def test_scan_run_implicit_is_stepping_with_the_scan_temperature(orc):
    import workload
    wl = workload.single_track()
    idx = np.arange(0, wl.grid.n, 331)
    xyz = wl.grid.coords(idx)
    st1 = orc.State.initial(idx.size)
    orc.scan_run_implicit(wl.scan, xyz, st1, 0.0, wl.grid.h, 0.0, 4e-6, 150)
    st2 = orc.State.initial(idx.size)
    T = orc.temperature(wl.scan, xyz, 0.0)
    for s in range(150):
        T1 = orc.temperature(wl.scan, xyz, (s + 1) * 4e-6)
        orc.step_implicit(st2, T, T1, 4e-6)
        T = T1
    assert np.array_equal(st1.alpha_s, st2.alpha_s) and np.array_equal(st1.alpha_m, st2.alpha_m)


def test_second_order_alpha_m_to_alpha_s_at_constant_T(orc):
    # pure tempering (eq. alpha_m_to_alpha_s) at 900 K with X_as + X_am = 0.9:
    # the Appendix A form with D = 0.9, k~ = 0.9 k_as, c = c_as is exact
    # (derivation beside the explicit test of the same equation)
    T, a0, m0, t_end = 900.0, 0.3, 0.6, 2.0
    c = orc.constants()
    exact = orc.logistic_step(a0, 0.9, 0.9 * orc.k_as(T), c["c_as"], t_end)
    errs = []
    for h in (0.04, 0.02, 0.01):
        st = _run_cn(orc, a0, m0, lambda t: T, t_end, h, **TIGHT)
        assert st.alpha_s[0] + st.alpha_m[0] == pytest.approx(0.9, abs=1e-14)
        errs.append(abs(st.alpha_s[0] - exact))
    order = _order(errs)
    assert all(1.85 < o < 2.15 for o in order), (errs, order)
