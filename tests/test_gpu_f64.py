"""The float64 explicit step (mstruct_step_f64) with the device math library,
with exponent-bit exp2 / log2 and with the paper's own exp / ln (Sec. 3.3,
MSTRUCT_F64_PAPER), against the FP64 oracle (libm).  The first two evaluate
the formulas to double accuracy, so they agree with the oracle to a few ulps
per step and stay at rounding level over a 2000-step history.

The paper's method is only as accurate as its fitted correction polynomials:
2^y to e_exp (relative) and log2 to e_log (absolute), as measured on the
CPU from the printed coefficients (tests/paper_polynomials.py: 1.2e-10 and
3.0e-8).  A rate k x^p y^q evaluated as 2^(p log2 x + q log2 y) is then off
by at most (p + q) ln2 e_log + e_exp relative (p + q = 2 for every rate);
the closed-form start-up raises w to the power c (c_beta = 11 at most) after
log2 and exp2, (c + 1) ln2 e_log + 2 e_exp relative; a fraction or an
increment is at most 0.9.  So one step is off by at most
0.9 ((c_beta + 1) ln2 e_log + 2 e_exp) ~ 2.3e-7; the bar is twice that.  Over
a history the increments' errors add up to the total variation of the
fractions (a few times 0.9) times the rate error, plus the start-up steps:
the bar is ten times the step bar."""
import math

import numpy as np
import pytest

import workload
from paper_polynomials import error_bounds


def paper_bars():
    e_exp, e_log = error_bounds()
    step = 2.0 * 0.9 * ((11.0 + 1.0) * math.log(2.0) * e_log + 2.0 * e_exp) + 1e-13
    return step, 10.0 * step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2402_17580_amd as ms
    c = ms.Context(0)
    yield c
    c.close()


def _random_case(seed, n):
    rng = np.random.default_rng(seed)
    am = rng.uniform(0, 0.9, n)
    a = rng.uniform(0, 1, n) * (0.9 - am)
    a[:1000] = 0.0
    am[:1000] = 0.0
    a[1000:2000] = 0.9
    am[1000:2000] = 0.0
    b = 1 - a - am
    Tp = rng.uniform(290, 2000, n)
    Tn = np.clip(Tp + rng.normal(0, 200, n), 290, 2100)
    Tp[:2000] = rng.uniform(940, 1270, 2000)
    Tn[:2000] = Tp[:2000] + rng.normal(0, 5, 2000)
    return b, a, am, Tp, Tn


@pytest.mark.parametrize("math_mode", [0, 1, 2])
def test_f64_step_matches_oracle(torch, ctx, orc, math_mode):
    b, a, am, Tp, Tn = _random_case(11, 100_003)
    bar = 1e-13 if math_mode != 2 else paper_bars()[0]
    worst = 0.0
    for dt in (1e-6, 2e-6, 1e-3, 0.1):
        g = [torch.from_numpy(x.copy()).cuda() for x in (b, a, am)]
        ctx.step_f64(torch.from_numpy(Tp).cuda(), torch.from_numpy(Tn).cuda(), dt, *g, math=math_mode)
        st = orc.State(b, a, am)
        orc.step(st, Tp, Tn, dt)
        for name, x, y in zip(("beta", "alpha_s", "alpha_m"), g, (st.beta, st.alpha_s, st.alpha_m)):
            d = np.abs(x.cpu().numpy() - y)
            worst = max(worst, float(d.max()))
            assert d.max() <= bar, (math_mode, dt, name, float(d.max()), bar)
    print(f"float64 step, math {math_mode}: max difference from the oracle {worst:.3g} (bar {bar:.3g})")
    if math_mode == 2:
        assert worst > 1e-13  # the fitted polynomials are in use, not the library's functions


def test_f64_histories_match_oracle(torch, ctx, orc):
    """2000 steps of 1 us of the single track on every 8th point, with the
    oracle's float64 temperatures, in both math modes."""
    wl = workload.single_track()
    idx = np.arange(0, wl.grid.n, 8)
    xyz = wl.grid.coords(idx)
    n_steps = wl.n_steps
    T = np.stack([orc.temperature(wl.scan, xyz, s * wl.dt) for s in range(n_steps + 1)], 1)
    st = orc.State.initial(idx.size)
    orc.history_run(st, T, wl.dt)
    Td = torch.from_numpy(np.ascontiguousarray(T.T)).cuda()
    for math_mode in (0, 1, 2):
        bar = 1e-11 if math_mode != 2 else paper_bars()[1]
        g = [torch.from_numpy(x).cuda() for x in workload.initial_state(idx.size, np.float64)]
        for s in range(n_steps):
            ctx.step_f64(Td[s], Td[s + 1], wl.dt, *g, math=math_mode)
        for name, x, y in zip(("beta", "alpha_s", "alpha_m"), g, (st.beta, st.alpha_s, st.alpha_m)):
            d = np.abs(x.cpu().numpy() - y)
            assert d.max() <= bar, (math_mode, name, float(d.max()), bar)
        assert float(g[2].max()) > 0.3  # the track formed martensite


def test_f64_argument_errors(torch, ctx):
    import paper_2402_17580_amd as ms
    T = torch.full((4,), 1000.0, dtype=torch.float64, device="cuda")
    g = [torch.full((4,), v, dtype=torch.float64, device="cuda") for v in (0.5, 0.4, 0.1)]
    with pytest.raises(ms.MstructError):
        ctx.step_f64(T, T, 0.0, *g)
    with pytest.raises(ms.MstructError):
        ctx.step_f64(T, T, 1e-6, *g, math=3)
    with pytest.raises(ms.MstructError):  # float32 arrays are refused by the binding
        ctx.step_f64(T.float(), T.float(), 1e-6, *[x.float() for x in g])
