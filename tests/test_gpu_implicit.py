"""The implicit step (Crank-Nicolson with fixed-point iteration, WRMS stop,
subcycling) through the C-ABI against the FP64 oracle with the same
tolerances.  Both sides take the stop decision in their own precision; the
residual test is rarely close to 1, so the iteration counts agree and the
results differ by float32 rounding, growing with the number of substeps."""
import numpy as np
import pytest

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
    am = rng.uniform(0, 0.9, n).astype(np.float32)
    a = (rng.uniform(0, 1, n) * (0.9 - am)).astype(np.float32)
    a[:1000] = 0.0
    am[:1000] = 0.0  # pure beta: start-up states
    b = (1 - a - am).astype(np.float32)
    Tp = rng.uniform(290, 2000, n).astype(np.float32)
    Tn = np.clip(Tp + rng.normal(0, 100, n), 290, 2100).astype(np.float32)
    k = n // 3  # a third inside the diffusive range
    Tp[:k] = rng.uniform(900, 1270, k)
    Tn[:k] = Tp[:k] + rng.normal(0, 20, k).astype(np.float32)
    return b, a, am, Tp, Tn


@pytest.mark.parametrize("dt,tol", [(1e-6, 1e-6), (1e-3, 1e-6), (1e-2, 1e-6), (0.05, 2e-6), (0.1, 2e-6),
                                    (1.0, 1e-5)])
def test_implicit_matches_oracle_random(torch, ctx, orc, dt, tol):
    b, a, am, Tp, Tn = _random_case(11, 100_003)  # ragged size
    g = [torch.from_numpy(x.copy()).cuda() for x in (b, a, am)]
    unc = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.step_implicit(torch.from_numpy(Tp).cuda(), torch.from_numpy(Tn).cuda(), dt, *g, unconverged=unc)
    st = orc.State(b.astype(np.float64), a.astype(np.float64), am.astype(np.float64))
    bad, _ = orc.step_implicit(st, Tp.astype(np.float64), Tn.astype(np.float64), dt)
    gb, ga, gm = [x.double().cpu().numpy() for x in g]
    for name, x, y in (("beta", gb, st.beta), ("alpha_s", ga, st.alpha_s), ("alpha_m", gm, st.alpha_m)):
        d = np.abs(x - y)
        assert d.max() <= tol, (dt, name, float(d.max()))
    assert int(unc.item()) == bad == 0


def test_unconverged_substeps_are_counted(torch, ctx, orc):
    # one 1 s step at 1250 K without subcycling: a single iteration does not
    # meet the WRMS test for most points, fifty do
    rng = np.random.default_rng(4)
    n = 4096
    am = rng.uniform(0.1, 0.4, n).astype(np.float32)
    a = (rng.uniform(0.2, 0.9, n) * (0.9 - am)).astype(np.float32)
    b = (1 - a - am).astype(np.float32)
    T = torch.full((n,), 1250.0, device="cuda")
    for max_iter in (1, 50):
        g = [torch.from_numpy(x.copy()).cuda() for x in (b, a, am)]
        unc = torch.zeros(1, dtype=torch.int64, device="cuda")
        ctx.step_implicit(T, T, 1.0, *g, dt_sub=10.0, max_iter=max_iter, unconverged=unc)
        st = orc.State(b.astype(np.float64), a.astype(np.float64), am.astype(np.float64))
        bad, _ = orc.step_implicit(st, 1250.0, 1250.0, 1.0, dt_sub=10.0, max_iter=max_iter)
        got = int(unc.item())
        if max_iter == 1:
            assert bad > 0.9 * n
            assert abs(got - bad) <= 0.01 * n, (got, bad)
        else:
            assert got == bad == 0


def test_startup_states_match_the_explicit_step(torch, ctx):
    n = 1000
    z = torch.zeros(n, device="cuda")
    for a0, T in ((0.0, 1000.0), (0.9, 1200.0)):
        Tt = torch.full((n,), T, device="cuda")
        g1 = [torch.full((n,), 1.0 - a0, device="cuda"), torch.full((n,), a0, device="cuda"), z.clone()]
        g2 = [x.clone() for x in g1]
        ctx.step_implicit(Tt, Tt, 1e-3, *g1)
        ctx.step(Tt, Tt, 1e-3, *g2)
        for x, y in zip(g1, g2):
            assert torch.equal(x, y)


def test_cooldown_history(torch, ctx, orc):
    """Exponential cooling from 1300 K towards 300 K (time constants 0.5-5 s)
    over 10 s in 100 steps of 0.1 s (ten substeps each)."""
    rng = np.random.default_rng(8)
    n = 20_000
    am = rng.uniform(0, 0.3, n)
    a = rng.uniform(0, 1, n) * (0.9 - am)
    tau = rng.uniform(0.5, 5.0, n)
    T_of = lambda t: (300.0 + 1000.0 * np.exp(-t / tau)).astype(np.float32)
    g = [torch.from_numpy(x.astype(np.float32)).cuda() for x in (1 - a - am, a, am)]
    st = orc.State(*[x.astype(np.float32).astype(np.float64) for x in (1 - a - am, a, am)])
    unc = torch.zeros(1, dtype=torch.int64, device="cuda")
    for s in range(100):
        T0, T1 = T_of(0.1 * s), T_of(0.1 * (s + 1))
        ctx.step_implicit(torch.from_numpy(T0).cuda(), torch.from_numpy(T1).cuda(), 0.1, *g, unconverged=unc)
        bad, _ = orc.step_implicit(st, T0.astype(np.float64), T1.astype(np.float64), 0.1)
        assert bad == 0
    assert int(unc.item()) == 0
    gb, ga, gm = [x.double().cpu().numpy() for x in g]
    for name, x, y in (("beta", gb, st.beta), ("alpha_s", ga, st.alpha_s), ("alpha_m", gm, st.alpha_m)):
        d = np.abs(x - y)
        assert d.max() <= 1e-4, (name, float(d.max()))
    assert float(st.alpha_m.max()) > 0.5  # the quench formed martensite
    assert ctx.check_invariants(*g, tol=2e-6) == 0


def test_implicit_argument_errors(torch, ctx):
    import paper_2402_17580_amd as ms
    n = 10
    T = torch.full((n,), 1000.0, device="cuda")
    g = [torch.full((n,), v, device="cuda") for v in (0.5, 0.4, 0.1)]
    for kw in (dict(dt=0.0), dict(dt=1e-3, dt_sub=0.0), dict(dt=1e-3, max_iter=0), dict(dt=1e-3, max_iter=1001),
               dict(dt=1e4, dt_sub=1e-3)):
        dt = kw.pop("dt")
        with pytest.raises(ms.MstructError) as e:
            ctx.step_implicit(T, T, dt, *g, **kw)
        assert e.value.code == -1
    empty = [torch.empty(0, device="cuda") for _ in range(3)]
    ctx.step_implicit(empty[0], empty[0], 1e-3, *empty)


def _errors(torch, g, st):
    out = {}
    for name, x, y in zip(("beta", "alpha_s", "alpha_m"), g, (st.beta, st.alpha_s, st.alpha_m)):
        out[name] = float(np.abs(x.double().cpu().numpy() - y).max())
    return out


@pytest.mark.parametrize("K", [1, 16])
def test_fused_implicit_single_track(torch, ctx, orc, K):
    """The single track (2000 steps of 1 us) with the implicit scheme in the
    fused kernel against the oracle's implicit scan run, all points."""
    import paper_2402_17580_amd as ms
    import workload
    wl = workload.single_track()
    n = wl.grid.n
    g = [torch.from_numpy(x).cuda() for x in workload.initial_state(n, np.float32)]
    ctx.implicit_unconverged(reset=True)
    ms.run_layers(ctx, wl, *g, K=K, mode=ms.MODE_IMPLICIT)
    assert ctx.implicit_unconverged() == 0
    st = orc.run_workload(wl, np.arange(n), implicit=True)
    err = _errors(torch, g, st)
    assert max(err.values()) <= 1e-4, err
    assert float(g[2].max()) > 0.3


def test_fused_implicit_preheated_cooldown(torch, ctx, orc):
    """A track on a body preheated to 1000 K, then 1 s in steps of 20 ms
    (two substeps each): diffusive transformations everywhere, the implicit
    scheme with subcycling in the fused kernel against the oracle."""
    import dataclasses

    import paper_2402_17580_amd as ms
    import workload
    wl0 = workload.single_track(nx=32, ny=32, nz=8)
    scan = dataclasses.replace(wl0.scan, T0=1000.0)
    n = wl0.grid.n
    g = [torch.from_numpy(x).cuda() for x in workload.initial_state(n, np.float32)]
    xyz = wl0.grid.coords(np.arange(n))
    st = orc.State.initial(n)
    ctx.implicit_unconverged(reset=True)
    # the scan itself (600 steps of 1 us), then the cool-down calls
    for t0, dt, steps, K in ((0.0, 1e-6, 600, 16), (6e-4, 0.02, 50, 8)):
        ctx.fused_scan_steps(scan, wl0.grid, t0, dt, steps, K, *g, mode=ms.MODE_IMPLICIT)
        bad = orc.scan_run_implicit(scan, xyz, st, 0.0, wl0.grid.h, t0, dt, steps)
        assert bad == 0
    assert ctx.implicit_unconverged() == 0
    err = _errors(torch, g, st)
    assert max(err.values()) <= 1e-4, err
    # the long steps transformed alpha_s towards the 1000 K equilibrium
    assert abs(float(st.alpha_s.mean()) - 0.9) > 0.01
