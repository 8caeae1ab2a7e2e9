"""The two switchable readings of the paper (mstruct_params.correction_T and
martensite_mode) through the C-ABI against the oracle with the same
readings.  Bars as in the parity tests: 2e-6 per step (float32 arithmetic
with hardware exp2/log2), 1e-4 per run, 1e-13 per float64 step.  Each
non-default reading also has to change the result somewhere, so that a flag
the kernels ignore cannot pass."""
import numpy as np
import pytest

import workload

pytestmark = pytest.mark.gpu

STEP_TOL = 2e-6
RUN_TOL = 1e-4
READINGS = [("prev", "max"), ("next", "assign"), ("prev", "assign")]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ms():
    import paper_2402_17580_amd as m
    return m


def _random_states(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0, 0.9, n).astype(np.float32)
    m = (rng.uniform(0, 1, n) * (0.9 - a)).astype(np.float32)
    a[:500] = 0.0
    m[500:1000] = 0.0
    Tp = rng.uniform(300, 1500, n).astype(np.float32)
    Tn = (Tp + rng.uniform(-400, 400, n)).astype(np.float32)
    # quenches and reheats across the martensite start
    Tp[1000:2000], Tn[1000:2000] = 1400.0, 300.0
    Tp[2000:3000], Tn[2000:3000] = 300.0, 700.0
    return Tp, Tn, (1.0 - a - m).astype(np.float32), a, m


@pytest.mark.parametrize("corr,mart", READINGS)
def test_step_with_readings(torch, ms, orc, corr, mart):
    n = 20_011
    Tp, Tn, b, a, m = _random_states(n, 31)
    ctx = ms.Context(0, correction_T=corr, martensite=mart)
    try:
        for dt in (2e-6, 1e-3):
            g = [torch.from_numpy(x.copy()).cuda() for x in (b, a, m)]
            ctx.step(torch.from_numpy(Tp).cuda(), torch.from_numpy(Tn).cuda(), dt, *g)
            st = orc.State(b.astype(np.float64), a.astype(np.float64), m.astype(np.float64))
            with orc.readings(correction_T=corr, martensite=mart):
                orc.step(st, Tp.astype(np.float64), Tn.astype(np.float64), dt)
            torch.cuda.synchronize()
            for name, x, y in zip(("beta", "alpha_s", "alpha_m"), g, (st.beta, st.alpha_s, st.alpha_m)):
                d = float(np.abs(x.double().cpu().numpy() - y).max())
                assert d <= STEP_TOL, (corr, mart, dt, name, d)
        # the implicit step: only the formation law switches (g at T^{n+1} either way)
        g = [torch.from_numpy(x.copy()).cuda() for x in (b, a, m)]
        ctx.step_implicit(torch.from_numpy(Tp).cuda(), torch.from_numpy(Tn).cuda(), 1e-3, *g)
        st = orc.State(b.astype(np.float64), a.astype(np.float64), m.astype(np.float64))
        with orc.readings(correction_T=corr, martensite=mart):
            orc.step_implicit(st, Tp.astype(np.float64), Tn.astype(np.float64), 1e-3)
        torch.cuda.synchronize()
        for name, x, y in zip(("beta", "alpha_s", "alpha_m"), g, (st.beta, st.alpha_s, st.alpha_m)):
            d = float(np.abs(x.double().cpu().numpy() - y).max())
            assert d <= 1e-5, ("implicit", corr, mart, name, d)
        # the float64 step in both math modes
        for math_mode in (ms.F64_LIBRARY, ms.F64_SYNTH):
            g = [torch.from_numpy(x.astype(np.float64)).cuda() for x in (b, a, m)]
            ctx.step_f64(torch.from_numpy(Tp.astype(np.float64)).cuda(), torch.from_numpy(Tn.astype(np.float64)).cuda(),
                         1e-3, *g, math=math_mode)
            st = orc.State(b.astype(np.float64), a.astype(np.float64), m.astype(np.float64))
            with orc.readings(correction_T=corr, martensite=mart):
                orc.step(st, Tp.astype(np.float64), Tn.astype(np.float64), 1e-3)
            torch.cuda.synchronize()
            for name, x, y in zip(("beta", "alpha_s", "alpha_m"), g, (st.beta, st.alpha_s, st.alpha_m)):
                d = float(np.abs(x.cpu().numpy() - y).max())
                assert d <= 1e-13, ("f64", math_mode, corr, mart, name, d)
    finally:
        ctx.close()


def test_readings_change_the_step(torch, ms):
    """Each non-default reading changes mstruct_step on the quench and reheat
    states (and mstruct_correct follows the formation law)."""
    n = 4000
    Tp, Tn, b, a, m = _random_states(n, 7)
    outs = {}
    for corr, mart in [("next", "max")] + READINGS:
        ctx = ms.Context(0, correction_T=corr, martensite=mart)
        g = [torch.from_numpy(x.copy()).cuda() for x in (b, a, m)]
        ctx.step(torch.from_numpy(Tp).cuda(), torch.from_numpy(Tn).cuda(), 1e-6, *g)
        c = [torch.from_numpy(x.copy()).cuda() for x in (b, a, m)]
        ctx.correct(torch.from_numpy(Tn).cuda(), *c)
        torch.cuda.synchronize()
        outs[(corr, mart)] = ([x.cpu().numpy() for x in g], [x.cpu().numpy() for x in c])
        ctx.close()
    base_step, base_corr = outs[("next", "max")]
    for key, (step, corr_out) in outs.items():
        if key == ("next", "max"):
            continue
        assert not np.array_equal(step[2], base_step[2]), key
        assert np.array_equal(corr_out[2], base_corr[2]) == (key[1] == "max"), key


@pytest.mark.parametrize("corr,mart", READINGS)
def test_fused_runs_with_readings(torch, ms, orc, corr, mart):
    """The single track (all 32,768 points, 2000 steps) and a two-layer block
    whose second layer reheats the first one's martensite, fused PLAIN at
    K = 16, and the block in fused IMPLICIT mode; SURROGATE mode is rejected."""
    ctx = ms.Context(0, correction_T=corr, martensite=mart)
    try:
        c1 = workload.single_track()
        blk = workload.multilayer_block(nx=48, ny=40, nz=12, n_layers=2, layer_thick=30e-6, steps_per_layer=600,
                                        hatch=100e-6, seed=8)
        for wl, mode in ((c1, ms.MODE_PLAIN), (blk, ms.MODE_PLAIN), (blk, ms.MODE_IMPLICIT)):
            g = [torch.from_numpy(x).cuda() for x in workload.initial_state(wl.grid.n, np.float32)]
            ms.run_layers(ctx, wl, *g, K=16, mode=mode)
            with orc.readings(correction_T=corr, martensite=mart):
                st = orc.run_workload(wl, np.arange(wl.grid.n), implicit=mode == ms.MODE_IMPLICIT)
            torch.cuda.synchronize()
            for name, x, y in zip(("beta", "alpha_s", "alpha_m"), g, (st.beta, st.alpha_s, st.alpha_m)):
                d = float(np.abs(x.double().cpu().numpy() - y).max())
                assert d <= RUN_TOL, (wl.name, mode, corr, mart, name, d)
        from paper_2402_17580_amd import surrogate as S
        S.Surrogate.load(S.DEFAULT_WEIGHTS).load_into(ctx)
        g = [torch.from_numpy(x).cuda() for x in workload.initial_state(c1.grid.n, np.float32)]
        with pytest.raises(ms.MstructError) as e:
            ctx.fused_scan_steps(c1.scan, c1.grid, 0.0, c1.dt, 8, 8, *g, mode=ms.MODE_SURROGATE)
        assert e.value.code == -4
    finally:
        ctx.close()
