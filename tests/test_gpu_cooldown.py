"""The inter-layer cool-down workload (the paper's schedule: after each
layer's scan, 2000 steps at the scan step, then the step doubled after every
ten steps, the microstructure subcycled at 0.01 s; explicit scheme while
scanning, implicit scheme while cooling; a final 100 s cool-down after the
last layer) against the oracle."""
import numpy as np
import pytest

import workload

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


def _run(torch, ctx, pw, K=16):
    import paper_2402_17580_amd as ms
    g = [torch.from_numpy(x).cuda() for x in workload.initial_state(pw.grid.n, np.float32)]
    ctx.implicit_unconverged(reset=True)
    ms.run_phases(ctx, pw, *g, K=K)
    torch.cuda.synchronize()
    return g


def _check(g, st, idx, tol=1e-4):
    err = {}
    for name, x, y in zip(("beta", "alpha_s", "alpha_m"), g, (st.beta, st.alpha_s, st.alpha_m)):
        d = np.abs(x.double().cpu().numpy()[idx] - y)
        err[name] = float(d.max())
    assert max(err.values()) <= tol, err
    return err


def test_cooldown_small_all_points(torch, ctx, orc):
    pw = workload.multilayer_cooldown(nx=48, ny=40, nz=12, n_layers=2, steps_per_layer=400)
    assert any(p.dt > 0.01 for p in pw.phases)  # the schedule reaches subcycled steps
    g = _run(torch, ctx, pw)
    assert ctx.implicit_unconverged() == 0
    idx = np.arange(pw.grid.n)
    st, bad = orc.run_phases(pw, idx)
    assert bad == 0
    print(_check(g, st, idx))
    assert float(st.alpha_m.max()) > 0.5


def test_multilayer_cooldown_full_size_sampled(torch, ctx, orc):
    """256x256x128, 10 layers of 2000 scan steps, each followed by 1 s of
    cool-down (2146 steps), then the final 100 s (1000 steps of 0.1 s); a
    seeded 0.1 % sample against the oracle, in launches of 16 and of 64
    steps (the benchmark's)."""
    pw = workload.multilayer_cooldown()
    idx = workload.sample_indices(pw.grid.n, 1e-3, pw.seed)
    st, bad = orc.run_phases(pw, idx)
    assert bad == 0
    for K in (16, 64):
        g = _run(torch, ctx, pw, K=K)
        assert ctx.implicit_unconverged() == 0
        print("multilayer cooldown sample", idx.size, "K", K, _check(g, st, idx))
        assert ctx.check_invariants(*g, tol=2e-6) == 0
