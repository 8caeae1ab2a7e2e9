"""The largest inputs the boundary accepts (2^31 - 1 points per call; a box of
at most 2^31 - 1 points), checked on sampled points against the oracle, and
the host-side rejection of anything larger.  The arrays of one test take
about 45 GB of the GPU's memory."""
import ctypes

import numpy as np
import pytest

import workload

pytestmark = pytest.mark.gpu

N_MAX = (1 << 31) - 1


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


def _sample(n, rng, extra=()):
    idx = np.concatenate([np.arange(64), np.arange(n - 64, n), rng.integers(0, n, 4096), *extra])
    return np.unique(idx.astype(np.int64))


def test_largest_point_count_steps(torch, ctx, orc):
    """mstruct_step and mstruct_step_implicit on 2^31 - 1 points (a ragged
    tail after the 4-point vector groups), random states and temperatures."""
    n = N_MAX
    gen = torch.Generator(device="cuda").manual_seed(7)
    a = torch.rand(n, generator=gen, device="cuda").mul_(0.9)
    m = torch.rand(n, generator=gen, device="cuda").mul_(0.9 - a)
    b = torch.ones(n, device="cuda").sub_(a).sub_(m)
    Tp = torch.rand(n, generator=gen, device="cuda").mul_(1710.0).add_(290.0)
    Tn = torch.randn(n, generator=gen, device="cuda").mul_(50.0).add_(Tp)
    idx = _sample(n, np.random.default_rng(8))
    it = torch.from_numpy(idx).cuda()
    inputs = [x[it].double().cpu().numpy() for x in (b, a, m, Tp, Tn)]
    a0, m0 = a.clone(), m.clone()
    for step, dt in (("step", 1e-3), ("step_implicit", 0.05)):
        a.copy_(a0)
        m.copy_(m0)
        torch.cuda.synchronize()
        getattr(ctx, step)(Tp, Tn, dt, b, a, m)
        torch.cuda.synchronize()
        st = orc.State(*[x.copy() for x in inputs[:3]])
        if step == "step":
            orc.step(st, inputs[3], inputs[4], dt)
        else:
            orc.step_implicit(st, inputs[3], inputs[4], dt)
        for x, y in zip((b, a, m), (st.beta, st.alpha_s, st.alpha_m)):
            d = np.abs(x[it].double().cpu().numpy() - y)
            assert float(d.max()) <= 2e-6, (step, float(d.max()))
    del a, m, b, Tp, Tn, a0, m0
    torch.cuda.empty_cache()


def test_largest_box_fused(torch, ctx, orc):
    """The fused kernels on a 2047 x 1024 x 1024 box (2,146,435,072 points,
    the largest box below 2^31 with these factors): the single track on its
    top surface, 32 steps of 1 us in two launches of 16 (the second on the
    slot kernel, with the wave flags of 33.5M waves); sampled points
    including the track's neighbourhood and the last planes, against the
    oracle."""
    import dataclasses

    import paper_2402_17580_amd as ms
    wl0 = workload.single_track()
    grid = workload.Grid(2047, 1024, 1024, wl0.grid.h)
    wl = dataclasses.replace(wl0, grid=grid, layers=[workload.Layer(0, 32, 0.0)])
    n = grid.n
    assert n < 1 << 31
    g = [torch.full((n,), v, device="cuda") for v in (0.1, 0.9, 0.0)]
    ms.run_layers(ctx, wl, *g, K=16)
    torch.cuda.synchronize()
    near = np.array([i + grid.nx * (j + grid.ny * k) for k in range(4) for j in range(12, 20) for i in range(8)])
    idx = _sample(n, np.random.default_rng(9), extra=(near,))
    it = torch.from_numpy(idx).cuda()
    st = orc.run_workload(wl, idx)
    for x, y in zip(g, (st.beta, st.alpha_s, st.alpha_m)):
        d = np.abs(x[it].double().cpu().numpy() - y)
        assert float(d.max()) <= 1e-4, float(d.max())
    assert float(st.alpha_s.min()) < 0.9  # the track changed the sampled neighbourhood
    del g
    torch.cuda.empty_cache()


def test_sizes_beyond_the_limit_are_rejected(torch, ctx):
    """Rejected on the host with MSTRUCT_EINVAL before anything is launched
    (the pointers are valid but far too short, and are never touched)."""
    import paper_2402_17580_amd as ms
    L = ms.lib()
    buf = torch.zeros(16, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ph = ms.PhasesC(p.value, p.value, p.value, 1 << 31, None)
    assert L.mstruct_step(ctx._h, p, p, ctypes.c_double(1e-3), ctypes.byref(ph), stream) == -1
    assert L.mstruct_step_implicit(ctx._h, p, p, ctypes.c_double(1e-3), ctypes.c_double(0.01), 50,
                                   ctypes.byref(ph), None, stream) == -1
    wl = workload.single_track()
    sc = ms.scan_struct(wl.scan)
    for dims in ((2048, 1024, 1024), (1 << 40, 1 << 40, 4), (1 << 31, 1, 1), (1, 1, 1 << 62)):
        n = 16
        pts = ms.PointsC(*dims, wl.grid.h, 0.0, 0.0, 0.0, None, n, float("inf"))
        ph = ms.PhasesC(p.value, p.value, p.value, n, None)
        rc = L.mstruct_fused_scan_steps(ctx._h, ctypes.byref(sc), ctypes.byref(pts), ctypes.c_double(0.0),
                                        ctypes.c_double(1e-6), ctypes.c_int64(16), 16, 0, ctypes.byref(ph), stream)
        assert rc == -1, dims
    torch.cuda.synchronize()
