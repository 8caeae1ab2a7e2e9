"""The allocation-free fused call, mstruct_fused_scan_steps_noalloc, through
the C-ABI.  It runs the kernels of mstruct_fused_scan_steps on buffers in the
library's fixed per-GPU array, so its results must equal that entry point's
bit for bit (stricter than the float32 path's 1e-4 run tolerance against the
oracle, which is checked as well).  Two calls in a row, the second on a
smaller input, so that what the first call left in the array cannot leak
into the second; the host-side rejections (mode, table size) leave the state
untouched."""
import math

import numpy as np
import pytest

import workload

pytestmark = pytest.mark.gpu

RUN_TOL = 1e-4


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


@pytest.fixture(scope="module")
def ctx(torch, ms):
    c = ms.Context(0)
    yield c
    c.close()


def _state(torch, n):
    return [torch.from_numpy(x).cuda() for x in workload.initial_state(n, np.float32)]


def _run(fn, wl, K, mode, g, index=None):
    for L in wl.layers:
        fn(wl.scan, wl.grid, wl.t0(L), wl.dt, L.step_end - L.step_begin, K, *g, z_top=L.z_top, mode=mode,
           index=index)


def _masked():
    wl0 = workload.island_scan(96, 64, 24, n_layers=2, layer_thick=20e-6, steps_per_layer=300, dt=2e-6,
                               seed=77, island=0.5e-3)
    idx = workload.cantilever_mask(96, 64, 24, seed=77, top=6, base=6, leg_frac=0.1)
    return workload.Workload("masked", workload.Grid(96, 64, 24, 10e-6, index=idx), wl0.scan, wl0.layers, wl0.dt,
                             wl0.seed), idx


@pytest.mark.parametrize("mode_name", ["PLAIN", "IMPLICIT"])
def test_noalloc_equals_fused_on_two_calls(torch, ms, ctx, orc, mode_name):
    mode = getattr(ms, "MODE_" + mode_name)
    big = workload.multilayer_block(nx=64, ny=48, nz=24, n_layers=3, layer_thick=30e-6, steps_per_layer=300,
                                    hatch=100e-6, seed=5)
    small = workload.single_track(nx=32, ny=24, nz=8, n_steps=400)
    for wl, K in ((big, 16), (small, 7)):  # the second call is the smaller one
        print(f"noalloc {mode_name}: {wl.name} {wl.grid.n} points, K = {K}", flush=True)
        ref, out = _state(torch, wl.grid.n), _state(torch, wl.grid.n)
        _run(ctx.fused_scan_steps, wl, K, mode, ref)
        _run(ctx.fused_scan_steps_noalloc, wl, K, mode, out)
        torch.cuda.synchronize()
        for x, y in zip(ref, out):
            assert torch.equal(x, y), (mode_name, wl.name)
        if wl is small:
            st = orc.run_workload(wl, np.arange(wl.grid.n), implicit=mode_name == "IMPLICIT")
            for name, x, o in zip(("beta", "alpha_s", "alpha_m"), out, (st.beta, st.alpha_s, st.alpha_m)):
                assert float(np.abs(x.double().cpu().numpy() - o).max()) <= RUN_TOL, (mode_name, name)


def test_noalloc_index_list_then_box(torch, ms, ctx):
    """A masked grid (wave boxes in the array), then a smaller box grid."""
    wl, idx = _masked()
    it = torch.from_numpy(idx).cuda()
    print(f"noalloc masked: {wl.grid.n} points", flush=True)
    ref, out = _state(torch, wl.grid.n), _state(torch, wl.grid.n)
    _run(ctx.fused_scan_steps, wl, 16, ms.MODE_PLAIN, ref, index=it)
    _run(ctx.fused_scan_steps_noalloc, wl, 16, ms.MODE_PLAIN, out, index=it)
    torch.cuda.synchronize()
    for x, y in zip(ref, out):
        assert torch.equal(x, y)
    small = workload.single_track(nx=16, ny=16, nz=4, n_steps=100)
    ref, out = _state(torch, small.grid.n), _state(torch, small.grid.n)
    _run(ctx.fused_scan_steps, small, 64, ms.MODE_PLAIN, ref)
    _run(ctx.fused_scan_steps_noalloc, small, 64, ms.MODE_PLAIN, out)
    torch.cuda.synchronize()
    for x, y in zip(ref, out):
        assert torch.equal(x, y)


def test_noalloc_takes_no_device_memory(torch, ms, ctx):
    """After a first call, a call on a larger grid leaves the device's free
    memory as it was (the allocating entry point would grow its wave flags)."""
    wl0 = workload.single_track(nx=32, ny=32, nz=8, n_steps=50)
    g0 = _state(torch, wl0.grid.n)
    _run(ctx.fused_scan_steps_noalloc, wl0, 16, ms.MODE_PLAIN, g0)
    wl = workload.multilayer_block(nx=128, ny=128, nz=32, n_layers=1, layer_thick=30e-6, steps_per_layer=200,
                                   hatch=100e-6, seed=9)
    g = _state(torch, wl.grid.n)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    _run(ctx.fused_scan_steps_noalloc, wl, 64, ms.MODE_PLAIN, g)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_rejections_leave_state(torch, ms, ctx):
    wl = workload.single_track(nx=16, ny=16, nz=4, n_steps=10)
    g = _state(torch, wl.grid.n)
    before = [x.clone() for x in g]
    # SURROGATE mode needs the context's network buffers
    with pytest.raises(ms.MstructError) as e:
        ctx.fused_scan_steps_noalloc(wl.scan, wl.grid, 0.0, wl.dt, 10, 8, *g, mode=ms.MODE_SURROGATE)
    assert e.value.code == -4
    # a table of 70,001 time points is beyond the 65,536 records of the array
    with pytest.raises(ms.MstructError) as e:
        ctx.fused_scan_steps_noalloc(wl.scan, wl.grid, 0.0, 1e-9, 70_000, 64, *g)
    assert e.value.code == -1 and "allocation-free limit" in str(e.value)
    # envelopes that do not fit: 4-track window, K = 1, ten tracks switching
    # on per step, 12,000 steps (the 49,504 records and pairs alone fit)
    rows = [[20e-6, 50e-6 + 1e-6 * j, 0.0, 1.0, 0.0, 1e-7 * j, 1e-4, 70.0, 1.0] for j in range(20_000)]
    scan = workload.Scan(np.array(rows), wl.scan.conductivity, wl.scan.diffusivity, wl.scan.T0, wl.scan.T_clamp, 4)
    with pytest.raises(ms.MstructError) as e:
        ctx.fused_scan_steps_noalloc(scan, wl.grid, 0.0, 1e-6, 12_000, 1, *g)
    assert e.value.code == -1 and "envelopes" in str(e.value)
    torch.cuda.synchronize()
    for x, y in zip(before, g):
        assert torch.equal(x, y)
    # zero steps: nothing to do
    ctx.fused_scan_steps_noalloc(wl.scan, wl.grid, 0.0, wl.dt, 0, 8, *g)
