"""MSTRUCT_OPTION_COUNT_WAVES: the fused launches' device-side counts of the
points whose state they read and write and of their waves by class.  The
counts must add up to the launches' points, agree with what the launch
certificates switched off implies, and leave the results bit for bit as
they are (the counts are measurement only)."""
import math

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


def _point_launches(wl, K):
    """Active points summed over the launches of every layer."""
    g = wl.grid
    return sum((g.nz - g.first_active_k(L.z_top)) * g.nx * g.ny * math.ceil((L.step_end - L.step_begin) / K)
               for L in wl.layers)


@pytest.mark.parametrize("mode_name", ["PLAIN", "IMPLICIT"])
def test_wave_counts_add_up(torch, mode_name):
    import paper_2402_17580_amd as ms
    mode = getattr(ms, "MODE_" + mode_name)
    # 64 x 48 points per plane: every wave of 64 points is whole
    wl = workload.multilayer_block(nx=64, ny=48, nz=20, n_layers=3, layer_thick=30e-6, steps_per_layer=400,
                                   hatch=100e-6, seed=12)
    K = 32
    total = _point_launches(wl, K)
    ctx = ms.Context(0)
    try:
        outs, counts = [], []
        for count, skip in ((0, 1), (1, 1), (1, 0)):
            ctx.set_option(ms.OPTION_COUNT_WAVES, count)
            ctx.set_option(ms.OPTION_SKIP_COLD_WAVES, skip)
            ctx.wave_counts(reset=True)
            g = [torch.from_numpy(x).cuda() for x in workload.initial_state(wl.grid.n, np.float32)]
            ms.run_layers(ctx, wl, *g, K=K, mode=mode)
            outs.append([x.cpu().numpy() for x in g])
            counts.append(ctx.wave_counts(reset=True))
        for x, y in zip(outs[0], outs[1]):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
        assert all(v == 0 for v in counts[0].values())  # not counted while the option is off
        c = counts[1]
        assert c["points_loaded"] + 64 * c["flagged_waves"] == total, c
        assert c["points_loaded"] == 64 * (c["still_waves"] + c["cold_waves"] + c["hot_waves"]), c
        assert c["points_stored"] == 64 * (c["cold_waves"] + c["hot_waves"]), c
        assert c["flagged_waves"] > 0 and c["still_waves"] > 0 and c["hot_waves"] > 0, c
        # certificates off: every wave reads, steps and stores
        c = counts[2]
        assert c["points_loaded"] == total and c["points_stored"] == total, c
        assert c["hot_waves"] * 64 == total and c["still_waves"] == c["cold_waves"] == c["flagged_waves"] == 0, c
    finally:
        ctx.set_option(ms.OPTION_COUNT_WAVES, 0)
        ctx.set_option(ms.OPTION_SKIP_COLD_WAVES, 1)
        ctx.close()
