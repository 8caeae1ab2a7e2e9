"""The BF16-MFMA network kernels (through the C-ABI) against the FP64
reference with the same bf16 rounding points, element by element.

Both sides round the same values to bfloat16 (inputs, weights, activations,
backward gradients); they differ by float32 against float64 accumulation
(relative ~64 x 2^-24 of the sum of absolute terms) and, through that, by an
occasional activation that rounds to the neighbouring bfloat16 (one bf16
ulp, 2^-8 relative).  Forward bound, per output: every hidden activation
one ulp off, 2^-8 (|W3| |h2| + |W3| |W2| |h1|) with absolute values of the
reference's own weights and activations, plus 1e-5 of the largest output for
the accumulation.  Gradient bound, per entry: 1e-2 |g_ref| (the bf16
rounding of the output gradient, 2^-9, and of the two hidden-layer
gradients, compounded) plus 1e-3 of the largest entry of the same parameter
block (sums over the batch in which terms cancel)."""
import numpy as np
import pytest

import workload
from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu

MEAN = np.array([600.0, 600.0, -13.0, 0.3, 0.4, 0.3])
SCALE = np.array([150.0, 150.0, 0.5, 0.3, 0.3, 0.3])
OSC = np.array([1e-6, 2e-6, 1e-6])


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


def _data(B, seed=2):
    rng = np.random.default_rng(seed)
    X = (rng.normal(0, 1, (B, 6)) * SCALE + MEAN).astype(np.float32)
    Y = (rng.normal(0, 1, (B, 3)) * OSC).astype(np.float32)
    return X, Y


def _params(seed=5):
    p = workload.mlp_init_params(seed)
    p[4544:4608] = 0.02  # b2: some positive bias
    return p


@pytest.mark.parametrize("B", [1, 63, 1000, 70_001])
def test_forward_matches_reference(torch, ctx, B):
    p = _params()
    ctx.mlp_set_params(p, MEAN, SCALE, OSC)
    X, _ = _data(B)
    Xt = torch.from_numpy(X).cuda()
    Yt = torch.empty(B, 3, device="cuda")
    ctx.mlp_forward(Xt, Yt)
    got = Yt.double().cpu().numpy() / OSC
    want, (x, h1, h2) = M.forward(p, X.astype(np.float64), MEAN, SCALE, bf16_round=True)
    P = M.unpack(p)
    W2, W3 = np.abs(M.bf16(P["W2"])), np.abs(M.bf16(P["W3"]))
    bound = 2.0 ** -8 * (h2 @ W3.T + (h1 @ W2.T) @ W3.T) + 1e-5 * np.abs(want).max()
    err = np.abs(got - want)
    assert np.all(err <= bound), (float((err / bound).max()), int(np.argmax(err / bound)))
    # and in aggregate far inside the bound
    assert err.mean() <= 1e-3 * np.abs(want).max(), float(err.mean())


def test_gradient_matches_reference(torch, ctx):
    p = _params(7)
    ctx.mlp_set_params(p, MEAN, SCALE, OSC)
    B = 5000
    X, Y = _data(B, 3)
    g = torch.empty(4803, device="cuda")
    loss = torch.empty(1, device="cuda")
    ctx.mlp_grad(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), g, loss)
    lw, gw = M.loss_and_grad(p, X.astype(np.float64), Y.astype(np.float64), MEAN, SCALE, OSC, bf16_round=True)
    gg = g.double().cpu().numpy()
    assert loss.item() == pytest.approx(lw, rel=5e-3)
    for name, (a, b, _) in M.SLICES.items():
        ref, got = gw[a:b], gg[a:b]
        bound = 1e-2 * np.abs(ref) + 1e-3 * np.abs(ref).max()
        over = np.abs(got - ref) / bound
        assert np.all(over <= 1.0), (name, float(over.max()), int(over.argmax()))
        d = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
        assert d < 2e-2, (name, d)
    # deterministic: same call, same bits
    g2 = torch.empty_like(g)
    loss2 = torch.empty_like(loss)
    ctx.mlp_grad(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), g2, loss2)
    assert torch.equal(g, g2) and torch.equal(loss, loss2)


def test_adam_first_step(torch, ctx):
    p = _params(9)
    ctx.mlp_set_params(p, MEAN, SCALE, OSC)
    B = 2048
    X, Y = _data(B, 4)
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    g = torch.empty(4803, device="cuda")
    loss = torch.empty(1, device="cuda")
    ctx.mlp_grad(Xt, Yt, g, loss)
    lr = 1e-3
    ctx.mlp_train_step(Xt, Yt, lr)
    p1 = ctx.mlp_get_params()
    gg = g.cpu().numpy()
    big = np.abs(gg) > 1e-5
    # first Adam step: m^ = g, v^ = g^2, so the step is lr * g / (|g| + eps)
    assert np.allclose((p1 - p)[big], -lr * np.sign(gg[big]), rtol=1e-3, atol=1e-7)


def test_training_reduces_loss(torch, ctx):
    # a smooth synthetic target: the network must fit it
    p = _params(11)
    ctx.mlp_set_params(p, MEAN, SCALE, OSC)
    B = 16384
    rng = np.random.default_rng(12)
    X = (rng.normal(0, 1, (B, 6)) * SCALE + MEAN).astype(np.float32)
    xn = (X - MEAN) / SCALE
    Y = (np.stack([np.tanh(xn[:, 0] - xn[:, 4]), xn[:, 1] * xn[:, 5], np.sin(xn[:, 3])], 1) * OSC).astype(np.float32)
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    loss = torch.empty(1, device="cuda")
    first = None
    for it in range(300):
        ctx.mlp_train_step(Xt, Yt, 3e-3, loss)
        if it == 0:
            first = loss.item()
    torch.cuda.synchronize()
    assert loss.item() < 0.1 * first, (first, loss.item())


def test_surrogate_mode_with_zero_network(torch, ctx, orc):
    """Surrogate mode with an all-zero network: unflagged blocks take one
    explicit step of K dt, flagged ones the K plain steps.
    The result stays within the surrogate tolerance of the oracle and keeps
    the invariants."""
    import paper_2402_17580_amd as ms
    ctx.mlp_set_params(np.zeros(4803, np.float32), MEAN, SCALE, OSC)
    wl = workload.single_track()
    n = wl.grid.n
    g = [torch.from_numpy(x).cuda() for x in workload.initial_state(n, np.float32)]
    ms.run_layers(ctx, wl, *g, K=8, mode=ms.MODE_SURROGATE)
    torch.cuda.synchronize()
    st = orc.run_workload(wl, np.arange(n))
    errs = [float(np.abs(x.double().cpu().numpy() - y).max()) for x, y in zip(g, (st.beta, st.alpha_s, st.alpha_m))]
    print("zero-network surrogate errors", errs)
    assert max(errs) <= 1e-3
    assert ctx.check_invariants(*g, tol=2e-6) == 0


@pytest.mark.parametrize("K,window,masked", [(1, 1, False), (64, 3, False), (8, 2, True), (13, 4, True)])
def test_surrogate_mode_edge_cases(torch, ctx, orc, K, window, masked):
    """The shipped K = 8 network in surrogate mode with other block lengths
    (1, 13 with a partial last block, 64), other window sizes and a masked
    grid (index list, points above the layers inactive); within the surrogate
    tolerance of the oracle, inactive points untouched."""
    import paper_2402_17580_amd as ms
    from paper_2402_17580_amd import surrogate as S
    S.Surrogate.load(S.DEFAULT_WEIGHTS).load_into(ctx)
    if masked:
        wl0 = workload.island_scan(96, 64, 24, n_layers=3, layer_thick=20e-6, steps_per_layer=303, dt=2e-6,
                                   seed=77, island=0.5e-3, window=window)
        idx = workload.cantilever_mask(96, 64, 24, seed=77, top=6, base=6, leg_frac=0.1)
        wl = workload.Workload("masked", workload.Grid(96, 64, 24, 10e-6, index=idx), wl0.scan, wl0.layers, wl0.dt,
                               wl0.seed)
        index = torch.from_numpy(idx).cuda()
    else:
        wl = workload.multilayer_block(nx=48, ny=40, nz=12, n_layers=2, layer_thick=30e-6, steps_per_layer=401,
                                       hatch=100e-6, seed=3, window=window)
        index = None
    n = wl.grid.n
    g = [torch.from_numpy(x).cuda() for x in workload.initial_state(n, np.float32)]
    ms.run_layers(ctx, wl, *g, K=K, mode=ms.MODE_SURROGATE, index=index)
    torch.cuda.synchronize()
    st = orc.run_workload(wl, np.arange(n))
    errs = [float(np.abs(x.double().cpu().numpy() - y).max()) for x, y in zip(g, (st.beta, st.alpha_s, st.alpha_m))]
    print("surrogate edge case", K, window, masked, errs)
    assert max(errs) <= 1e-3
    assert ctx.check_invariants(*g, tol=2e-6) == 0
    z = wl.grid.coords(np.arange(n))[:, 2]
    never = z > wl.layers[-1].z_top + 1e-3 * wl.grid.h
    assert never.sum() == 0 or np.all(g[1].cpu().numpy()[never] == np.float32(0.9))
