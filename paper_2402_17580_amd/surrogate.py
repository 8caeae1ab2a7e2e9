"""Training data and training driver for the surrogate network.

Transitions come from the plain explicit method itself, run on the GPU by the
library: during a run of a workload, at block boundaries, a seeded subset of
the points the error indicator leaves to the network is advanced K plain
steps for several dt; the target is the difference of (alpha_s, alpha_m,
beta) between those K steps and one explicit step of K dt over the block
(``mstruct_step`` with the block-end temperatures), i.e. the network learns a
correction to the method's own large-step update.  Training uses the library's BF16-MFMA kernels
(``mstruct_mlp_train_step``).  torch is used for buffers and index selection
only.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

import paper_2402_17580_amd as ms

# error-indicator thresholds (K): network only for blocks entirely below
# T_COLD, or entirely inside [T_HOT_LO, T_HOT_HI], with |T_end - T_start| <= DT_MAX
T_COLD, T_HOT_LO, T_HOT_HI, DT_MAX = 823.0, 1398.0, 1853.0, 50.0
INDICATOR = (T_COLD, T_HOT_LO, T_HOT_HI, DT_MAX)
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "surrogate_multilayer_block.npz")  # K = 8
WEIGHTS_K16 = os.path.join(HERE, "surrogate_multilayer_block_k16.npz")


@dataclasses.dataclass
class Surrogate:
    params: np.ndarray
    in_mean: np.ndarray
    in_scale: np.ndarray
    out_scale: np.ndarray
    K: int
    indicator: tuple = INDICATOR

    def load_into(self, ctx: ms.Context):
        ctx.mlp_set_params(self.params, self.in_mean, self.in_scale, self.out_scale, self.indicator)

    def save(self, path):
        np.savez(path, params=self.params, in_mean=self.in_mean, in_scale=self.in_scale, out_scale=self.out_scale,
                 K=np.array(self.K), indicator=np.array(self.indicator))

    @classmethod
    def load(cls, path):
        z = np.load(path, allow_pickle=False)
        return cls(z["params"], z["in_mean"], z["in_scale"], z["out_scale"], int(z["K"]),
                   tuple(float(v) for v in z["indicator"]))


def network_allowed(torch, T0, TK):
    """The indicator of the surrogate kernel, for selecting training points."""
    lo, hi = torch.minimum(T0, TK), torch.maximum(T0, TK)
    cold = hi < T_COLD
    hot = (lo >= T_HOT_LO) & (hi <= T_HOT_HI)
    return (cold | hot) & ((TK - T0).abs() <= DT_MAX)


def generate_transitions(ctx, wl, K=8, dts=(1e-6, 2e-6, 4e-6), every=512, per_pick=16000, seed=4,
                         layers=None, K_run=16):
    """Run the workload (plain, fused) and collect transitions at every
    `every`-th step of each layer.  Returns X [N, 6], Y [N, 3] torch tensors
    (float32, on the GPU)."""
    import torch
    dev = torch.device("cuda")
    g = wl.grid
    n = g.n
    b, a, m = [torch.from_numpy(x).to(dev) for x in workload_initial(n)]
    T0 = torch.empty(n, device=dev)
    TK = torch.empty(n, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    Xs, Ys = [], []
    for L in (wl.layers if layers is None else layers):
        s = L.step_begin
        off = g.first_active_k(L.z_top) * g.nx * g.ny if g.index is None else 0
        while s < L.step_end:
            seg = min(every, L.step_end - s)
            t_s = float(s) * wl.dt
            ctx.temperature(wl.scan, g, t_s, T0, z_top=L.z_top)
            for dtp in dts:
                ctx.temperature(wl.scan, g, t_s + K * dtp, TK, z_top=L.z_top)
                ok = network_allowed(torch, T0[off:], TK[off:])
                idx = _pick(torch, a[off:], m[off:], ok, per_pick, gen) + off
                if idx.numel() == 0:
                    continue
                Xs_, Ys_ = _transitions(ctx, wl, L, idx, b, a, m, T0, TK, t_s, dtp, K)
                Xs.append(Xs_)
                Ys.append(Ys_)
            ctx.fused_scan_steps(wl.scan, g, t_s, wl.dt, seg, K_run, b, a, m, z_top=L.z_top)
            s += seg
    return torch.cat(Xs), torch.cat(Ys)


def workload_initial(n):
    import workload
    return workload.initial_state(n, np.float32)


def _pick(torch, a, m, ok, k, gen):
    """Seeded choice of up to k allowed points, three quarters of them from
    non-trivial states (martensite present or partial stable alpha)."""
    nontrivial = ok & ((m > 1e-7) | ((a > 1e-7) & (a < 0.9 - 1e-6)))
    trivial = ok & ~nontrivial
    out = []
    for mask, share in ((nontrivial, 0.75), (trivial, 0.25)):
        cand = torch.nonzero(mask).flatten()
        take = min(int(k * share), cand.numel())
        if take:
            out.append(cand[torch.randperm(cand.numel(), generator=gen, device=cand.device)[:take]])
    if not out:
        return torch.zeros(0, dtype=torch.int64, device=a.device)
    return torch.sort(torch.cat(out)).values


def _transitions(ctx, wl, L, idx, b, a, m, T0, TK, t_s, dtp, K):
    import torch
    dev = b.device
    cnt = idx.numel()
    before = [torch.empty(cnt, device=dev) for _ in range(3)]
    for src, dst in zip((b, a, m), before):
        ctx.gather(src, idx, dst)
    t0s, tks = torch.empty(cnt, device=dev), torch.empty(cnt, device=dev)
    ctx.gather(T0, idx, t0s)
    ctx.gather(TK, idx, tks)
    # K plain steps of the selected points (masked grid = the selected indices)
    after = [x.clone() for x in before]
    sub = dataclasses.replace(wl.grid, index=None)
    ctx.fused_scan_steps(wl.scan, sub, t_s, dtp, K, K, *after, z_top=L.z_top,
                         index=idx.to(torch.int32))
    big = [x.clone() for x in before]
    ctx.step(t0s, tks, K * dtp, *big)
    X = torch.stack([t0s, tks, torch.full_like(t0s, math.log(dtp)), before[0], before[1], before[2]], 1)
    Y = torch.stack([after[1] - big[1], after[2] - big[2], after[0] - big[0]], 1)
    return X, Y


def ramp_transitions(ctx, n, K=8, T_range=(600.0, 820.0), dT=40.0, dts=(1e-3, 4e-3, 16e-3), seed=0):
    """Transitions of a cool-down regime: over a block of K steps the
    temperature is linear in time from T0 to TK, both inside the network's
    cold band; states are seeded random solid states.  The target is the
    difference between K plain steps (``mstruct_step`` per sub-step) and one
    explicit step of K dt.  Returns X [n, 6], Y [n, 3] (float32, GPU)."""
    import torch
    dev = torch.device("cuda")
    rng = np.random.default_rng(seed)
    T0 = rng.uniform(T_range[0], T_range[1], n)
    TK = np.clip(T0 + rng.uniform(-dT, dT, n), T_range[0], T_range[1])
    dt = np.asarray(dts, np.float64)[rng.integers(0, len(dts), n)]
    am = rng.uniform(0.0, 0.9, n)
    am[rng.random(n) < 0.25] = 0.0
    a_s = rng.uniform(0.0, 1.0, n) * (0.9 - am)
    beta = 1.0 - a_s - am
    X = torch.empty(n, 6, device=dev)
    Y = torch.empty(n, 3, device=dev)
    f32 = lambda v: torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(dev)
    for d in dts:
        sel = np.nonzero(dt == d)[0]
        if sel.size == 0:
            continue
        t0, tk = T0[sel], TK[sel]
        start = [f32(v[sel]) for v in (beta, a_s, am)]
        small = [x.clone() for x in start]
        for s in range(K):
            ctx.step(f32(t0 + (tk - t0) * s / K), f32(t0 + (tk - t0) * (s + 1) / K), float(d), *small)
        big = [x.clone() for x in start]
        ctx.step(f32(t0), f32(tk), float(d) * K, *big)
        it = torch.from_numpy(sel).to(dev)
        X[it] = torch.stack([f32(t0), f32(tk), torch.full_like(start[0], math.log(d)), *start], 1)
        Y[it] = torch.stack([small[1] - big[1], small[2] - big[2], small[0] - big[0]], 1)
    return X, Y


def corrections_only_delta(ctx, X, K):
    """Change of (alpha_s, alpha_m, beta) that the correction g at the block
    start and end temperatures alone gives, relative to one explicit step of
    K dt (the surrogate's base).  Returns [N, 3]."""
    import torch
    T0, TK, dt = X[:, 0].contiguous(), X[:, 1].contiguous(), torch.exp(X[:, 2])
    res = torch.empty(X.shape[0], 3, device=X.device)
    for d in torch.unique(dt):
        sel = torch.nonzero(dt == d).flatten()
        b, a, m = [X[sel, c].contiguous() for c in (3, 4, 5)]
        step = [b.clone(), a.clone(), m.clone()]
        ctx.step(T0[sel].contiguous(), TK[sel].contiguous(), float(d) * K, *step)
        cor = [b.clone(), a.clone(), m.clone()]
        ctx.correct(T0[sel].contiguous(), *cor)
        ctx.correct(TK[sel].contiguous(), *cor)
        res[sel] = torch.stack([cor[1] - step[1], cor[2] - step[2], cor[0] - step[0]], 1)
    return res


def fit(ctx, X, Y, K, epochs=6, batch=16384, lr=2e-3, seed=0, val_frac=0.05, log=None):
    """Normalise, initialise (seeded) and train with the library's kernels.
    Returns (Surrogate, report dict)."""
    import torch

    import workload
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    perm = torch.randperm(X.shape[0], generator=gen, device=X.device)
    nv = max(1, int(val_frac * X.shape[0]))
    Xv, Yv = X[perm[:nv]].contiguous(), Y[perm[:nv]].contiguous()
    Xt, Yt = X[perm[nv:]].contiguous(), Y[perm[nv:]].contiguous()
    in_mean = Xt.mean(0).double().cpu().numpy()
    in_scale = np.maximum(Xt.std(0).double().cpu().numpy(), 1e-6)
    out_scale = np.maximum(Yt.std(0).double().cpu().numpy(), 1e-12)
    sur = Surrogate(workload.mlp_init_params(seed), in_mean, in_scale, out_scale, K)
    sur.load_into(ctx)
    loss = torch.empty(1, device=X.device)
    nt = Xt.shape[0]
    steps = 0
    total = epochs * ((nt + batch - 1) // batch)
    for ep in range(epochs):
        order = torch.randperm(nt, generator=gen, device=X.device)
        for i in range(0, nt, batch):
            sel = order[i:i + batch]
            # cosine-decayed learning rate
            lr_i = lr * 0.5 * (1 + math.cos(math.pi * steps / total))
            ctx.mlp_train_step(Xt[sel].contiguous(), Yt[sel].contiguous(), max(lr_i, lr * 1e-3), loss)
            steps += 1
        if log:
            log(f"epoch {ep}: batch loss {loss.item():.4g}")
    sur.params = ctx.mlp_get_params()
    report = evaluate(ctx, sur, Xv, Yv)
    report.update({"train_samples": int(nt), "val_samples": int(nv), "epochs": epochs, "steps": steps})
    return sur, report


def evaluate(ctx, sur, Xv, Yv):
    """Errors in (alpha_s, alpha_m) of the block update against K plain steps
    on held-out transitions: one explicit step of K dt alone (the method
    without the network), the same plus the network (the surrogate), and the
    instantaneous corrections alone."""
    import torch
    sur.load_into(ctx)
    pred = torch.empty_like(Yv)
    ctx.mlp_forward(Xv, pred)
    cor = corrections_only_delta(ctx, Xv, sur.K)

    def stats(err):
        d = err[:, :2].double()
        return {"max": float(d.abs().max()), "rms": float(d.pow(2).mean().sqrt())}

    return {"one_big_step": stats(Yv), "one_big_step_plus_network": stats(Yv - pred),
            "corrections_only": stats(Yv - cor)}


def main(argv=None):
    """Generate transitions on the multi-layer block, train, report, save."""
    import argparse
    import json
    import time

    import torch

    import workload
    ap = argparse.ArgumentParser()
    ap.add_argument("--layers", type=int, default=10)
    ap.add_argument("--steps-per-layer", type=int, default=2000)
    ap.add_argument("--every", type=int, default=512)
    ap.add_argument("--per-pick", type=int, default=93200)  # 10 layers x 4 picks x 3 dt: ~10M transitions
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--K", type=int, default=8)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    wl = workload.truncated(workload.multilayer_block(), n_layers=args.layers, steps_per_layer=args.steps_per_layer)
    assert wl.grid.index is None
    ctx = ms.Context(0)
    t0 = time.perf_counter()
    X, Y = generate_transitions(ctx, wl, K=args.K, every=args.every, per_pick=args.per_pick)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sur, rep = fit(ctx, X, Y, args.K, epochs=args.epochs, log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    rep.update({"transitions": int(X.shape[0]), "generate_s": t1 - t0, "train_s": t2 - t1})
    sur.save(args.out)
    print(json.dumps(rep))
    ctx.close()


if __name__ == "__main__":
    main()
