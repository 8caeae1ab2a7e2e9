"""Benchmark: microstructure point-updates/s on the 256x256x128 multi-layer
block (8.4M points, 10 layers of 30 um, 20,000 steps of 2 us), float32 on one
MI355X.

One benchmark step = one whole run of the workload from the initial state
through every layer (all 20,000 time steps; 150,077,440,000 active
point-updates) with the temperature evaluated from the scan inside the fused
kernel (K = 64 steps per launch).  `value` is the plain float32 path; the
`surrogate` entries are the same workload with the learned surrogate (K = 8
and K = 16 networks).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workload  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
# VALU ceiling in lane-ops: the FP32 vector peak counts 2 FLOPs per FMA lane-op,
# i.e. 256 CUs x 128 lane-ops/clock x 2.4 GHz = 78.6 T lane-ops/s
VALU_PEAK_TLANEOPS = FP32_VECTOR_PEAK_TFLOPS / 2
K_FUSED = 64
K_SURROGATE = 8
STEP_BYTES = 28  # plain step: reads alpha_s, alpha_m, T^n, T^{n+1}; writes beta, alpha_s, alpha_m (float32)


def fused_bytes_per_launch(wl, K, read, written):
    """Algorithmic HBM bytes per fused launch, averaged over the run: alpha_s,
    alpha_m are read (8 B) for the fraction `read` of the active points whose
    wave does not exit on its flags, and written (8 B) for the fraction
    `written` whose wave is not still; the last launch of each call (one per
    layer) also writes beta (4 B per active point)."""
    g = wl.grid
    pts = [(g.nz - g.first_active_k(L.z_top)) * g.nx * g.ny for L in wl.layers]
    launches = [math.ceil((L.step_end - L.step_begin) / K) for L in wl.layers]
    state = sum(n * p for n, p in zip(launches, pts)) * (8.0 * read + 8.0 * written)
    return (state + 4.0 * sum(pts)) / sum(launches)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--K", type=int, default=K_FUSED)
    ap.add_argument("--sample", type=float, default=1e-2, help="oracle sample fraction (cpu_baseline, errors)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stepwise", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-cooldown", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--island-block", action="store_true",
                    help="instead: the 512x512x256 island block (100 layers, 200,000 steps), plain K = 16 and "
                         "surrogate K = 8 side by side, errors on a 0.1 %% sample")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; the multi-GPU path is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_2402_17580_amd as ms

    if args.island_block:
        print(json.dumps(bench_island_block(torch, ms, args)))
        return
    dev = torch.device("cuda:0")
    wl = workload.multilayer_block()
    n = wl.grid.n
    updates = wl.point_updates()
    launches = sum(math.ceil((L.step_end - L.step_begin) / args.K) for L in wl.layers)
    ctx = ms.Context(0)
    init = [torch.from_numpy(x).to(dev) for x in workload.initial_state(n, np.float32)]
    b, a, m = [x.clone() for x in init]

    def reset():
        for dst, src in zip((b, a, m), init):
            dst.copy_(src)

    def timed(mode, K):
        def one_step():
            reset()
            ms.run_layers(ctx, wl, b, a, m, K=K, mode=mode)

        for _ in range(args.warmup):
            one_step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        w0 = time.perf_counter()
        for _ in range(args.steps):
            one_step()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), time.perf_counter() - w0

    ms_total, wall = timed(ms.MODE_PLAIN, args.K)
    ms_per_step = ms_total / args.steps
    value = updates * args.steps / (ms_total * 1e-3)
    # average duration of one fused launch over the timed region (the fused
    # kernel is the only kernel in it besides three state resets per step)
    avg_launch_s = ms_total * 1e-3 / (args.steps * launches)
    upd_per_launch = updates / launches
    bytes_per_launch = fused_bytes_per_launch(wl, args.K, FUSED_PROFILE["read_fraction"],
                                              FUSED_PROFILE["written_fraction"])

    result = {
        "metric": "microstructure point-updates/s @8.4M pts (256x256x128 block, 10 layers, 20k steps): FP32 plain",
        "value": value,
        "unit": "point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded scan, analytic moving-source temperature)",
        "config": {"workload": "multilayer_block", "grid": [256, 256, 128], "points": n, "layers": 10,
                   "time_steps": wl.n_steps, "dt_s": wl.dt, "active_point_updates": updates,
                   "K": args.K, "window": wl.scan.window, "path": "fused (mstruct_fused_scan_steps, PLAIN)"},
        "wall_s_timed": wall,
    }
    rate = upd_per_launch / avg_launch_s  # point-updates/s inside one launch
    ops = FUSED_PROFILE["valu_lane_ops_per_update"]
    result["roofline"] = {
        "kernel": f"fused_plain_kernel<{wl.scan.window}> (first launch of each call) + "
                  f"fused_plain_slots_kernel<{wl.scan.window}> (the others)",
        "bound": "alu",
        "achieved": rate * ops / 1e12,
        "peak": VALU_PEAK_TLANEOPS,
        "unit": "Tlane-op/s",
        "frac": rate * ops / 1e12 / VALU_PEAK_TLANEOPS,
        "traffic": FUSED_PROFILE["traffic_bytes_per_launch"] if args.K == K_FUSED else None,
        "traffic_unit": "bytes/launch",
        "algorithmic_bytes_per_launch": bytes_per_launch,
        "lane_ops_per_update": ops,
        "fp32_tflops": rate * FUSED_PROFILE["fp32_flops_per_update"] / 1e12,
        "fp32_tflops_peak": FP32_VECTOR_PEAK_TFLOPS,
        "hbm_GBs": bytes_per_launch / avg_launch_s / 1e9,
        "avg_launch_us": avg_launch_s * 1e6,
        "launches_timed": args.steps * launches,
    }
    final_state = [x.clone() for x in (b, a, m)]

    # the same run with every temperature evaluated (cold-wave certificate
    # off): the same bits, for comparison
    ctx.set_option(ms.OPTION_SKIP_COLD_WAVES, 0)
    ms_all, _ = timed(ms.MODE_PLAIN, args.K)
    ctx.set_option(ms.OPTION_SKIP_COLD_WAVES, 1)
    avg_all_s = ms_all * 1e-3 / (args.steps * launches)
    ops_all = FUSED_PROFILE_EVERY_T["valu_lane_ops_per_update"]
    result["plain_every_temperature"] = {
        "value": updates * args.steps / (ms_all * 1e-3), "unit": "point-updates/s",
        "ms_per_step": ms_all / args.steps, "value_speedup": ms_all / ms_total,
        "bitwise_equal_to_value_run": all(bool(torch.equal(x, y)) for x, y in zip((b, a, m), final_state)),
        "roofline": {"kernel": f"fused_plain_kernel<{wl.scan.window}>", "bound": "alu",
                     "achieved": upd_per_launch / avg_all_s * ops_all / 1e12, "peak": VALU_PEAK_TLANEOPS,
                     "unit": "Tlane-op/s", "frac": upd_per_launch / avg_all_s * ops_all / 1e12 / VALU_PEAK_TLANEOPS,
                     "lane_ops_per_update": ops_all, "avg_launch_us": avg_all_s * 1e6},
    }

    sur_states = {}
    if not args.no_surrogate:
        from paper_2402_17580_amd import surrogate as S
        for key, path in (("surrogate", S.DEFAULT_WEIGHTS), ("surrogate_k16", S.WEIGHTS_K16)):
            t_tr = 0.0
            if os.path.exists(path):
                sur = S.Surrogate.load(path)
            else:
                K_s = K_SURROGATE if key == "surrogate" else 16
                t0 = time.perf_counter()
                X, Y = S.generate_transitions(ctx, wl, K=K_s)
                sur, _ = S.fit(ctx, X, Y, K_s)
                t_tr = time.perf_counter() - t0
            sur.load_into(ctx)
            ms_sur, _ = timed(ms.MODE_SURROGATE, sur.K)
            sur_states[key] = [x.clone() for x in (b, a, m)]
            result[key] = {
                "value": updates * args.steps / (ms_sur * 1e-3), "unit": "point-updates/s",
                "ms_per_step": ms_sur / args.steps, "speedup_vs_plain": ms_total / ms_sur,
                "speedup_vs_plain_every_temperature": ms_all / ms_sur, "K": sur.K,
                "path": "mstruct_fused_scan_steps, SURROGATE: one explicit step of K dt + BF16-MFMA network "
                        "correction where the indicator allows, K plain steps elsewhere",
                "indicator": list(sur.indicator), "trained_in_bench_s": t_tr,
            }

    if not args.no_stepwise:
        result["plain_step"] = bench_stepwise(torch, ms, ctx, wl, dev)
        result["implicit_step"] = bench_implicit(torch, ms, ctx, wl, final_state)
        result["divergence"] = bench_divergence(torch, ctx, n)
        result["f64_step"] = bench_f64(torch, ms, ctx, wl, final_state)
    if not args.no_cooldown:
        result["cooldown"], cool_state = bench_cooldown(torch, ms, ctx)

    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_probe_bytes"] = {"read": src.numel() * 4, "write": src.numel() * 4}

    if not args.no_cpu_baseline:
        base, st, idx = cpu_baseline(wl, args)
        base["gpu_vs_oracle"] = result["value"] / base["value"]
        result["cpu_baseline"] = base
        result["errors_vs_oracle"] = errors(final_state, st, idx)
        for key, state in sur_states.items():
            result[key]["errors_vs_oracle"] = errors(state, st, idx)
        if not args.no_cooldown:
            import oracle
            pw = workload.multilayer_cooldown()
            cidx = workload.sample_indices(pw.grid.n, 1e-3, pw.seed)
            cst, _ = oracle.run_phases(pw, cidx, threads=args.threads or min(16, os.cpu_count() or 1))
            result["cooldown"]["errors_vs_oracle"] = errors(cool_state, cst, cidx)
            result["cooldown"]["errors_sample"] = f"{cidx.size} seeded points (p=1e-3)"

    print(json.dumps(result))
    ctx.close()


# Per-kernel figures of the fused kernel on this workload, from rocprofv3
# counter runs of this script (profiles/fused_plain_kernel_multilayer_block.txt):
# executed VALU instructions x 64 lanes and FP32 FLOPs per point-update, and
# HBM bytes per launch (FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0: the factors a
# plain 1 GiB device copy reads on the same counters), and the fractions of
# the points whose state the kernel reads (waves that do not exit on their
# flags) and writes (waves that are not still), at K = 64.
# the same kernel with every temperature evaluated (MSTRUCT_OPTION_SKIP_COLD_WAVES = 0)
FUSED_PROFILE_EVERY_T = {"valu_lane_ops_per_update": 128.07}
FUSED_PROFILE = {
    "valu_lane_ops_per_update": 10.26,
    "fp32_flops_per_update": 8.31,
    "traffic_bytes_per_launch": (3364.18 * 2.0 + 3476.92) * 1024,
    "read_fraction": 0.1148,
    "written_fraction": 0.0437,
}

def bench_stepwise(torch, ms, ctx, wl, dev):
    """The unfused path: temperature-field kernel + plain step kernel per time
    step (T arrays ping-pong in HBM), timed on the first 200 steps of the top
    layer; the step kernel alone is timed over T arrays already in HBM."""
    n = wl.grid.n
    L = wl.layers[-1]
    b, a, m = [torch.from_numpy(x).to(dev) for x in workload.initial_state(n, np.float32)]
    Ta, Tb = torch.empty(n, device=dev), torch.empty(n, device=dev)
    sub = workload.Layer(L.step_begin, L.step_begin + 200, L.z_top)
    ms.run_layers_stepwise(ctx, wl, b, a, m, Ta, Tb, layers=[workload.Layer(L.step_begin, L.step_begin + 20, L.z_top)])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ms.run_layers_stepwise(ctx, wl, b, a, m, Ta, Tb, layers=[sub])
    e1.record()
    torch.cuda.synchronize()
    ms_stepwise = e0.elapsed_time(e1)
    off = wl.grid.first_active_k(L.z_top) * wl.grid.nx * wl.grid.ny
    n_act = n - off
    rate_stepwise = n_act * 200 / (ms_stepwise * 1e-3)
    # the step kernel alone, 200 launches on resident T arrays
    reps = 200
    e0.record()
    for _ in range(reps):
        ctx.step(Ta[off:], Tb[off:], wl.dt, b[off:], a[off:], m[off:])
    e1.record()
    torch.cuda.synchronize()
    avg = e0.elapsed_time(e1) * 1e-3 / reps
    achieved = STEP_BYTES * n_act / avg / 1e9
    return {"value": rate_stepwise, "unit": "point-updates/s",
            "path": "mstruct_temperature + mstruct_step per time step (200 steps of the top layer)",
            "roofline": {"kernel": "step_kernel<true>", "bound": "hbm", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "bytes_per_update": STEP_BYTES, "avg_launch_us": avg * 1e6,
                         "point_updates_per_s": n_act / avg}}


# Per-point VALU lane-ops of the implicit step kernel on the two regimes timed
# below, from rocprofv3 counter runs of this script (SQ_INSTS_VALU x 64 / points)
IMPLICIT_PROFILE = {"scan": 96.8, "cooldown": 385.8}


def bench_implicit(torch, ms, ctx, wl, state):
    """The implicit step (mstruct_step_implicit) on all 8.4M points, starting
    from the state the plain run leaves: (a) a scan step of 2 us with the
    temperature arrays of the top layer, (b) a cool-down step of 0.1 s
    (ten substeps of 0.01 s) with T relaxing towards 300 K.  Each launch moves
    28 bytes per point, like the explicit step."""
    n = wl.grid.n
    L = wl.layers[-1]
    b, a, m = [x.clone() for x in state]
    Ta, Tb = torch.empty(n, device="cuda"), torch.empty(n, device="cuda")
    t = wl.t0(L) + 1000 * wl.dt
    ctx.temperature(wl.scan, wl.grid, t, Ta, z_top=L.z_top)
    ctx.temperature(wl.scan, wl.grid, t + wl.dt, Tb, z_top=L.z_top)
    Tc = 300.0 + (Ta - 300.0) * math.exp(-0.05)
    unc = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = {"path": "mstruct_step_implicit on all points of the block (state after the plain run)"}
    for key, T1, dt, reps in (("scan", Tb, wl.dt, 100), ("cooldown", Tc, 0.1, 20)):
        ctx.step_implicit(Ta, T1, dt, b, a, m, unconverged=unc)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ctx.step_implicit(Ta, T1, dt, b, a, m, unconverged=unc)
        e1.record()
        torch.cuda.synchronize()
        avg = e0.elapsed_time(e1) * 1e-3 / reps
        gbs = STEP_BYTES * n / avg / 1e9
        entry = {"dt_s": dt, "substeps": max(1, math.ceil(dt / 0.01 * (1 - 1e-12))), "avg_launch_us": avg * 1e6,
                 "point_updates_per_s": n / avg, "hbm_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
        ops = IMPLICIT_PROFILE[key]
        if ops is not None:
            entry["lane_ops_per_point"] = ops
            entry["valu_frac"] = n * ops / avg / 1e12 / VALU_PEAK_TLANEOPS
        out[key] = entry
    out["unconverged_substeps"] = int(unc.item())
    return out


def bench_cooldown(torch, ms, ctx):
    """The multi-layer block with the paper's inter-layer cool-down (each
    layer: 2000 scan steps of 2 us, explicit; then 1 s of cool-down on the
    doubling schedule, implicit with 0.01 s substeps) and the final 100 s
    cool-down in steps of 0.1 s, one run."""
    pw = workload.multilayer_cooldown()
    n = pw.grid.n
    g = [torch.from_numpy(x).cuda() for x in workload.initial_state(n, np.float32)]
    ms.run_phases(ctx, pw, *g)  # warm-up
    for dst, src in zip(g, workload.initial_state(n, np.float32)):
        dst.copy_(torch.from_numpy(src))
    ctx.implicit_unconverged(reset=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ms.run_phases(ctx, pw, *g)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3
    upd = pw.point_updates()
    scan_upd = sum((pw.grid.nz - pw.grid.first_active_k(p.z_top)) * pw.grid.nx * pw.grid.ny * p.n_steps
                   for p in pw.phases if p.scheme == "explicit")
    return {"value": upd / t, "unit": "point-updates/s", "seconds": t, "point_updates": upd,
            "scan_point_updates": scan_upd, "simulated_s": pw.phases[-1].t0 + pw.phases[-1].dt * pw.phases[-1].n_steps,
            "calls": len(pw.phases), "unconverged_substeps": ctx.implicit_unconverged(),
            "path": "run_phases: fused PLAIN while scanning, fused IMPLICIT while cooling (K = 16)"}, g


F64_STEP_BYTES = 56  # float64 step: reads alpha_s, alpha_m, T^n, T^{n+1}; writes beta, alpha_s, alpha_m


def bench_f64(torch, ms, ctx, wl, state):
    """The explicit step in float64 on all 8.4M points (state after the plain
    run, top-layer temperatures at 2 us apart), with the device math library
    and with exponent-bit exp2 / log2: HBM-bound at 56 bytes per point."""
    n = wl.grid.n
    L = wl.layers[-1]
    Ta, Tb = torch.empty(n, device="cuda"), torch.empty(n, device="cuda")
    t = wl.t0(L) + 1000 * wl.dt
    ctx.temperature(wl.scan, wl.grid, t, Ta, z_top=L.z_top)
    ctx.temperature(wl.scan, wl.grid, t + wl.dt, Tb, z_top=L.z_top)
    Ta, Tb = Ta.double(), Tb.double()
    out = {"path": "mstruct_step_f64 on all points (state after the plain run, cast to float64)"}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for key, math_mode in (("library", ms.F64_LIBRARY), ("synth", ms.F64_SYNTH)):
        b, a, m = [x.double() for x in state]
        ctx.step_f64(Ta, Tb, wl.dt, b, a, m, math=math_mode)
        torch.cuda.synchronize()
        reps = 100
        e0.record()
        for _ in range(reps):
            ctx.step_f64(Ta, Tb, wl.dt, b, a, m, math=math_mode)
        e1.record()
        torch.cuda.synchronize()
        avg = e0.elapsed_time(e1) * 1e-3 / reps
        gbs = F64_STEP_BYTES * n / avg / 1e9
        out[key] = {"avg_launch_us": avg * 1e6, "point_updates_per_s": n / avg, "hbm_GBs": gbs,
                    "hbm_frac": gbs / HBM_PEAK_GBS}
    return out


def bench_divergence(torch, ctx, n):
    """Cost of branch divergence (the paper's synthetic layouts, Sec. 4.1):
    points of two kinds that take different branches of the update, laid out
    alternating, in blocks of 10, 64 (one wave) and 100, or all of one kind.
    Kind A: a diffusive state at 1050-1150 K (the three rate laws); kind B: pure
    beta at 1000 K (the closed-form start of diffusion).  Explicit
    (mstruct_step, HBM-bound) and implicit (mstruct_step_implicit, dt = 1 ms)
    steps on n points; point-updates/s per layout."""
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    idx = torch.arange(n, device="cuda")
    TA0 = 1050.0 + 100.0 * torch.rand(n, device="cuda", generator=g)
    TA1 = TA0 + 2.0
    aA = 0.2 + 0.3 * torch.rand(n, device="cuda", generator=g)
    mA = 0.1 * torch.rand(n, device="cuda", generator=g)
    layouts = {"uniform_A": torch.zeros(n, dtype=torch.bool, device="cuda"),
               "uniform_B": torch.ones(n, dtype=torch.bool, device="cuda"),
               "alternating": (idx % 2) == 1, "blocks_10": ((idx // 10) % 2) == 1,
               "blocks_64": ((idx // 64) % 2) == 1, "blocks_100": ((idx // 100) % 2) == 1}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"points": n, "kinds": "A: diffusive state at 1050-1150 K; B: pure beta at 1000 K (start-up)"}
    for name, kb in layouts.items():
        Tp = torch.where(kb, torch.full_like(TA0, 1000.0), TA0)
        Tn = torch.where(kb, torch.full_like(TA0, 1000.0), TA1)
        a0 = torch.where(kb, torch.zeros_like(aA), aA)
        m0 = torch.where(kb, torch.zeros_like(mA), mA)
        b0 = 1.0 - a0 - m0
        entry = {}
        for scheme, dt, reps in (("explicit", 2e-6, 50), ("implicit", 1e-3, 50)):
            b, a, m = b0.clone(), a0.clone(), m0.clone()
            call = ctx.step if scheme == "explicit" else ctx.step_implicit
            call(Tp, Tn, dt, b, a, m)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                b.copy_(b0)
                a.copy_(a0)
                m.copy_(m0)
            e1.record()
            torch.cuda.synchronize()
            copies = e0.elapsed_time(e1)
            e0.record()
            for _ in range(reps):
                b.copy_(b0)
                a.copy_(a0)
                m.copy_(m0)
                call(Tp, Tn, dt, b, a, m)
            e1.record()
            torch.cuda.synchronize()
            avg = (e0.elapsed_time(e1) - copies) * 1e-3 / reps
            entry[scheme] = {"point_updates_per_s": n / avg, "avg_launch_us": avg * 1e6}
        out[name] = entry
    return out


def cpu_baseline(wl, args):
    """The FP64 oracle on a seeded sample of the workload's points (all
    20,000 steps), timed on the host cores."""
    import oracle
    threads = args.threads or min(16, os.cpu_count() or 1)
    idx = workload.sample_indices(wl.grid.n, args.sample, wl.seed)
    xyz = wl.grid.coords(idx)
    upd = sum(int(np.count_nonzero(xyz[:, 2] <= L.z_top + 1e-3 * wl.grid.h)) * (L.step_end - L.step_begin)
              for L in wl.layers)
    t0 = time.perf_counter()
    st = oracle.run_workload(wl, idx, threads=threads)
    el = time.perf_counter() - t0
    base = {"value": upd / el, "unit": "point-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{idx.size} seeded points (p={args.sample}) x all 20,000 steps "
                      f"({upd} point-updates, FP64, {el:.1f} s)",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}
    # one core, on a 32 times smaller sample
    idx1 = workload.sample_indices(wl.grid.n, args.sample / 32, wl.seed + 1)
    xyz1 = wl.grid.coords(idx1)
    upd1 = sum(int(np.count_nonzero(xyz1[:, 2] <= L.z_top + 1e-3 * wl.grid.h)) * (L.step_end - L.step_begin)
               for L in wl.layers)
    t0 = time.perf_counter()
    oracle.run_workload(wl, idx1, threads=1)
    el1 = time.perf_counter() - t0
    base["single_core"] = {"value": upd1 / el1, "sample": f"{idx1.size} seeded points x all 20,000 steps "
                                                          f"({upd1} point-updates, {el1:.1f} s)"}
    return base, st, idx


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_island_block(torch, ms, args):
    """The 64M-point island block at full length (512x512x256 points, 100
    layers of 20 um, 2000 steps of 2 us each): the plain fused path (K = 16)
    and the surrogate (K = 8 network) one after the other on the same GPU,
    each timed once, and both against the oracle on a seeded 0.1 % sample."""
    import oracle
    from paper_2402_17580_amd import surrogate as S
    wl = workload.island_block()
    n = wl.grid.n
    upd = wl.point_updates()
    ctx = ms.Context(0)
    out = {"workload": "island_block", "points": n, "layers": len(wl.layers), "time_steps": wl.n_steps,
           "active_point_updates": upd}
    states = {}
    for key, mode, K in (("plain", ms.MODE_PLAIN, 16), ("surrogate", ms.MODE_SURROGATE, 8)):
        if mode == ms.MODE_SURROGATE:
            sur = S.Surrogate.load(S.DEFAULT_WEIGHTS)
            sur.load_into(ctx)
        g = [torch.from_numpy(x).cuda() for x in workload.initial_state(n, np.float32)]
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ms.run_layers(ctx, wl, *g, K=K, mode=mode)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        out[key] = {"seconds": t, "point_updates_per_s": upd / t, "K": K}
        print(f"island block {key}: {t:.2f} s", file=sys.stderr, flush=True)
        states[key] = g
    out["surrogate"]["speedup_vs_plain"] = out["plain"]["seconds"] / out["surrogate"]["seconds"]
    idx = workload.sample_indices(n, 1e-3, wl.seed)
    t0 = time.perf_counter()
    threads = args.threads or min(16, os.cpu_count() or 1)
    st = None
    for first in range(0, len(wl.layers), 10):  # ten layers per call, with a progress line each
        st = oracle.run_workload(wl, idx, state=st, threads=threads, layers=wl.layers[first:first + 10])
        print(f"oracle: {first + 10} layers, {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    out["oracle"] = {"sample": f"{idx.size} seeded points (p=1e-3), all 200,000 steps", "seconds": el,
                     "threads": threads}
    for key, g in states.items():
        out[key]["errors_vs_oracle"] = errors(g, st, idx)
    ctx.close()
    return out


def errors(state, st, idx):
    out = {}
    for name, g, o in zip(("beta", "alpha_s", "alpha_m"), state, (st.beta, st.alpha_s, st.alpha_m)):
        d = np.abs(g.double().cpu().numpy()[idx] - o)
        out[name] = {"max": float(d.max()), "rms": float(np.sqrt(np.mean(d * d)))}
    return out


if __name__ == "__main__":
    main()
