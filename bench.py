"""Benchmark: microstructure point-updates/s on the 256x256x128 multi-layer
block (8.4M points, 10 layers of 30 um, 20,000 steps of 2 us), float32 on one
MI355X.

One benchmark step = one whole run of the workload from the initial state
through every layer (all 20,000 time steps; 150,077,440,000 active
point-updates) with the temperature evaluated from the scan inside the fused
kernel (K = 64 steps per launch).  `value` is the plain float32 path.  The
same JSON line carries the surrogate on the same workload, the unfused and
implicit steps, the cool-down workload, the 33.5M-point masked cantilever
with island scan (`c3`), the 67M-point island block at full length, plain
and surrogate side by side (`c5`), the oracle timed on the host cores
(`cpu_baseline`) and the paper's own CPU figures (`paper_cpu`).
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
# VALU issue ceiling in lane-ops: 256 CUs x 4 SIMDs x 2 wave64 VALU
# instructions per 4 cycles (a SIMD can issue two VALU instructions in one
# quad-cycle: SQ_ACTIVE_INST_VALU2) x 64 lanes x 2.4 GHz = 78.6 T lane-ops/s,
# the FP32 vector peak of 157.3 TFLOP/s at 2 FLOPs per FMA lane-op.  Measured
# on the calibration probes: unpacked v_fmamk_f32 chains 48.5 T, v_exp_f32
# 18.6 T (profiles/valu_probes_calibration.txt).
VALU_PEAK_TLANEOPS = FP32_VECTOR_PEAK_TFLOPS / 2
PEAK_DERIVATION = ("256 CUs x 4 SIMDs x 2 wave64 VALU instructions per quad-cycle (dual issue, "
                   "SQ_ACTIVE_INST_VALU2) x 64 lanes x 2.4 GHz = 78.65 T lane-ops/s = 157.3 TFLOP/s / 2")
K_FUSED = 64
K_C3 = 16  # the masked cantilever's configuration names K = 16
K_SURROGATE = 8
STEP_BYTES = 28  # plain step: reads alpha_s, alpha_m, T^n, T^{n+1}; writes beta, alpha_s, alpha_m (float32)

# The paper's own CPU figures (Sec. 4.1, hardware of Sec. 4).  A DoF is one
# phase fraction: 3 per point (Sec. 3.2: 24 B per DoF, 72 B per point).
PAPER_CPU = {
    "source": "Sec. 4.1 (explicit step on synthetic data layouts) and Sec. 4 (hardware); 3 DoF per point",
    "intel_node": {
        "hardware": "2x Intel Xeon Gold 6230 (40 cores, 2.1 GHz), DAXPY 162 GB/s, 2.5 TFLOP/s",
        "explicit_step_plateau": "above 6 GDoF/s, i.e. above 2.0e9 point-updates/s (FP64, AVX-512)",
        "explicit_step_plateau_point_updates_s": 2.0e9,
        "memory_bound_point_updates_s": 162e9 / 72.0,
    },
    "amd_node": {
        "hardware": "2x AMD EPYC 9354 (64 cores, 3.25 GHz), DAXPY 617 GB/s, 3.75 TFLOP/s",
        "memory_bound_point_updates_s": 617e9 / 72.0,
        "note": "derived here from 617 GB/s and 72 B per point; the paper prints no throughput for this node",
    },
}

# Per-kernel figures from rocprofv3 counter runs of this script (the profile
# files named below): executed VALU instructions x 64 per point-update
# (SQ_INSTS_VALU), the fraction of the dual-issue VALU capacity used
# (SQ_ACTIVE_INST_VALU / (2 x SIMDs x quad-cycles)), the fraction of
# quad-cycles with any VALU issue ((SQ_ACTIVE_INST_VALU - SQ_ACTIVE_INST_VALU2)
# / (SIMDs x quad-cycles)), and HBM bytes per dispatch (FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0: the factors a plain 1 GiB device copy reads on the same
# counters; the PLAIN path's persistent kernel runs once per chunk of
# launches of a call, the surrogate's slot kernel once per launch).  Each
# holds for the launch size K it was taken at; at another K the figures are
# reported null.
FUSED_PROFILE = {
    "file": "profiles/fused_plain_kernel_multilayer_block.txt", "K": 64,
    "valu_lane_ops_per_update": 8.765, "valu_issue": 0.370, "valu_busy": 0.530,
    # the persistent kernel with its list and still-flag passes, per dispatch (one per call)
    "traffic_bytes_per_dispatch": 139802356,
}
FUSED_PROFILE_EVERY_T = {"K": 64, "valu_lane_ops_per_update": 130.31, "valu_issue": 0.730,
                         "valu_busy": 0.927}
SURROGATE_PROFILE = {"file": "profiles/fused_surrogate_kernels_multilayer_block.txt", "K": 64,
                     8: {"valu_lane_ops_per_update": 3.809, "valu_issue": 0.253, "valu_busy": 0.392},
                     16: {"valu_lane_ops_per_update": 3.241, "valu_issue": 0.228, "valu_busy": 0.368}}
C3_PROFILE = {"file": "profiles/fused_plain_kernel_cantilever_islands.txt", "K": K_C3,
              "valu_lane_ops_per_update": 1.392, "valu_issue": 0.284, "valu_busy": 0.425,
              "traffic_bytes_per_dispatch": 2046456748}
C5_PROFILE = {"file": "profiles/fused_kernels_island_block.txt",
              "plain": {"K": K_FUSED, "kernel": "fused_plain_call_kernel<2> + chunk_list_kernel + still_flags_kernel",
                        "valu_lane_ops_per_update": 1.945, "valu_issue": 0.507, "valu_busy": 0.702,
                        "traffic_bytes": 721815966, "traffic_unit": "bytes/dispatch"},
              "surrogate": {"K": K_SURROGATE,
                            "kernel": "fused_surrogate_call_kernel<2> + surrogate_resume_call_kernel<2> + list passes",
                            "valu_lane_ops_per_update": 0.443, "valu_issue": 0.284, "valu_busy": 0.430,
                            "traffic_bytes": 721103344, "traffic_unit": "bytes/dispatch"}}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--K", type=int, default=K_FUSED)
    ap.add_argument("--sample", type=float, default=1e-2, help="oracle sample fraction (cpu_baseline, errors)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="no oracle runs (no errors either)")
    ap.add_argument("--no-stepwise", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-cooldown", action="store_true")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--only", choices=("c2", "c3", "c5", "steps", "cooldown"),
                    help="one part only, without the oracle (profiling runs): a workload, the unfused steps "
                         "(plain, implicit, float64, divergence layouts) or the cool-down workload")
    ap.add_argument("--threads", type=int, default=0, help="oracle threads (default: OpenMP's, all host cores)")
    ap.add_argument("--calibrate", action="store_true",
                    help="instead: the VALU probes (FMA, exp, both) and a 1 GiB device copy, timed, for the "
                         "counter calibration under rocprofv3")
    args = ap.parse_args()
    if args.only:
        args.no_cpu_baseline = True
        args.no_stepwise = args.only != "steps"
        args.no_cooldown = args.only != "cooldown"
        args.no_c3 = args.only != "c3"
        args.no_c5 = args.only != "c5"
        args.no_surrogate = args.only != "c2"
    return args


def _timer(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def call_launches(wl, K):
    """Fused launches of one run of a layered workload (one call per layer)."""
    return sum(math.ceil((L.step_end - L.step_begin) / K) for L in wl.layers)


FLAG_BUDGET = 256 << 20  # bytes of still flags per chunk of launches of a fused call


def call_chunks(wl, K):
    """Per call of a layered workload: (active points, waves, launches, chunks
    of launches).  A fused PLAIN call with wave flags runs one list pass and
    one persistent kernel per chunk of launches whose still flags fit in 256 MiB
    (1 byte per wave and launch)."""
    out = []
    for L in wl.layers:
        pts = wl.active_count(L.z_top) if wl.grid.index is None else wl.grid.n
        waves = (pts + 63) // 64
        nl = math.ceil((L.step_end - L.step_begin) / K)
        chunk = max(1, min(nl, FLAG_BUDGET // waves))
        out.append((wl.active_count(L.z_top), waves, nl, math.ceil(nl / chunk)))
    return out


def call_dispatches(wl, K):
    """Dispatches of the persistent PLAIN kernel in one run."""
    return sum(c[3] for c in call_chunks(wl, K))


def call_algorithmic_bytes(wl, K):
    """Bytes a fused PLAIN run must move at least: per call the state read
    once (8 B), beta written once (4 B) and the state written once (8 B, an
    upper bound: still and frozen waves write nothing) per active point, 4 B
    of index per point of an index list, and one byte of still flag per wave
    and launch."""
    idx = 4 if wl.grid.index is not None else 0
    return sum((20 + idx) * pts + waves * nl for pts, waves, nl, _ in call_chunks(wl, K))


def point_launches(wl, K):
    """Active points summed over the launches of one run."""
    return sum(wl.active_count(L.z_top) * math.ceil((L.step_end - L.step_begin) / K) for L in wl.layers)


def counted_run(torch, ms, ctx, wl, K, index=None):
    """One untimed run with the device-side wave counts on: the points whose
    state the fused launches read and wrote (waves that do not exit on their
    flags, waves that are not still), the waves by class, and the hot waves'
    sub-blocks that the surrogate's indicator would allow.  Results are the
    same bits as without the counts."""
    g = [torch.from_numpy(x).cuda() for x in workload.initial_state(wl.grid.n, np.float32)]
    ctx.set_option(ms.OPTION_COUNT_WAVES, 1)
    ctx.wave_counts(reset=True)
    try:
        ms.run_layers(ctx, wl, *g, K=K, index=index)
        c = ctx.wave_counts(reset=True)
    finally:
        ctx.set_option(ms.OPTION_COUNT_WAVES, 0)
    total = point_launches(wl, K)
    waves = c["still_waves"] + c["cold_waves"] + c["hot_waves"] + c["flagged_waves"]
    out = {"counts": c, "point_launches": total, "read_fraction": c["points_loaded"] / total,
           "written_fraction": c["points_stored"] / total,
           "wave_classes": {k: c[k] / waves for k in ("flagged_waves", "still_waves", "cold_waves", "hot_waves")},
           "algorithmic_bytes_per_dispatch": call_algorithmic_bytes(wl, K) / call_dispatches(wl, K),
           "bytes_rule": "per call: 8 B of state read, 8 B of state written (an upper bound) and 4 B of beta per "
                         "active point, 1 B of still flag per wave and launch"
                         + (", 4 B of index per point" if wl.grid.index is not None else "")
                         + "; per dispatch of the persistent kernel (one per chunk of launches)",
           "counts_note": "classes per wave and launch: a wave that is not still by its flags reads its state "
                          "from registers inside a call, from memory once per call"}
    if c["hot_subblocks"]:
        s = c["indicator_subblocks"] / c["hot_subblocks"]
        out["surrogate_share_of_hot_subblocks"] = s
    return out


def fused_roofline(kernel, prof, K, rate, avg_dispatch_s, counts):
    """The fused PLAIN path's roofline entry: VALU-bound.  achieved =
    point-updates per second over the timed region (live HIP-event time, the
    persistent kernel with its list and still-flag passes) x the profile's
    executed VALU lane-ops per update; traffic per dispatch of the persistent
    kernel (with its passes) from the profile's counters; algorithmic bytes
    per dispatch from the call sizes."""
    ok = prof["K"] == K
    ops = prof["valu_lane_ops_per_update"] if ok else None
    traffic = prof["traffic_bytes_per_dispatch"] if ok else None
    alg = counts["algorithmic_bytes_per_dispatch"] if counts else None
    r = {"kernel": kernel, "bound": "alu",
         "achieved": rate * ops / 1e12 if ops else None, "peak": VALU_PEAK_TLANEOPS, "unit": "Tlane-op/s",
         "frac": rate * ops / 1e12 / VALU_PEAK_TLANEOPS if ops else None,
         "frac_source": "live point-updates/s x the profile's VALU instructions per update (null: the profile "
                        "was taken at another K)",
         "measured_limit": "neither roofline is reached: the waves near the tracks (3 % of the wave-launches "
                           "on a layer scan) run chains of K dependent steps launch after launch, a few per "
                           "SIMD, and leave the VALU idle for part of the time (valu_busy_frac); HBM traffic is "
                           "under 1 % of 8 TB/s",
         "traffic": traffic, "traffic_unit": "bytes/dispatch",
         "algorithmic_bytes_per_dispatch": alg,
         "traffic_over_algorithmic": traffic / alg if traffic and alg else None,
         "hbm_GBs": alg / avg_dispatch_s / 1e9 if alg else None,
         "lane_ops_per_update": ops, "valu_issue_frac": prof.get("valu_issue") if ok else None,
         "valu_busy_frac": prof.get("valu_busy") if ok else None,
         "peak_derivation": PEAK_DERIVATION, "avg_dispatch_us": avg_dispatch_s * 1e6,
         "point_updates_per_s": rate, "profile": prof.get("file"), "profile_K": prof["K"]}
    return r


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; the multi-GPU path is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_2402_17580_amd as ms

    if args.calibrate:
        print(json.dumps(bench_calibrate(torch)))
        return
    ctx = ms.Context(0)
    result = {}
    states = {}
    wl = workload.multilayer_block()
    if args.only in (None, "c2"):
        result, states = bench_c2(torch, ms, ctx, args)
    else:
        result = {"metric": f"profiling run: {args.only} only", "value": None}
        if args.only == "steps":  # the state the plain run leaves, for the step kernels
            g = [torch.from_numpy(x).cuda() for x in workload.initial_state(wl.grid.n, np.float32)]
            ms.run_layers(ctx, wl, *g, K=K_FUSED)
            states = {"plain": g}
    if not args.no_stepwise:
        result["plain_step"] = bench_stepwise(torch, ms, ctx, wl, torch.device("cuda:0"))
        result["implicit_step"] = bench_implicit(torch, ms, ctx, wl, states["plain"])
        result["divergence"] = bench_divergence(torch, ctx, wl.grid.n)
        result["f64_step"] = bench_f64(torch, ms, ctx, wl, states["plain"])
    if not args.no_cooldown:
        result["cooldown"], states["cooldown"] = bench_cooldown(torch, ms, ctx)
    if not args.no_c3:
        result["c3"], states["c3"] = bench_c3(torch, ms, ctx, args)
    if not args.no_c5:
        result["c5"], states["c5"] = bench_c5(torch, ms, ctx, args)

    if not args.no_cpu_baseline:
        import oracle
        threads = args.threads or oracle.num_threads()
        base, st, idx = cpu_baseline(wl, args, threads)
        base["gpu_vs_oracle"] = result["value"] / base["value"]
        result["cpu_baseline"] = base
        result["errors_vs_oracle"] = errors(states["plain"], st, idx)
        for key in ("surrogate", "surrogate_k16"):
            if key in states:
                result[key]["errors_vs_oracle"] = errors(states[key], st, idx)
        if "cooldown" in states:
            pw = workload.multilayer_cooldown()
            cidx = workload.sample_indices(pw.grid.n, 1e-3, pw.seed)
            cst, _ = oracle.run_phases(pw, cidx, threads=threads)
            result["cooldown"]["errors_vs_oracle"] = errors(states["cooldown"], cst, cidx)
            result["cooldown"]["errors_sample"] = f"{cidx.size} seeded points (p=1e-3)"
        if "c3" in states:
            oracle_errors_layered(result["c3"], states["c3"], workload.cantilever_islands(), threads)
        if "c5" in states:
            oracle_errors_layered(result["c5"], states["c5"], workload.island_block(), threads)
    result["paper_cpu"] = PAPER_CPU
    print(json.dumps(result))
    ctx.close()


def bench_c2(torch, ms, ctx, args):
    """The metric workload: the plain fused path timed over `steps` whole
    runs, its launch certificates off for comparison, and the surrogate."""
    dev = torch.device("cuda:0")
    wl = workload.multilayer_block()
    n = wl.grid.n
    updates = wl.point_updates()
    launches = call_launches(wl, args.K)
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
        e0, e1 = _timer(torch)
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
    # average duration of one dispatch of the persistent kernel over the timed
    # region (with its list and still-flag passes, one each per dispatch, and
    # three state resets per step)
    dispatches = call_dispatches(wl, args.K)
    avg_dispatch_s = ms_total * 1e-3 / (args.steps * dispatches)
    rate = updates * args.steps / (ms_total * 1e-3)
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
    final = [x.clone() for x in (b, a, m)]
    counts = counted_run(torch, ms, ctx, wl, args.K)
    result["roofline"] = fused_roofline(
        f"fused_plain_call_kernel<{wl.scan.window}> (one per call) + chunk_list_kernel + still_flags_kernel",
        FUSED_PROFILE, args.K, rate, avg_dispatch_s, counts)
    result["roofline"]["dispatches_timed"] = args.steps * dispatches
    result["roofline"]["launches_of_K_steps_timed"] = args.steps * launches
    result["wave_counts"] = counts

    # the same run with every temperature evaluated (launch certificates
    # off): the same bits, for comparison
    ctx.set_option(ms.OPTION_SKIP_COLD_WAVES, 0)
    ms_all, _ = timed(ms.MODE_PLAIN, args.K)
    ctx.set_option(ms.OPTION_SKIP_COLD_WAVES, 1)
    avg_all_s = ms_all * 1e-3 / (args.steps * launches)
    ok = FUSED_PROFILE_EVERY_T["K"] == args.K
    ops_all = FUSED_PROFILE_EVERY_T["valu_lane_ops_per_update"] if ok else None
    rate_all = updates / launches / avg_all_s
    result["plain_every_temperature"] = {
        "value": updates * args.steps / (ms_all * 1e-3), "unit": "point-updates/s",
        "ms_per_step": ms_all / args.steps, "value_speedup": ms_all / ms_total,
        "bitwise_equal_to_value_run": all(bool(torch.equal(x, y)) for x, y in zip((b, a, m), final)),
        "roofline": {"kernel": f"fused_plain_kernel<{wl.scan.window}>", "bound": "alu",
                     "achieved": rate_all * ops_all / 1e12 if ops_all else None, "peak": VALU_PEAK_TLANEOPS,
                     "unit": "Tlane-op/s",
                     "frac": rate_all * ops_all / 1e12 / VALU_PEAK_TLANEOPS if ops_all else None,
                     "lane_ops_per_update": ops_all,
                     "valu_issue_frac": FUSED_PROFILE_EVERY_T["valu_issue"] if ok else None,
                     "valu_busy_frac": FUSED_PROFILE_EVERY_T["valu_busy"] if ok else None,
                     "avg_launch_us": avg_all_s * 1e6},
    }
    states = {"plain": final}
    if not args.no_surrogate:
        from paper_2402_17580_amd import surrogate as S
        for key, path in (("surrogate", S.DEFAULT_WEIGHTS), ("surrogate_k16", S.WEIGHTS_K16)):
            sur = S.Surrogate.load(path)
            sur.load_into(ctx)
            ms_sur, _ = timed(ms.MODE_SURROGATE, sur.K)
            states[key] = [x.clone() for x in (b, a, m)]
            sp = SURROGATE_PROFILE.get(sur.K) if SURROGATE_PROFILE["K"] == K_FUSED else None
            sur_rate = updates * args.steps / (ms_sur * 1e-3)
            result[key] = {
                "value": sur_rate, "unit": "point-updates/s",
                "ms_per_step": ms_sur / args.steps, "speedup_vs_plain": ms_total / ms_sur,
                "target_speedup_vs_plain": 3.0, "target_met": ms_total / ms_sur >= 3.0, "K": sur.K,
                "path": "mstruct_fused_scan_steps, SURROGATE: launches of 64 steps, a call's launches in one "
                        "persistent kernel; per block of K steps a wave takes one explicit step of K dt + BF16-MFMA "
                        "network correction where every point passes the indicator, K plain steps otherwise",
                "indicator": list(sur.indicator),
                "roofline": None if sp is None else {
                    "kernel": "fused_surrogate_call_kernel<2> + surrogate_resume_call_kernel<2> (one each per call) "
                              "+ chunk_list_kernel + still_flags_kernel",
                    "bound": "alu", "lane_ops_per_update": sp["valu_lane_ops_per_update"],
                    "achieved": sur_rate * sp["valu_lane_ops_per_update"] / 1e12, "peak": VALU_PEAK_TLANEOPS,
                    "unit": "Tlane-op/s", "frac": sur_rate * sp["valu_lane_ops_per_update"] / 1e12 / VALU_PEAK_TLANEOPS,
                    "valu_issue_frac": sp["valu_issue"], "valu_busy_frac": sp["valu_busy"],
                    "profile": SURROGATE_PROFILE["file"]},
            }
        if "surrogate_share_of_hot_subblocks" in counts:
            result["surrogate_ceiling"] = surrogate_ceiling(counts, ms_total, launches * args.steps)
    return result, states


def surrogate_ceiling(counts, ms_total, launches):
    """Bound on the surrogate's speedup over the plain path from the counted
    run: the plain launches' time is set by their hot waves, and the
    indicator lets the network replace a hot wave's sub-block of 8 steps only
    where every point of the wave passes it.  If every such sub-block cost
    nothing, and nothing else changed, the run would take (1 - s) of its
    time; at one temperature evaluation and one step per sub-block instead
    of eight, 1 - s (1 - 1/8)."""
    s = counts["surrogate_share_of_hot_subblocks"]
    return {"indicator_share_of_hot_subblocks": s, "speedup_bound_free": 1.0 / (1.0 - s) if s < 1 else None,
            "speedup_bound_one_step_per_subblock": 1.0 / (1.0 - s * 7.0 / 8.0),
            "hot_subblocks": counts["counts"]["hot_subblocks"],
            "indicator_subblocks": counts["counts"]["indicator_subblocks"]}


def bench_c3(torch, ms, ctx, args):
    """The masked cantilever (32.4M points of a 1024x512x128 box, seeded
    legs, 10 layers of 30 um, 5 mm islands, 50,000 steps of 2 us) on the
    plain fused path at K = 16: one warm-up run, one timed run, its roofline
    and its wave counts."""
    wl = workload.cantilever_islands()
    n = wl.grid.n
    idx = torch.from_numpy(wl.grid.index).cuda()
    upd = wl.point_updates()
    K = K_C3
    g = [torch.from_numpy(x).cuda() for x in workload.initial_state(n, np.float32)]
    ms.run_layers(ctx, wl, *g, K=K, index=idx)  # warm-up
    for dst, src in zip(g, workload.initial_state(n, np.float32)):
        dst.copy_(torch.from_numpy(src))
    torch.cuda.synchronize()
    e0, e1 = _timer(torch)
    e0.record()
    ms.run_layers(ctx, wl, *g, K=K, index=idx)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3
    dispatches = call_dispatches(wl, K)
    counts = counted_run(torch, ms, ctx, wl, K, index=idx)
    out = {"workload": "cantilever_islands", "points": n, "box": [wl.grid.nx, wl.grid.ny, wl.grid.nz],
           "layers": len(wl.layers), "time_steps": wl.n_steps, "active_point_updates": upd, "K": K,
           "point_order": "8 x 8 tiles of each plane (workload.tile_order)",
           "seconds": t, "value": upd / t, "unit": "point-updates/s",
           "roofline": fused_roofline("fused_plain_call_kernel<2> (index list) + chunk_list_kernel + still_flags_kernel",
                                      C3_PROFILE, K, upd / t, t / dispatches, counts),
           "wave_counts": counts}
    out["roofline"]["dispatches_timed"] = dispatches
    print(f"c3: {t:.2f} s", file=sys.stderr, flush=True)
    return out, g


def bench_c5(torch, ms, ctx, args):
    """The 64M-point island block at full length (512x512x256 points, 100
    layers of 20 um, 2000 steps of 2 us each): the plain fused path (K = 64)
    and the surrogate (K = 8 network) one after the other on the same GPU,
    each timed once."""
    from paper_2402_17580_amd import surrogate as S
    wl = workload.island_block()
    n = wl.grid.n
    upd = wl.point_updates()
    out = {"workload": "island_block", "points": n, "layers": len(wl.layers), "time_steps": wl.n_steps,
           "active_point_updates": upd}
    states = {}
    for key, mode, K in (("plain", ms.MODE_PLAIN, K_FUSED), ("surrogate", ms.MODE_SURROGATE, K_SURROGATE)):
        if mode == ms.MODE_SURROGATE:
            S.Surrogate.load(S.DEFAULT_WEIGHTS).load_into(ctx)
        g = [torch.from_numpy(x).cuda() for x in workload.initial_state(n, np.float32)]
        torch.cuda.synchronize()
        e0, e1 = _timer(torch)
        e0.record()
        ms.run_layers(ctx, wl, *g, K=K, mode=mode)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        prof = C5_PROFILE[key]
        rate = upd / t
        # both paths: one persistent kernel per chunk of launches (the
        # surrogate's launches are 64 steps too)
        units = call_dispatches(wl, 64)
        out[key] = {"seconds": t, "value": rate, "unit": "point-updates/s", "K": K,
                    "roofline": {"kernel": prof["kernel"], "bound": "alu", "peak": VALU_PEAK_TLANEOPS,
                                 "unit": "Tlane-op/s",
                                 "achieved": rate * prof["valu_lane_ops_per_update"] / 1e12,
                                 "frac": rate * prof["valu_lane_ops_per_update"] / 1e12 / VALU_PEAK_TLANEOPS,
                                 "lane_ops_per_update": prof["valu_lane_ops_per_update"],
                                 "valu_issue_frac": prof["valu_issue"], "valu_busy_frac": prof["valu_busy"],
                                 "traffic": prof["traffic_bytes"], "traffic_unit": prof["traffic_unit"],
                                 "hbm_GBs": prof["traffic_bytes"] * units / t / 1e9 if prof["traffic_bytes"] else None,
                                 "profile": C5_PROFILE["file"]}}
        print(f"c5 {key}: {t:.2f} s", file=sys.stderr, flush=True)
        states[key] = g
    out["surrogate"]["speedup_vs_plain"] = out["plain"]["seconds"] / out["surrogate"]["seconds"]
    return out, states


def oracle_errors_layered(entry, states, wl, threads):
    """Errors of the GPU state(s) on a seeded 0.1 % sample against the
    oracle, run ten layers per call with a progress line each."""
    import oracle
    idx = workload.sample_indices(wl.grid.n, 1e-3, wl.seed)
    t0 = time.perf_counter()
    st = None
    for first in range(0, len(wl.layers), 10):
        st = oracle.run_workload(wl, idx, state=st, threads=threads, layers=wl.layers[first:first + 10])
        print(f"oracle {wl.name}: {min(first + 10, len(wl.layers))} layers, {time.perf_counter() - t0:.0f} s",
              file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    entry["oracle"] = {"sample": f"{idx.size} seeded points (p=1e-3), all {wl.n_steps} steps", "seconds": el,
                       "threads": threads}
    if isinstance(states, dict):
        for key, g in states.items():
            entry[key]["errors_vs_oracle"] = errors(g, st, idx)
    else:
        entry["errors_vs_oracle"] = errors(states, st, idx)


def cpu_baseline(wl, args, threads):
    """The FP64 oracle on a seeded sample of the workload's points (all
    20,000 steps), timed on the host cores (OpenMP's thread count: all the
    cores the process may use, OMP_NUM_THREADS where it is set)."""
    import oracle
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
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
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
IMPLICIT_PROFILE = {"scan": 94.37, "cooldown": 370.37}


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
    cool-down in steps of 0.1 s, one run, in launches of 64 steps (258 ms per
    run at K = 16, 241 ms at 32, 234 ms at 64)."""
    pw = workload.multilayer_cooldown()
    n = pw.grid.n
    g = [torch.from_numpy(x).cuda() for x in workload.initial_state(n, np.float32)]
    ms.run_phases(ctx, pw, *g, K=K_FUSED)  # warm-up
    for dst, src in zip(g, workload.initial_state(n, np.float32)):
        dst.copy_(torch.from_numpy(src))
    ctx.implicit_unconverged(reset=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ms.run_phases(ctx, pw, *g, K=K_FUSED)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3
    upd = pw.point_updates()
    scan_upd = sum((pw.grid.nz - pw.grid.first_active_k(p.z_top)) * pw.grid.nx * pw.grid.ny * p.n_steps
                   for p in pw.phases if p.scheme == "explicit")
    return {"value": upd / t, "unit": "point-updates/s", "seconds": t, "point_updates": upd,
            "scan_point_updates": scan_upd, "simulated_s": pw.phases[-1].t0 + pw.phases[-1].dt * pw.phases[-1].n_steps,
            "calls": len(pw.phases), "unconverged_substeps": ctx.implicit_unconverged(),
            "path": "run_phases: fused PLAIN while scanning, fused IMPLICIT while cooling (K = 64)", "K": K_FUSED}, g


F64_STEP_BYTES = 56  # float64 step: reads alpha_s, alpha_m, T^n, T^{n+1}; writes beta, alpha_s, alpha_m


def bench_f64(torch, ms, ctx, wl, state):
    """The explicit step in float64 on all 8.4M points (state after the plain
    run, top-layer temperatures at 2 us apart), with the device math library,
    with exponent-bit exp2 / log2 of double accuracy, and with the paper's
    own exp / ln (Sec. 3.3, its fitted correction polynomials): HBM-bound at
    56 bytes per point."""
    n = wl.grid.n
    L = wl.layers[-1]
    Ta, Tb = torch.empty(n, device="cuda"), torch.empty(n, device="cuda")
    t = wl.t0(L) + 1000 * wl.dt
    ctx.temperature(wl.scan, wl.grid, t, Ta, z_top=L.z_top)
    ctx.temperature(wl.scan, wl.grid, t + wl.dt, Tb, z_top=L.z_top)
    Ta, Tb = Ta.double(), Tb.double()
    out = {"path": "mstruct_step_f64 on all points (state after the plain run, cast to float64)"}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for key, math_mode in (("library", ms.F64_LIBRARY), ("synth", ms.F64_SYNTH), ("paper", ms.F64_PAPER)):
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




def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None




def bench_calibrate(torch):
    """Launches of known work for reading the counters: the VALU probes of
    libmstruct_probe.so (8 independent chains per lane of v_fma_f32, of
    v_exp_f32, or 16 of both interleaved; a known number of wave64 VALU
    instructions per launch) and a plain 1 GiB device copy (known bytes)."""
    import ctypes
    L = ctypes.CDLL(os.path.join(ROOT, "paper_2402_17580_amd", "libmstruct_probe.so"))
    L.probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.probe_valu_insts_per_wave.restype = ctypes.c_int64
    L.probe_valu_insts_per_wave.argtypes = [ctypes.c_int, ctypes.c_int]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks, iters, reps = 32 * cus, 20000, 5
    waves = blocks * 256 // 64
    out = torch.empty(blocks * 256, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {"compute_units": cus, "blocks": blocks, "threads_per_block": 256, "iters": iters}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for kind, name in ((0, "fma"), (1, "exp"), (2, "fma_exp")):
        assert L.probe_valu(kind, iters, blocks, ctypes.c_void_p(out.data_ptr()), st) == 0
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            L.probe_valu(kind, iters, blocks, ctypes.c_void_p(out.data_ptr()), st)
        e1.record()
        torch.cuda.synchronize()
        avg = e0.elapsed_time(e1) * 1e-3 / reps
        insts = waves * L.probe_valu_insts_per_wave(kind, iters)
        res[name] = {"avg_launch_us": avg * 1e6, "wave_insts_per_launch": insts,
                     "T_lane_ops_per_s": insts * 64 / avg / 1e12}
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    avg = e0.elapsed_time(e1) * 1e-3 / reps
    res["copy"] = {"bytes_read": src.numel() * 4, "bytes_written": src.numel() * 4, "avg_launch_us": avg * 1e6,
                   "GBs": 2 * src.numel() * 4 / avg / 1e9}
    return res




def errors(state, st, idx):
    out = {}
    for name, g, o in zip(("beta", "alpha_s", "alpha_m"), state, (st.beta, st.alpha_s, st.alpha_m)):
        d = np.abs(g.double().cpu().numpy()[idx] - o)
        out[name] = {"max": float(d.max()), "rms": float(np.sqrt(np.mean(d * d)))}
    return out



if __name__ == "__main__":
    main()
