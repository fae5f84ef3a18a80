"""Throughput of the all-pairs Oseen dumbbell step on one MI355X.

A step is one RK4 step of the whole hot path: four stages of spring forces,
the O(N^2) Oseen pair sum and the RK4 update, for S = 2048 dumbbells
(N = 4096 spheres) in a cube of side 240 (seed 0, a = eta = k = 1, ell = 4,
lambda = 1, T = 100, dt = 0.01), FP32 pair arithmetic with compensated
accumulation and FP64 state. The inputs are resident on the device before
the timed region starts. Prints one JSON line. `--workload` selects another
of the seeded workloads (the 512-sphere suspension, the 512-system ensemble,
the 65536-sphere suspension with steric repulsion) for profiles; N = 4096 is
the default and the measured configuration.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_FP64_TFLOPS = 78.6       # MI355X published FP64 vector peak
FLOPS_PER_PAIR = 28           # algorithmic flops of one ordered pair term (Oseen)
FLOPS_PER_PAIR_RPY = 34       # with the Rotne-Prager-Yamakawa-Mazur correction

# HBM bytes per pair-kernel launch from two rocprofv3 --pmc runs of
# `bench.py --counter-probe` (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch),
# each scaled by what the counter reads for a plain 256 MiB device copy.
# Valid only for the kernel source and launch shape they were taken with.
COUNTED = {
    "workload": "n4096",
    "source_sha256": "c9a2be618902a28e62734fc84f63095f761e81517385eed2fad1c330ae39f8eb",
    "launch": {"ipl": 1, "jchunk": 256, "wg": 256, "wj": 4, "posmode": 2, "fused": 3},
    "fetch_kib": 645.73, "fetch_scale": 262144.0 / 131088.5,
    "write_kib": 288.05, "write_scale": 262144.0 / 262144.0,
}


# the kernel that a launch of each form runs (the one bracketed by events)
KERNEL_NAMES = {0: "k_pairs_f32c", 1: "k_stage_fused (pair sum and stage update)",
                2: "k_stage_wide (pair sum and stage update, 64 targets per work-group)",
                3: "k_stage_stream (pair sum and stage update, sources streamed per wave)",
                4: "k_resident (every stage of a run of steps, one work-group per system)"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_steps(sim, steps, warmup):
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    sim.step(steps)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / 1e3, wall


def cpu_baseline(w, sizes, budget_s):
    """The oracle on the host cores: RK4 steps of the same workload."""
    from oracle import adref
    adref.build(force=False)
    p = w.params
    N = w.X.shape[0]
    Nb = 2.0 * np.asarray(sizes, dtype=np.float64)
    t = time.perf_counter()
    X, _, _, _ = adref.run(p, w.X, w.phi, 1, S_per_sys=sizes)
    one = time.perf_counter() - t
    n = max(1, int(budget_s / max(one, 1e-6)) - 1)
    t = time.perf_counter()
    adref.run(p, X, w.phi, n, step0=1, S_per_sys=sizes)
    dt = time.perf_counter() - t
    pairs_per_step = 4.0 * float((Nb * (Nb - 1)).sum())
    cores = adref.max_threads()
    out = {"value": pairs_per_step * n / dt, "unit": "pair interactions/s", "cores": cores,
           "kind": "oracle",
           "sample": f"{n} RK4 steps of the {N}-sphere workload ({dt:.1f} s), FP64, OpenMP over target spheres",
           "sphere_steps_per_s": N * n / dt, "cpu_model": cpu_model()}
    # the same on one core, for a few seconds
    adref.set_threads(1)
    try:
        t = time.perf_counter()
        adref.run(p, X, w.phi, 1, step0=1, S_per_sys=sizes)
        one = time.perf_counter() - t
        n1 = max(1, int(0.2 * budget_s / max(one, 1e-6)))
        t = time.perf_counter()
        adref.run(p, X, w.phi, n1, step0=1, S_per_sys=sizes)
        dt1 = time.perf_counter() - t
    finally:
        adref.set_threads(cores)
    out["one_core"] = {"value": pairs_per_step * n1 / dt1, "sample": f"{n1} RK4 steps ({dt1:.1f} s)"}
    return out


# VALU instructions per loop trip of 8 terms in the issue-rate probe, from the
# gfx950 assembly of k_valu_rate (8 terms plus the target's step; with hi/lo
# positions the lo differences and the lo step as well; 8 FMAs for kind 1)
PROBE_VALU_PER_TRIP = {0: 147, 1: 8, 2: 189, 3: 147}
PROBE_KINDS = {0: "Oseen pair term, single-float positions", 1: "independent FMA chains",
               2: "Oseen pair term, hi/lo positions",
               3: "Oseen pair term, single-float positions, four accumulators"}


def calibrate(iters: int = 4096):
    """Issue rate of the pair term's own instruction mix (operands in
    registers, no memory traffic) at 1, 2, 4 and 8 waves per SIMD, and the
    shader clock under the load, one JSON line per case."""
    import torch
    import paper_1004_1932_amd as P
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    out = []
    for kind in (0, 3, 2, 1):
        for wps in (1, 2, 4, 8):
            blocks = cus * wps  # 256-thread groups: one wave per SIMD each
            sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
            clk = torch.zeros(2, dtype=torch.int64, device="cuda")
            P.ad_valu_probe(kind, blocks, 64, sink, clk)  # warm-up
            times = []
            for _ in range(5):
                clk.zero_()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                P.ad_valu_probe(kind, blocks, iters, sink, clk)
                b.record()
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b) * 1e-3)
            t = sorted(times)[len(times) // 2]
            cyc_max, _ = (int(v) for v in clk.cpu())
            # the longest-lived work-group spans about the whole kernel: its
            # life in shader cycles over the event-timed duration is the clock
            ghz = cyc_max / t / 1e9
            trips = blocks * 256.0 * iters
            lane_instr = trips * PROBE_VALU_PER_TRIP[kind] / t
            line = {"calibrate": PROBE_KINDS[kind], "kind": kind, "waves_per_simd": wps, "blocks": blocks,
                    "seconds": t, "shader_clock_GHz": ghz, "valu_lane_instr_per_s": lane_instr,
                    "valu_instr_per_cu_per_clock": lane_instr / 64.0 / cus / (ghz * 1e9),
                    "cus": cus}
            if kind != 1:
                line["pair_terms_per_s"] = trips * 8 / t
                line["tflops_at_28_per_term"] = trips * 8 * 28 / t / 1e12
            else:
                line["fma_tflops"] = trips * 8 * 2 / t / 1e12
            print(json.dumps(line), flush=True)
            out.append(line)
    return out


def stroke_averaged_timing(steps: int = 2000):
    """The stroke-averaged equations (Sec. III) on the GPU: one checkerboard
    lattice of x^3 dumbbells at spacing 10 ell with the Fig. 1 parameters,
    RK4 steps of T/20, for x = 5, 7, 9 (the paper's arrays) and 16 (4096
    dumbbells); one JSON line per size (microseconds per RK4 step, pair
    evaluations 4 S (S - 1) per step per second)."""
    import torch
    import paper_1004_1932_amd as P
    from workload import fig1_params, lattice_array
    p = fig1_params(0.2, 5000)
    for x in (5, 7, 9, 16):
        R, N, phi = lattice_array(x, 10 * p.ell, 3, "checkerboard")
        sa = P.StrokeAveraged(p, R, N, phi)
        assert sa.run(p.T / 20, 20) == 0  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        assert sa.run(p.T / 20, steps) == 0
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        S = len(R)
        print(json.dumps({"stroke_averaged": True, "dumbbells": S, "us_per_step": dt / steps * 1e6,
                          "pair_evaluations_per_s": 4 * S * (S - 1) * steps / dt}), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


DESCRIPTIONS = {
    "n16": "suspension of S=8 active dumbbells (N=16 spheres), cube side 40, RK4 dt=0.01, Oseen, "
           "FP32-compensated pair sum, FP64 state",
    "n4096": "suspension of S=2048 active dumbbells (N=4096 spheres), cube side 240, RK4 dt=0.01, Oseen, "
             "FP32-compensated pair sum, FP64 state",
    "n512": "suspension of S=256 active dumbbells (N=512 spheres), cube side 120, RK4 dt=0.01, Oseen, "
            "FP32-compensated pair sum, FP64 state",
    "ens512": "ensemble of 512 suspensions, S uniform in [16, 400] (221,234 spheres in all), density 0.02, "
              "RK4 dt=0.01, Oseen, FP32-compensated pair sum, FP64 state",
    "n65536": "suspension of S=32768 active dumbbells (N=65536 spheres), cube side 800, steric repulsion "
              "100 (2a - r), RK4 dt=0.01, Oseen, FP32-compensated pair sum, FP64 state",
}


def counted_traffic(launch):
    """Counter-derived HBM bytes per launch, or None once the kernel source
    or the launch shape differs from the counted one."""
    import hashlib
    src = os.path.join(ROOT, "paper_1004_1932_amd", "csrc", "ad_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if sha != COUNTED["source_sha256"] or dict(launch) != COUNTED["launch"]:
        return None
    kib = COUNTED["fetch_kib"] * COUNTED["fetch_scale"] + COUNTED["write_kib"] * COUNTED["write_scale"]
    return kib * 1024.0


def workload_name(name: str) -> str:
    """A preset name, arrays:x:W (W checkerboard x^3 lattices, one ensemble)
    or single:N (one suspension of N spheres at the density of the 4096-sphere
    one)."""
    if (name in DESCRIPTIONS or re.fullmatch(r"arrays:[1-9][0-9]*:[1-9][0-9]*", name)
            or re.fullmatch(r"single:[1-9][0-9]*", name)):
        return name
    raise argparse.ArgumentTypeError(f"{name!r}: one of {sorted(DESCRIPTIONS)}, arrays:x:W or single:N")


def describe(name: str) -> str:
    if name in DESCRIPTIONS:
        return DESCRIPTIONS[name]
    if name.startswith("single:"):
        N = int(name.split(":")[1])
        return (f"suspension of S={N // 2} active dumbbells (N={N} spheres) at the density of the 4096-sphere "
                f"one, RK4 dt=0.01, Oseen, FP32-compensated pair sum, FP64 state")
    _, x, W = name.split(":")
    return (f"ensemble of {W} lattices of {x}^3 active dumbbells, spacing 10 ell, checkerboard phases, "
            f"a = 0.2 ell, lambda = 0.1 ell, RK4, Oseen, FP32-compensated pair sum, FP64 state")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="n4096", type=workload_name,
                    help="the N = 4096 suspension is the measured configuration; the others are for profiles")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--fp64-steps", type=int, default=200)
    ap.add_argument("--dense-steps", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--unfused", action="store_true",
                    help="tuned launch with pair kernel and epilogue as two kernels (for profiles of that path)")
    ap.add_argument("--fused", type=int, choices=(0, 1, 2, 3, 4), default=None,
                    help="tuned launch with this stage form (0: two kernels, 1: 16 targets per work-group, "
                         "2: 64 targets per work-group, 3: 16 targets per work-group with streamed "
                         "sources, 4: resident, one work-group per system for a run of steps), for profiles "
                         "of the form the table did not choose")
    ap.add_argument("--precision", choices=("fp32c", "fp64"), default="fp32c",
                    help="arithmetic of the measured leg (the measured configuration is fp32c; fp64 for "
                         "the plain-FP64 workloads)")
    ap.add_argument("--tensor", choices=("oseen", "rpy"), default="oseen",
                    help="measurement runs of the RPY tensor (the measured configuration is Oseen)")
    ap.add_argument("--integrator", choices=("rk4", "heun"), default="rk4",
                    help="measurement runs of Heun steps (two stages; the measured configuration is RK4)")
    ap.add_argument("--kT", type=float, default=0.0, help="Brownian noise (Heun only)")
    ap.add_argument("--stroke-averaged", action="store_true",
                    help="time the stroke-averaged far-field equations on lattices of 5^3 to 16^3 dumbbells")
    ap.add_argument("--calibrate", action="store_true",
                    help="issue rate of the pair term's instruction mix and of FMA chains, and the shader clock")
    ap.add_argument("--calibrate-iters", type=int, default=4096)
    ap.add_argument("--counter-probe", action="store_true",
                    help="for rocprofv3 --pmc runs: a few steps plus one plain 256 MiB device copy")
    args = ap.parse_args()
    if args.kT != 0.0 and args.integrator != "heun":
        ap.error("--kT needs --integrator heun")
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)

    import torch
    import paper_1004_1932_amd as P
    from workload import make_preset

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.calibrate:
        calibrate(args.calibrate_iters)
        return
    if args.stroke_averaged:
        stroke_averaged_timing()
        return
    if args.workload.startswith(("arrays:", "single:")):
        from paper_1004_1932_amd.autotune import tuning_workload
        w = tuning_workload(args.workload)
    else:
        w = make_preset(args.workload)
    sizes = [int(v) for v in w.S_per_sys] if hasattr(w, "S_per_sys") else [w.S]
    Nb = 2.0 * np.asarray(sizes, dtype=np.float64)
    N, S = w.X.shape[0], int(sum(sizes))
    variant = args.tensor != "oseen" or args.integrator != "rk4" or args.kT != 0.0
    stages = 4 if args.integrator == "rk4" else 2
    flops_per_pair = FLOPS_PER_PAIR_RPY if args.tensor == "rpy" else FLOPS_PER_PAIR
    model = dict(tensor=args.tensor, integrator=args.integrator, kT=args.kT)
    pairs_per_step = stages * float((Nb * (Nb - 1)).sum())
    # FP32C: the dumbbell partner is summed in FP64 outside the pair kernel
    kernel_pairs = float((Nb * (Nb - 2)).sum()) if args.precision == "fp32c" else float((Nb * (Nb - 1)).sum())
    peak = PEAK_FP32_TFLOPS if args.precision == "fp32c" else PEAK_FP64_TFLOPS

    launch = "tuned"
    form = 0 if args.unfused else args.fused
    if form is not None and args.precision == "fp64":
        launch = dict(ipl=1, jchunk=0, wg=64, wj=1, posmode=0, fused=form)
    elif form is not None:
        from paper_1004_1932_amd.autotune import tuned_launch
        launch = dict(tuned_launch(sizes) or {}, fused=form)

    if args.counter_probe:
        # a known-size copy calibrates FETCH_SIZE / WRITE_SIZE against bytes
        src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        src.uniform_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        sim = P.Simulator(w.params, sizes, precision="fp32c", launch=launch)
        sim.set_state(w.X, w.phi)
        sim.step(3)
        torch.cuda.synchronize()
        print(json.dumps({"counter_probe": True, "copy_bytes": src.numel() * 8, "launch": sim.launch}), flush=True)
        return

    # The plain FP64 form (tiled) and the paper's dense-tensor design are timed
    # first, each with its own warm-up: the FP32C steps are then measured on a
    # device that has been busy for a while (at N = 4096 a few dozen steps are
    # about a millisecond of work, too short for the clocks to settle from idle).
    # plain FP64 form (tiled), on about 2e11 pair terms at most
    fp64_steps = max(2, min(args.fp64_steps, int(2e11 / pairs_per_step)))
    sim64 = P.Simulator(w.params, sizes, precision="fp64_tiled", graph=not args.no_graph, **model)
    sim64.set_state(w.X, w.phi)
    secs64, _ = time_steps(sim64, fp64_steps, max(1, fp64_steps // 10))
    v64 = pairs_per_step * fp64_steps / secs64
    log(f"fp64_tiled: {secs64 / fp64_steps * 1e3:.4f} ms/step, {v64:.4e} pairs/s")
    sim64.close()
    del sim64

    # FP64 in the FP32C form's own shape: the streamed stage kernel in FP64
    # arithmetic (rsqrt with a Newton step and FMAs), for a like-for-like
    # comparison of the two arithmetics (no steric forces)
    stream64 = None
    if getattr(w.params, "steric_k", 0.0) == 0.0:
        sims = P.Simulator(w.params, sizes, precision="fp64_tiled", graph=not args.no_graph,
                           launch=dict(ipl=1, jchunk=256, wg=64, wj=1, posmode=0, fused=3), **model)
        sims.set_state(w.X, w.phi)
        secss, _ = time_steps(sims, fp64_steps, max(1, fp64_steps // 10))
        assert sims.check() == 0
        vs = pairs_per_step * fp64_steps / secss
        log(f"fp64 streamed: {secss / fp64_steps * 1e3:.4f} ms/step, {vs:.4e} pairs/s")
        stream64 = {"value": vs, "unit": "pair interactions/s", "ms_per_step": secss / fp64_steps * 1e3,
                    "steps": fp64_steps,
                    "form": "the streamed stage kernel in FP64 (v_rsq_f64 with one Newton step, FMAs)"}
        sims.close()
        del sims

    # FP64 with the oracle's sum order (bitwise equal to it), the library's
    # tuned form for this size
    bitwise64 = None
    if args.precision == "fp32c":
        simb = P.Simulator(w.params, sizes, precision="fp64", graph=not args.no_graph, launch="tuned", **model)
        simb.set_state(w.X, w.phi)
        secsb, _ = time_steps(simb, fp64_steps, max(1, fp64_steps // 10))
        assert simb.check() == 0
        vb = pairs_per_step * fp64_steps / secsb
        log(f"fp64 bitwise: {secsb / fp64_steps * 1e3:.4f} ms/step, {vb:.4e} pairs/s")
        bitwise64 = {"value": vb, "unit": "pair interactions/s", "ms_per_step": secsb / fp64_steps * 1e3,
                     "steps": fp64_steps, "launch": simb.launch,
                     "form": "FP64 summed in ascending source order, bitwise equal to the oracle"}
        simb.close()
        del simb

    # the paper's own design: assembled full tensor, then the product (Sec. V);
    # per step 4 stages, each tensor written once and read once
    dense_bytes = 4 * 2 * 72.0 * float((Nb * Nb).sum())
    dense = None
    if dense_bytes / 8 <= 8e9 and not variant:
        simd = P.Simulator(w.params, sizes, precision="fp64_dense", graph=not args.no_graph)
        simd.set_state(w.X, w.phi)
        secsd, _ = time_steps(simd, args.dense_steps, max(1, args.dense_steps // 10))
        assert simd.check() == 0
        vd = pairs_per_step * args.dense_steps / secsd
        log(f"fp64_dense: {secsd / args.dense_steps * 1e3:.4f} ms/step, {vd:.4e} pairs/s")
        dense = {"value": vd, "unit": "pair interactions/s", "ms_per_step": secsd / args.dense_steps * 1e3,
                 "steps": args.dense_steps, "tensor_GBps": dense_bytes * args.dense_steps / secsd / 1e9}
        simd.close()
        del simd

    # FP32-compensated path, graph-replayed steps
    sim = P.Simulator(w.params, sizes, precision=args.precision, graph=not args.no_graph,
                      launch=launch, **model)
    sim.set_state(w.X, w.phi)
    log(f"{args.precision} launch {sim.launch}")

    # pair-kernel duration under HIP events on the launch stream (with fused
    # stages, the one kernel of a stage, which also does the stage update);
    # these event-bracketed steps also run before the timed ones, so that the
    # timed steps follow steps of their own kind with no idle pause
    P.ad_profile_pairs(sim.ctx, True)
    sim.step(args.profile_steps)
    kern_ms, launches = P.ad_profile_read(sim.ctx)
    P.ad_profile_pairs(sim.ctx, False)
    avg_ms = kern_ms / launches
    # stage-equivalents the timed launches covered: one per launch, or with
    # the resident form every stage of every step
    stage_units = args.profile_steps * stages if sim.launch.get("fused") == 4 else launches
    achieved = flops_per_pair * kernel_pairs * stage_units / (kern_ms * 1e-3) / 1e12
    log(f"pair kernel: {avg_ms * 1e3:.2f} us avg over {launches} launches, {achieved:.2f} TFLOP/s")

    secs, wall = time_steps(sim, args.steps, args.warmup)
    assert sim.check() == 0
    ms_per_step = secs / args.steps * 1e3
    value = pairs_per_step * args.steps / secs
    log(f"{args.precision}: {ms_per_step:.4f} ms/step, {value:.4e} pairs/s (wall {wall:.3f} s)")

    # With one kernel per stage (the fused forms) or per run of steps (the
    # resident form) the timed region runs nothing but that kernel, back to
    # back from graphs: its average duration per stage is the region's HIP
    # event time over the stages it ran (gaps between launches included).
    # The two-kernel form's pair kernel keeps the event-bracketed figure.
    isolated_us = kern_ms * 1e3 / stage_units  # per stage (the resident form: per stage of its launches)
    if sim.launch.get("fused", 0) in (1, 2, 3, 4):
        region_stages = args.steps * stages
        achieved = flops_per_pair * kernel_pairs * region_stages / secs / 1e12
        launch_us = secs / region_stages * 1e6
        timing = "timed region (HIP events on the launch stream) over its stage launches"
    else:
        launch_us = isolated_us
        timing = f"{launches} event-bracketed pair-kernel launches"

    out = {
        "metric": "Oseen pair interactions/s and sphere-steps/s at N=4096, FP32-comp vs FP64",
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32c" else "f64",
        "data": "synthetic",
        "config": {"workload": describe(args.workload), "name": args.workload,
                   "N": N, "S": S, "systems": len(sizes), "launch": sim.launch, "graph": not args.no_graph},
        "sphere_steps_per_s": N * args.steps / secs,
        "untimed_before": (f"{args.profile_steps} steps of event-bracketed launches (isolated_launch_us), then the "
                           f"{args.warmup} warm-up steps"),
        "fp64_tiled": {"value": v64, "unit": "pair interactions/s", "ms_per_step": secs64 / fp64_steps * 1e3,
                       "steps": fp64_steps},
        "speedup_vs_fp64": value / v64,
        "fp64_streamed": stream64,
        "speedup_vs_fp64_streamed": value / stream64["value"] if stream64 else None,
        "fp64_bitwise": bitwise64,
        "speedup_vs_fp64_bitwise": value / bitwise64["value"] if bitwise64 else None,
        "fp64_dense": dense,
        "speedup_vs_dense": value / dense["value"] if dense else None,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": (counted_traffic(sim.launch)
                                 if args.workload == COUNTED["workload"] and not variant else None),
                     "traffic_unit": "B per launch",
                     "kernel": KERNEL_NAMES[sim.launch.get("fused", 0)],
                     "avg_launch_us": launch_us,
                     "flops_per_launch": flops_per_pair * kernel_pairs,
                     "timing": timing,
                     "isolated_launch_us": isolated_us},
    }
    if variant:
        out["config"].update(model)
    if not args.no_cpu_baseline and not variant:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, sizes, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
