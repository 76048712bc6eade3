#!/usr/bin/env python3
"""Benchmark: full-scale cortical-microcircuit stand-in on one MI355X.

One step = one simulation time step of dt = 0.1 ms through the whole hot path
(Poisson drive, LIF exact update, spike staging, selection of matured
(source, delay-group) pairs, flat scan of their synapses, fixed-point
accumulation).  Default: 1,000 warm-up steps, then 100,000 timed steps
(10 s of biological time).  Inputs (network, state) are resident in HBM before
the timed region starts.

Prints ONE JSON line.  `value` is synaptic events/s (synapse deliveries per
wall-clock second over the timed steps); the real-time factor is reported
beside it.  The `roofline` object covers the dominant kernel (delivery) with
per-launch durations measured by HIP events inside this run; `cpu_baseline`
times the CPU oracle on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 100000] [--warmup 1000]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "real-time factor & synaptic events/s on 1 GPU; batched p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes of one step kernel (update + delivery):
#  - per delivered synapse: its 4-byte synapse word, plus
#      direct: one int64 accumulator read-modify-write (16 B),
#      binned: one 4-byte bin entry written and read back (8 B);
#  - per selected (source, delay-group) pair: 8-byte delay mask, 4-byte group
#    index, two 8-byte group offsets (28 B);
#  - per spike: stage entry written and read, raster entry, 16-byte record (28 B);
#  - per neuron: its state read and written (LIF: V, refractory count,
#    P synaptic currents; AdEx: V, w, h, P conductances) and I_e read;
#    direct delivery also reads its P int64 inputs.
BYTES_PER_EVENT = {"direct": 4 + 16, "binned": 4 + 8}
FP32_PEAK_TFLOPS = 157.3


def rk45_flops_per_attempt(ports: int, beta: bool = False) -> int:
    """fp32 operations of one attempted Cash-Karp substep of the AdEx model
    with `ports` conductances (fma = 2, exp2 / log2 / min / max / reciprocal =
    1): 6 right-hand sides of 15 + 4P (beta ports: 15 + 6P, the rising
    variable's decay and its fma into dg/dt), stage sums, fifth-order
    solution, error estimate and error ratio of 60 per each of the 2 + P
    (beta: 2 + 2P) components, and 9 of step control."""
    if beta:
        return 6 * (15 + 6 * ports) + 60 * (2 + 2 * ports) + 9
    return 6 * (15 + 4 * ports) + 60 * (2 + ports) + 9
BYTES_PER_PAIR = 28
BYTES_PER_SPIKE = 28


def measured_traffic(workload: str, kernel: str, tile_neurons: int = 0):
    """HBM bytes per launch of the step kernel from the committed counter
    summary, or None when the kernel sources have changed since it was taken
    (or it was taken for another kernel or tile size on this workload)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["kernel_sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["kernel_sources_sha256"] or workload not in rec["workloads"]:
        return None
    ent = rec["workloads"][workload]
    if ent["kernel"] != kernel or ent.get("tile_neurons", tile_neurons) != tile_neurons:
        return None
    return ent["bytes_per_launch"]


def bytes_per_step_neurons(spec: dict, delivery: str) -> int:
    tot = 0
    for p in spec["populations"]:
        ports = p["ports"]
        if p["model"] == "aeif_cond_exp":
            b = 8 * 3 + 8 * ports + 4
        elif p["model"] == "aeif_cond_beta":
            b = 8 * 3 + 16 * ports + 4
        elif p["model"] == "lif_exp":
            b = 8 * 2 + 8 * ports + 4
        else:
            b = 8 * 2 + 4
        if delivery == "direct":
            b += 8 * ports
        tot += b * p["n"]
    return tot


def step_roofline(net, specs: list, mode: str, steps: int, c0: dict, c1: dict, profile_steps: int,
                  workload: str) -> dict:
    """HBM roofline of the step kernel over the timed region: the algorithmic
    bytes of those steps (per-neuron state, per event, per selected pair, per
    spike) over the device time per step, measured with HIP events recorded on
    the library's stream around the timed call's graph launches (so it holds
    the step kernels and the short gaps between them).  Also: `profile_steps`
    further steps launched one by one with events on each dispatch (the
    isolated kernel, for reference), and the measured traffic where it is on
    record."""
    ps = max(1, steps)
    dev_ms = c1["last_call_device_ms"] / ps
    ev_p = (c1["events"] - c0["events"]) / ps
    pr_p = (c1["pairs"] - c0["pairs"]) / ps
    sp_p = (c1["spikes"] - c0["spikes"]) / ps
    c2 = net.counters()
    prof = net.profile(profile_steps) if profile_steps > 0 else {"step": 0.0}
    iso_ms = prof["step"] / max(1, profile_steps)
    kernel = "k_step" if mode != "binned" else "k_step_binned_runs" if c2.get("tile_runs") else "k_step_binned"
    neuron_bytes = sum(bytes_per_step_neurons(sp, mode) for sp in specs)
    dlv_bytes = neuron_bytes + ev_p * BYTES_PER_EVENT[mode] + pr_p * BYTES_PER_PAIR + sp_p * BYTES_PER_SPIKE
    achieved = dlv_bytes / (dev_ms * 1e-3) / 1e9 if dev_ms > 0 else 0.0
    return {
        "kernel": kernel, "bound": "hbm",
        "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": measured_traffic(workload, kernel, c2["tile_neurons"]),
        "avg_launch_us": round(dev_ms * 1e3, 3), "bytes_per_launch": round(dlv_bytes),
        "timing": "HIP events on the library stream around the timed call's graph launches, per step",
        "isolated_launch_us": round(iso_ms * 1e3, 3),
        "neuron_bytes_per_launch": neuron_bytes,
        "events_per_launch": round(ev_p, 1), "pairs_per_launch": round(pr_p, 1),
        "spikes_per_launch": round(sp_p, 1), "delivery": mode, "tile_neurons": c2["tile_neurons"],
        "spill_events": c2["spill_events"],
        "events_per_s_in_kernel": round(ev_p / (dev_ms * 1e-3), 1) if dev_ms > 0 else None,
    }


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100_000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--settle", type=int, default=1000,
                    help="untimed steps run right after the build, before the warm-up, so that the timed steps "
                         "sample the network's steady state rather than its onset transient")
    ap.add_argument("--profile-steps", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=10_000)
    ap.add_argument("--k-ext", type=int, default=None)
    ap.add_argument("--weight-sd", type=float, default=0.0,
                    help="microcircuit: draw every weight from a normal of this relative deviation (32 levels)")
    ap.add_argument("--requests", type=int, default=60, help="serve: requests in the arrival trace")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: mean arrivals per second")
    ap.add_argument("--slots", type=int, default=16, help="serve: requests in flight at once")
    ap.add_argument("--serve-delivery-blocks", type=int, default=64,
                    help="serve: delivery blocks of each served network (few, so that concurrent networks' "
                         "kernels find free slots)")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="serve: hardware queues HIP opens for the process (GPU_MAX_HW_QUEUES, at most 32; "
                         "0: HIP's default), so that that many request streams can run kernels at once")
    ap.add_argument("--workload", choices=["microcircuit", "adex", "alpha", "alpha_scan", "sweep", "serve"],
                    default="microcircuit",
                    help="microcircuit (default line); adex: 1e6 AdEx neurons, in-degree 1000, exponential "
                         "conductances; alpha: the balanced network with alpha conductances and normal delays "
                         "(--neurons, --indegree); alpha_scan: its simulation time over N at in-degree 1000 and "
                         "over the in-degree at N = 30000; sweep: batched Brunel instances vs the same instances "
                         "run one by one")
    ap.add_argument("--neurons", type=int, default=1_000_000, help="alpha: number of neurons")
    ap.add_argument("--indegree", type=int, default=1000, help="alpha: in-degree")
    ap.add_argument("--instances", type=int, default=128, help="sweep: number of instances")
    ap.add_argument("--seq-instances", type=int, default=16,
                    help="sweep: instances also run one by one (sequential baseline sample)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (delivery mode, tile size, delivery blocks chosen by timing)")
    ap.add_argument("--delivery", choices=["auto", "direct", "binned"], default="auto",
                    help="how events are summed: device atomics, or bins per target tile summed in LDS")
    ap.add_argument("--tile-neurons", type=int, default=0, help="binned delivery: neurons per tile (0: library)")
    ap.add_argument("--bin-capacity", type=int, default=0, help="binned delivery: entries per tile bin (0: library)")
    ap.add_argument("--delivery-blocks", type=int, default=0,
                    help="blocks that deliver delays of 2 steps or more (0: library)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a device copy of this many MiB (counter calibration) and exit")
    return ap.parse_args()


def cpu_baseline(steps: int) -> dict:
    """Oracle (plain C, fp64) on the microcircuit stand-in at N/10 with the
    full in-degrees and drive: same per-neuron input statistics and rates as
    the full network, one tenth of the neurons and synapses.  Timed twice:
    the plain build on one thread, and the same source built with OpenMP on
    all the host's cores (neuron and delivery loops split over threads; same
    results).  The all-core leg is the reported value."""
    from oracle import oracle as O
    from paper_2007_14236_amd import workloads as W
    spec = W.microcircuit(scale=0.1, k_scale=1.0)
    bio = steps * spec["dt"] * 1e-3
    legs = {}
    for name, omp in (("one_core", False), ("all_cores", True)):
        t0 = time.perf_counter()
        net = O.OracleNet(spec, O.FP64, openmp=omp)
        t_build = time.perf_counter() - t0
        net.simulate(1000)
        e0 = net.events
        t0 = time.perf_counter()
        net.simulate(steps)
        wall = time.perf_counter() - t0
        ev = net.events - e0
        legs[name] = {"value": ev / wall, "unit": "events/s", "cores": net.threads, "rtf": wall / bio,
                      "build_s": round(t_build, 2)}
        del net
    out = dict(legs["all_cores"])
    out.update({"kind": "oracle",
                "sample": (f"microcircuit stand-in at N/10 with full in-degrees ({W.total_neurons(spec)} neurons, "
                           f"{W.count_synapses(spec):.3g} synapses), fp64 oracle, {steps} steps ({bio:g} s bio) "
                           "after 1000 warm-up steps, build excluded; OpenMP build on all host cores "
                           "(one_core: the plain build on one thread)"),
                "one_core": legs["one_core"],
                "host": platform.processor() or platform.machine(), "host_cpus": os.cpu_count()})
    return out


def copy_calibration(mib: int):
    import torch
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": mib << 20}))


def main():
    args = parse()
    if args.workload == "serve" and args.hw_queues:  # before anything initialises HIP
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(1, args.hw_queues)))
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the engine has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2007_14236_amd import snn as S
    from paper_2007_14236_amd import workloads as W

    if args.workload == "sweep":
        return bench_sweep(args, S, W, torch)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "alpha_scan":
        return bench_alpha_scan(args, S, W, torch)
    if args.workload == "adex":
        spec = W.adex_balanced()
    elif args.workload == "alpha":
        spec = W.adex_balanced_alpha(n=args.neurons, k=args.indegree)
    else:
        kw = {} if args.k_ext is None else {"k_ext": args.k_ext}
        spec = W.microcircuit(scale=1.0, weight_sd=args.weight_sd, **kw)
    dt = spec["dt"]
    print(f"[bench] building {spec['name']}: {W.total_neurons(spec)} neurons, "
          f"{W.count_synapses(spec):.4g} synapses", file=sys.stderr, flush=True)
    tuned, tune_s = None, 0.0
    kw = dict(delivery=args.delivery, tile_neurons=args.tile_neurons, bin_capacity=args.bin_capacity,
              delivery_blocks=args.delivery_blocks)
    if not args.no_tune and args.delivery == "auto" and not args.tile_neurons:
        from paper_2007_14236_amd import autotune as A
        t0 = time.perf_counter()
        best, table = A.tune(spec, log=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
        tune_s = time.perf_counter() - t0
        tuned = {"chosen": best, "candidates": table, "seconds": round(tune_s, 2)}
        kw = dict(best, bin_capacity=args.bin_capacity)
    t0 = time.perf_counter()
    net = S.Net(spec, **kw)
    build_s = time.perf_counter() - t0
    mode = "binned" if net.counters()["delivery"] == 2 else "direct"
    net.simulate(args.settle)  # onset transient of the initial state, untimed
    net.simulate(args.warmup)
    torch.cuda.synchronize()
    c0 = net.counters()
    print(f"[bench] warm-up {args.warmup} steps done; timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.simulate(args.steps)  # returns after the device has finished
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c1 = net.counters()
    events = c1["events"] - c0["events"]
    pairs = c1["pairs"] - c0["pairs"]
    spikes = c1["spikes"] - c0["spikes"]
    bio_s = args.steps * dt * 1e-3
    ms_per_step = wall * 1e3 / args.steps
    print(f"[bench] {args.steps} steps in {wall:.3f} s (RTF {wall / bio_s:.4f}); profiling "
          f"{args.profile_steps} steps", file=sys.stderr, flush=True)

    c2 = net.counters()
    traffic_key = args.workload + ("_weight_sd" if args.weight_sd > 0 else "")
    roofline = step_roofline(net, [spec], mode, args.steps, c0, c1, args.profile_steps, traffic_key)
    dlv_ms = roofline["avg_launch_us"] * 1e-3
    out = {
        "metric": METRIC,
        "value": events / wall,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_steps": args.settle,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state, i64 fixed-point input",
        "data": "synthetic",
        "rtf": wall / bio_s,
        "bio_seconds": bio_s,
        "build_s": build_s,
        "spikes_per_s_bio": spikes / bio_s,
        "mean_rate_hz": spikes / bio_s / W.total_neurons(spec),
        "events_per_step": events / args.steps,
        "pairs_per_step": pairs / args.steps,
        "config": {"workload": "cortical microcircuit stand-in: 8 LIF-exp populations, 77,169 neurons, 3.0e8 synapses"
                               + (f", weights normal (sd {args.weight_sd:g} of the mean, 32 levels)"
                                  if args.weight_sd > 0 else ""),
                   "neurons": W.total_neurons(spec), "synapses": W.count_synapses(spec),
                   "populations": dict(zip(W.MC_NAMES, W.MC_SIZES)), "dt_ms": dt,
                   "t_bio_s": bio_s, "k_ext": spec["poisson"][0]["n_inputs"],
                   "parallelism": "single GPU"},
        "paper_context": {"rtf_rtx2080ti": 1.055, "rtf_v100": 1.641,
                          "note": "real microcircuit (this is a synthetic stand-in of the same size)"},
        "roofline": roofline,
        "autotune": tuned,
    }
    if args.workload in ("adex", "alpha"):
        if args.workload == "adex":
            out["config"] = {"workload": "balanced AdEx network: 1,000,000 neurons (800k E / 200k I), in-degree "
                                         "1000, exponential conductances on 2 ports, RK45 rtol 1e-6, delays U[1,2) ms",
                             "neurons": W.total_neurons(spec), "synapses": W.count_synapses(spec), "dt_ms": dt,
                             "t_bio_s": bio_s, "parallelism": "single GPU"}
            out["paper_context"] = {"rtf_rtx2080ti": 70.0, "note": "alpha conductances in the paper"}
        else:
            out["config"] = {"workload": f"balanced AdEx network as in Sec. 2.4 / Table 1: {W.total_neurons(spec):,} "
                                         f"neurons (80% E / 20% I), in-degree {args.indegree}, alpha conductances "
                                         "(tau 1 ms) on 2 ports, peak weights 0.05 / 0.35 / 0.37 nS, Poisson 20 kHz, "
                                         "delays normal 0.5 +- 0.25 ms, RK45 rtol 1e-6",
                             "neurons": W.total_neurons(spec), "synapses": W.count_synapses(spec), "dt_ms": dt,
                             "t_bio_s": bio_s, "parallelism": "single GPU"}
            out["paper_context"] = {"rtf_rtx2080ti": 70.0 if args.neurons == 1_000_000 and args.indegree == 1000
                                    else None, "rate_hz_table1": 30.7}
        att_p = (c1["rk_accepted"] + c1["rk_rejected"] - c0["rk_accepted"] - c0["rk_rejected"]) / max(1, args.steps)
        fpa = rk45_flops_per_attempt(2, beta=args.workload == "alpha")
        tflops = att_p * fpa / (dlv_ms * 1e-3) / 1e12 if dlv_ms > 0 else 0.0
        out["rk45"] = {"accepted_per_step": (c1["rk_accepted"] - c0["rk_accepted"]) / args.steps,
                       "rejected_per_step": (c1["rk_rejected"] - c0["rk_rejected"]) / args.steps}
        out["rk45_fp32_roofline"] = {"kernel": roofline["kernel"], "bound": "alu", "achieved": round(tflops, 3),
                                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                     "frac": round(tflops / FP32_PEAK_TFLOPS, 5), "flops_per_attempt": fpa,
                                     "attempts_per_launch": round(att_p, 1),
                                     "note": "attempted substeps x flops per attempt / step-kernel duration; the "
                                             "step is bounded by the serial RK45 chain of neurons in their spike "
                                             "step (~100 attempts), not by throughput"}
    net.close()
    if not args.no_cpu_baseline and args.workload == "microcircuit":
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(out), flush=True)


def bench_alpha_scan(args, S, W, torch):
    """Simulation time per biological second of the alpha-conductance
    balanced network (Sec. 2.4, Table 1) over the number of neurons at
    in-degree 1000, and over the in-degree at 30,000 neurons (the two scans of
    the paper's balanced-network results): each point built, warmed up for
    `--warmup` steps and timed over `--steps` steps with the library's default
    delivery."""
    points = [("N", n, 1000) for n in (10_000, 30_000, 100_000, 300_000, 1_000_000)]
    points += [("K", 30_000, k) for k in (1000, 3000, 10_000, 20_000, 30_000)]
    rows = []
    for scan, n, k in points:
        spec = W.adex_balanced_alpha(n=n, k=k)
        t0 = time.perf_counter()
        net = S.Net(spec)
        build_s = time.perf_counter() - t0
        net.simulate(args.warmup)
        torch.cuda.synchronize()
        c0 = net.counters()
        t0 = time.perf_counter()
        net.simulate(args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        c1 = net.counters()
        bio = args.steps * spec["dt"] * 1e-3
        ev = c1["events"] - c0["events"]
        row = {"scan": scan, "neurons": n, "indegree": k, "synapses": W.count_synapses(spec),
               "delivery": "binned" if c1["delivery"] == 2 else "direct", "build_s": round(build_s, 2),
               "rtf": round(wall / bio, 4), "events_per_s": round(ev / wall),
               "rate_hz": round((c1["spikes"] - c0["spikes"]) / bio / n, 2)}
        net.close()
        rows.append(row)
        print(f"[bench] {row}", file=sys.stderr, flush=True)
    big = [r for r in rows if r["neurons"] == 1_000_000 and r["indegree"] == 1000][0]
    out = {"metric": METRIC, "value": big["rtf"], "unit": "s wall / s bio (1e6 neurons, in-degree 1000)",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": big["rtf"] * 0.1, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 state, i64 fixed-point input", "data": "synthetic",
           "config": {"workload": "alpha-conductance balanced network scans (Sec. 2.4, Table 1): N at in-degree "
                                  "1000; in-degree at N = 30,000", "parallelism": "single GPU"},
           "paper_context": {"rtf_rtx2080ti_1e6": 70.0, "rate_hz_table1": 30.7},
           "points": rows}
    print(json.dumps(out), flush=True)


def bench_sweep(args, S, W, torch):
    """Batched sweep: all instances in one network (one set of launches per
    step) against the same instances simulated one after another."""
    specs = [W.brunel_sweep_instance(i) for i in range(args.instances)]
    steps = args.steps
    print(f"[bench] building the batch: {args.instances} instances, "
          f"{sum(W.total_neurons(sp) for sp in specs)} neurons, "
          f"{sum(W.count_synapses(sp) for sp in specs):.4g} synapses", file=sys.stderr, flush=True)
    kw = dict(delivery=args.delivery, tile_neurons=args.tile_neurons, bin_capacity=args.bin_capacity)
    tuned = None
    if not args.no_tune and args.delivery == "auto" and not args.tile_neurons:
        from paper_2007_14236_amd import autotune as A
        t0 = time.perf_counter()
        best, table = A.tune(specs, steps=200, warmup=100,
                             log=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
        tuned = {"chosen": best, "candidates": table, "seconds": round(time.perf_counter() - t0, 2)}
        kw = dict(best, bin_capacity=args.bin_capacity)
    t0 = time.perf_counter()
    net = S.Net(specs, record=True, **kw)
    build_s = time.perf_counter() - t0
    mode = "binned" if net.counters()["delivery"] == 2 else "direct"
    print(f"[bench] built in {build_s:.1f} s ({mode} delivery); warm-up {args.warmup} steps", file=sys.stderr,
          flush=True)
    net.simulate(args.warmup)
    torch.cuda.synchronize()
    c0 = net.counters()
    t0 = time.perf_counter()
    net.simulate(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c1 = net.counters()
    events = c1["events"] - c0["events"]
    print(f"[bench] batch: {steps} steps in {wall:.3f} s; profiling {args.profile_steps} steps", file=sys.stderr,
          flush=True)
    roofline = step_roofline(net, specs, mode, args.steps, c0, c1, args.profile_steps, "sweep")
    print("[bench] sequential sample next", file=sys.stderr, flush=True)
    net.close()
    del net
    # sequential baseline: a sample of the instances, one at a time, same steps,
    # each in the faster of the two delivery modes
    nseq = min(args.seq_instances, args.instances)
    seq_wall, seq_events = 0.0, 0
    for i in range(nseq):
        best = None
        for dmode in ("direct", "binned"):
            n1 = S.Net(specs[i], record=True, delivery=dmode)
            n1.simulate(args.warmup)
            torch.cuda.synchronize()
            e0 = n1.counters()["events"]
            t0 = time.perf_counter()
            n1.simulate(steps)
            torch.cuda.synchronize()
            w1 = time.perf_counter() - t0
            ev1 = n1.counters()["events"] - e0
            n1.close()
            if best is None or w1 < best[0]:
                best = (w1, ev1)
        seq_wall += best[0]
        seq_events += best[1]
        print(f"[bench] sequential instance {i + 1}/{nseq} done", file=sys.stderr, flush=True)
    bio = steps * specs[0]["dt"] * 1e-3
    sizes = [W.total_neurons(sp) for sp in specs]
    seq_est = seq_wall * args.instances / nseq
    out = {"metric": METRIC, "value": events / wall, "unit": "events/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 state, i64 fixed-point input", "data": "synthetic",
           "rtf": wall / bio, "build_s": build_s, "delivery": mode, "autotune": tuned,
           "batched_instance_seconds_per_wall_second": args.instances * bio / wall,
           "sequential_sample": {"instances": nseq, "delivery": "faster of direct and binned per instance",
                                 "wall_s": seq_wall, "events_per_s": seq_events / seq_wall,
                                 "estimated_wall_all_s": seq_est},
           "speedup_vs_sequential": seq_est / wall,
           "config": {"workload": f"batched sweep of {args.instances} Brunel LIF instances, N in [2k, 40k], "
                                  "in-degree 0.1 N, g in [3,7], drive 10-30 Hz, delays U[0.1,3) ms",
                      "neurons": sum(sizes), "synapses": sum(W.count_synapses(sp) for sp in specs),
                      "t_bio_s": bio, "parallelism": "single GPU"},
           "roofline": roofline}
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Serving: a seeded arrival trace through the library's request server
    (continuous admission by device-memory budget, `--slots` requests in
    flight) and through the same server with one slot (one request at a
    time, arrival order); p50/p99 latency from arrival to result, throughput,
    and a check that sampled requests give the same raster served as alone."""
    from paper_2007_14236_amd import serve as V

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    trace = V.request_trace(args.requests, rate_hz=args.rate)
    check = (0, 1, len(trace) - 1)
    budget = 200 << 30
    out = {}
    for name, slots in (("served", args.slots), ("fifo", 1)):
        log(f"serving {len(trace)} requests, {name} ({slots} slots)")
        rep = V.Server(budget_bytes=budget, slots=slots, log=log, digest_ids=set(check),
                       net_kw=dict(delivery_blocks=args.serve_delivery_blocks)).serve(trace)
        lat = rep.latencies()
        failed = [r.rid for r in rep.results if r.status != 0]
        if failed:
            raise RuntimeError(f"requests {failed} failed")
        out[name] = {"requests_per_s": len(trace) / rep.makespan_s, "makespan_s": rep.makespan_s,
                     "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                     "events_per_s": rep.events / rep.makespan_s, "slots": slots,
                     "peak_device_bytes": rep.peak_bytes,
                     "mean_wait_s": float(np.mean([r.start_s - r.arrival_s for r in rep.results]))}
        if name == "served":
            digests = {r.rid: r.digest for r in rep.results}
    sample = [r for r in trace if r.rid in check]
    same = all(V.run_alone(r) == digests[r.rid] for r in sample)
    log(f"alone-vs-served check on requests {[r.rid for r in sample]}: {same}")
    bio = sum(r.steps for r in trace) * trace[0].spec["dt"] * 1e-3
    res = {"metric": METRIC, "value": out["served"]["requests_per_s"], "unit": "requests/s", "n_gpus": 1,
           "steps": sum(r.steps for r in trace), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 state, i64 fixed-point input", "data": "synthetic",
           "p50_latency_s": out["served"]["p50_latency_s"], "p99_latency_s": out["served"]["p99_latency_s"],
           "served": out["served"], "fifo": out["fifo"],
           "throughput_vs_fifo": out["served"]["requests_per_s"] / out["fifo"]["requests_per_s"],
           "identical_alone_and_served": same, "delivery_blocks_per_request": args.serve_delivery_blocks,
           "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES", "HIP default"),
           "config": {"workload": f"serving trace: {len(trace)} requests, Poisson arrivals at {args.rate:g}/s, "
                                  "alternately microcircuit stand-in at scale U[0.1,1] and balanced AdEx with "
                                  "N ~ U[10k,200k], K = 1000, each for U[0.1,2] s of biological time",
                      "requests": len(trace), "bio_seconds_total": bio, "budget_bytes": budget,
                      "parallelism": "single GPU"}}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
