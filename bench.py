#!/usr/bin/env python
"""Throughput of the clock-driven work-queue SNN simulator on one MI355X.

Workload: Brunel-style network of 200,000 LIF neurons (4:1 exc./inh.), fixed
out-degree 5,000 with uniform random targets (1e9 synapses, int32 target + int32 Q16
weight), J = 0.1 mV, g = 5, uniform delay 1.5 ms (15 steps), Poisson drive of 1,000
virtual inputs per neuron at 20 Hz, dt = 0.1 ms.  Synthetic, generated on the device
from a seed.  One "step" is one simulation time step of the whole pipeline (update
neurons -> FIFO -> receive spikes); `--steps` steps are timed after `--warmup`.

Prints one JSON line: synaptic events/s over the timed steps (inputs resident in HBM,
network built before the clock starts), wall time per simulated second, the delivery
kernel's achieved HBM bandwidth (algorithmic bytes / mean launch time from HIP events
on the simulator's stream) against the 8 TB/s peak, and the CPU oracle's rate on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "synaptic events/sec and % HBM roofline, 1 GPU; wall-time per simulated second"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of spike delivery: per synaptic event the target id and the weight
# (4 + 4 B), per dequeued spike its id and its row pointers (4 + 8 B)
BYTES_PER_EVENT = 8
BYTES_PER_SPIKE = 12


def workload_spec():
    from paper_1912_07423_amd import workloads as W
    return W.brunel_fixed_out(n=200_000, k=5000, delay_steps=15, rate_hz=20.0, n_ext=1000,
                              j_mV=0.1, g=5.0, seed=2, steps=1000)


def cpu_baseline_child(steps):
    """Runs in a child process: the oracle on the same network for `steps` steps."""
    import oracle
    spec = workload_spec()
    t0 = time.perf_counter()
    net = oracle.OracleNet(spec, raster_cap=1)
    t1 = time.perf_counter()
    net.run(steps)
    t2 = time.perf_counter()
    print(json.dumps({"events": int(net.events), "seconds": t2 - t1, "build_s": t1 - t0,
                      "steps": steps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=15)
    ap.add_argument("--cpu-steps", type=int, default=1500,
                    help="steps of the CPU-oracle sample (0 disables it)")
    ap.add_argument("--delivery", default="auto")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child(args.cpu_steps)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} (WORLD_SIZE {world}) is not "
              "supported by this build (the multi-GPU design is documented, not built)",
              file=sys.stderr, flush=True)
        sys.exit(2)

    # the oracle sample runs on a host core while the GPU part runs
    child = None
    if args.cpu_steps > 0:
        child = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                                  "--cpu-steps", str(args.cpu_steps)], stdout=subprocess.PIPE,
                                 text=True, env=dict(os.environ, OMP_NUM_THREADS="1"))

    import torch
    from paper_1912_07423_amd import Network

    spec = workload_spec()
    print(f"[bench] building {spec['pops']} ...", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    net = Network(spec, raster_steps=4096, delivery=args.delivery)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - tb
    info = net.info()
    print(f"[bench] built in {build_s:.2f}s: {info}", file=sys.stderr, flush=True)
    net.run(args.warmup)
    net.sync()

    i0 = net.info()
    net.set_profiling(True)
    net.reset_profile()
    torch.cuda.synchronize()
    net.sync()
    t0 = time.perf_counter()
    net.run(args.steps)
    net.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = net.profile()
    i1 = net.info()
    net.set_profiling(False)

    events = i1["events"] - i0["events"]
    spikes = i1["spikes"] - i0["spikes"]
    emitted = int(net.raster(args.warmup, args.warmup + args.steps).sum()) if args.steps <= 4096 else None
    dt_ms = spec["params"]["dt_ms"]
    launches = max(1, prof["deliver_launches"])
    deliver_avg_ms = prof["deliver_ms"] / launches
    bytes_per_launch = (events * BYTES_PER_EVENT + spikes * BYTES_PER_SPIKE) / launches
    achieved = bytes_per_launch / (deliver_avg_ms * 1e-3) / 1e9 if deliver_avg_ms > 0 else 0.0
    print(f"[bench] {args.steps} steps in {wall * 1e3:.2f} ms; {events} events; "
          f"deliver {deliver_avg_ms * 1e3:.1f} us x {launches}; update "
          f"{prof['update_ms'] / max(1, prof['update_launches']) * 1e3:.1f} us x "
          f"{prof['update_launches']}", file=sys.stderr, flush=True)

    cpu = None
    if child is not None:
        out, _ = child.communicate()
        if child.returncode == 0 and out.strip():
            r = json.loads(out.strip().splitlines()[-1])
            cpu = {"value": r["events"] / r["seconds"], "unit": "events/s", "cores": 1,
                   "kind": "oracle",
                   "sample": f"the same 200k-neuron / 1e9-synapse network built by the oracle "
                             f"({r['build_s']:.0f} s, untimed), first {r['steps']} steps timed "
                             f"({r['seconds']:.1f} s, {r['events']} events), one host thread"}

    line = {
        "metric": METRIC,
        "value": events / wall,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "brunel_fixed_out_200k_k5000_d15_poisson20hz",
                   "neurons": info["n"], "synapses": info["nnz"], "delay_steps": info["delay"],
                   "dt_ms": dt_ms, "delivery": info["delivery_name"], "window": info["window"],
                   "tiles": info["tiles"], "parallelism": "single-gpu"},
        "wall_s_per_sim_s": wall / (args.steps * dt_ms * 1e-3),
        "events": events,
        "spikes_delivered": spikes,
        "spikes_emitted": emitted,
        "rate_hz": (emitted / info["n"] / (args.steps * dt_ms * 1e-3)) if emitted is not None else None,
        "build_s": build_s,
        "kernels": {"deliver_ms_mean": deliver_avg_ms, "deliver_launches": prof["deliver_launches"],
                    "update_ms_mean": prof["update_ms"] / max(1, prof["update_launches"]),
                    "update_launches": prof["update_launches"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_deliver_tiled" if info["delivery_name"] == "tiled" else "k_deliver_atomic"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    net.close()


if __name__ == "__main__":
    main()
