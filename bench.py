#!/usr/bin/env python
"""Throughput of the clock-driven work-queue SNN simulator on one MI355X.

Default workload (the headline line): Brunel-style network of 200,000 LIF neurons (4:1
exc./inh.), fixed out-degree 5,000 with uniform random targets (1e9 synapses stored as
int32 targets, with one Q16 weight per source population as in Table I), J = 0.1 mV,
g = 5, uniform delay 1.5 ms (15 steps), Poisson drive of 1,000 virtual inputs per neuron
at 20 Hz, dt = 0.1 ms.  Synthetic, generated on the device from a seed.  One "step" is
one run of the workload as configured: 1,000 simulation time steps (0.1 s simulated) of
the whole pipeline (update neurons -> FIFO -> receive spikes), continuing the same
network.  Every run first simulates SETTLE_STEPS = 300 simulation steps (30 ms): the
uniform random initial potentials cause a synchronous population burst in the first
~10 ms, and the timed steps are meant to measure the network's steady state (the
paper's runs simulate 10 s).  Then `--warmup` untimed bench steps, then exactly
`--steps` timed bench steps (defaults 1 and 5).

Prints one JSON line: synaptic events/s over the timed steps (inputs resident in HBM,
network built before the clock starts; the simulator runs as in production, windows
replayed from captured HIP graphs), wall time per simulated second, the delivery
kernel's achieved HBM bandwidth (algorithmic bytes / mean launch duration, from a pass
of the same length that follows the timed region with every launch stamped by HIP
events on the simulator's stream) against the 8 TB/s peak, its measured HBM traffic
when a counter summary of the same kernel source at the same operating point exists
under profiles/, and the CPU oracle's rate on a bounded sample of the same workload
with the host it ran on.

Other workloads (`--workload`, one JSON line each, not the headline):
  stdp   100,000-neuron plastic network (2e8 synapses, STDP on E->E), 2,000 steps
  sweep  512 independent networks (1k-20k neurons) in the batched persistent form,
         5,000 steps, against the plain per-network simulator on the same GPU
  bptt   surrogate-gradient BPTT (64 x 250 steps, 700 -> 1,024 -> 20), forward +
         adjoint, against the forward alone and a dense PyTorch reference on the GPU
  scaling  both models grown with the weight scaling of Eq. 1 (Vogels 4k-128k, Brunel
         20k-400k neurons), wall time per simulated second vs synapse count
  setup  network setup time vs size (Brunel, 1e7-1.6e10 synapses), cold and warm
         allocator, with the synapse fill's write bandwidth
  layout the delivery's bandwidth with CSR rows against 128-byte aligned rows, and with
         one weight per source against a weight per synapse
"""
import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "synaptic events/sec and % HBM roofline, 1 GPU; wall-time per simulated second"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of spike delivery: per synaptic event the target id (2 B from the
# tiled delivery's 16-bit target copy, 4 B for the atomic delivery) and, when weights are
# stored per synapse, the weight (4 B); per dequeued spike its id and its row pointers
# (4 + 8 B) and, with one weight per source, that weight (4 B)


def delivery_bytes(info):
    """(bytes per event, bytes per dequeued spike) of the network's delivery layout."""
    tb = int(info.get("target_bytes", 4))
    return (tb, 16) if info.get("source_weights") else (tb + 4, 12)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_deliver_tiled_brunel_200k_k5000_d15.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1912_07423_amd", "csrc", f)
                  for f in ("step.hip", "snn_internal.h", "device_math.h")]
WORKLOAD = "brunel_fixed_out_200k_k5000_d15_poisson20hz"
SETTLE_STEPS = 300  # past the start-up burst, always simulated before the warm-up
SIM_STEPS = 1000    # simulation steps per bench step: one run of the workload as configured


def workload_spec():
    from paper_1912_07423_amd import workloads as W
    return W.brunel_fixed_out(n=200_000, k=5000, delay_steps=15, rate_hz=20.0, n_ext=1000,
                              j_mV=0.1, g=5.0, seed=2, steps=1000)


def kernel_source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(point):
    """HBM bytes per delivery launch from the committed counter summary, if it was taken
    of the current kernel source at exactly this operating point (workload, settle,
    warm-up and timed steps, launch shape, and the timed region's events and spikes:
    the simulation is deterministic, so equal counts mean the same launches); otherwise
    None."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_sha() or t.get("operating_point") != point:
        return None
    return t.get("bytes_per_launch")


def host_info():
    """CPU model, usable hardware threads and RAM of this host."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = None
    try:
        for ln in open("/proc/meminfo"):
            if ln.startswith("MemTotal:"):
                ram = int(ln.split()[1]) * 1024
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(),
            "ram_gib": round(ram / 2**30, 1) if ram else None}


def launches_for(steps, window):
    """Delivery launches issued by one run(steps) call: windows of `window` steps (graph
    replays hold whole windows) and a shorter last window."""
    return -(-steps // window) if steps > 0 else 0


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


def copy_calibration(mib):
    """Plain device copies of a known size, for scaling the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: 3 copies of {mib} MiB", file=sys.stderr, flush=True)
    del a, b


def line(metric, value, unit, steps, warmup, ms_per_step, dtype, config, **extra):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
         "warmup": warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
         "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
         "config": config}
    d.update(extra)
    print(json.dumps(d), flush=True)


def bench_brunel(args):
    import torch
    from paper_1912_07423_amd import Network

    spec = workload_spec()
    print(f"[bench] building {spec['pops']} ...", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    net = Network(spec, raster_steps=4096, delivery=args.delivery, synapse_weights=args.synapse_weights)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - tb
    info = net.info()
    print(f"[bench] built in {build_s:.2f}s: {info}", file=sys.stderr, flush=True)
    K, Wb = args.steps, args.warmup
    sim_steps = K * SIM_STEPS
    net.run(SETTLE_STEPS)
    net.run(Wb * SIM_STEPS)
    net.sync()
    W = info["window"]
    print(f"[bench] settled {SETTLE_STEPS} + warm-up {Wb} x {SIM_STEPS} steps; timing {K} x {SIM_STEPS} steps",
          file=sys.stderr, flush=True)

    # (1) the timed region: the simulator as it runs in production, windows replayed from
    # captured HIP graphs, no per-launch timing
    i0 = net.info()
    torch.cuda.synchronize()
    net.sync()
    t0 = time.perf_counter()
    net.run(sim_steps)
    net.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    i1 = net.info()
    events = i1["events"] - i0["events"]
    spikes = i1["spikes"] - i0["spikes"]

    # (2) the kernel durations: the same number of steps again, continuing the run, every
    # launch issued on its own and stamped with its begin and end by HIP events on the
    # simulator's stream (stamping serialises the launches, which would add about 0.4 us
    # per step to the timed region, so it gets a pass of its own)
    before = (launches_for(SETTLE_STEPS, W) + launches_for(Wb * SIM_STEPS, W) +
              launches_for(sim_steps, W))
    net.set_profiling(True)
    net.reset_profile()
    j0 = net.info()
    net.run(sim_steps)
    net.sync()
    prof = net.profile()
    j1 = net.info()
    net.set_profiling(False)
    p_events = j1["events"] - j0["events"]
    p_spikes = j1["spikes"] - j0["spikes"]

    dt_ms = spec["params"]["dt_ms"]
    launches = max(1, prof["deliver_launches"])
    deliver_avg_ms = prof["deliver_ms"] / launches
    b_ev, b_spk = delivery_bytes(info)
    bytes_per_launch = (p_events * b_ev + p_spikes * b_spk) / launches
    achieved = bytes_per_launch / (deliver_avg_ms * 1e-3) / 1e9 if deliver_avg_ms > 0 else 0.0
    print(f"[bench] {sim_steps} steps in {wall * 1e3:.3f} ms; {events} events; stamped pass: "
          f"deliver {deliver_avg_ms * 1e3:.2f} us x {launches}; update "
          f"{prof['update_ms'] / max(1, prof['update_launches']) * 1e3:.2f} us x "
          f"{prof['update_launches']}", file=sys.stderr, flush=True)

    net.close()
    # the oracle sample runs after the GPU part, so that it takes no host core from the
    # launches being timed
    cpu = None
    if args.cpu_steps > 0:
        child = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                                  "--cpu-steps", str(args.cpu_steps)], stdout=subprocess.PIPE,
                                 text=True)
        out, _ = child.communicate()
        if child.returncode == 0 and out.strip():
            r = json.loads(out.strip().splitlines()[-1])
            cpu = {"value": r["events"] / r["seconds"], "unit": "events/s", "cores": 1,
                   "kind": "oracle",
                   "sample": f"the same 200k-neuron / 1e9-synapse network built by the oracle "
                             f"({r['build_s']:.0f} s on all host threads, untimed), first "
                             f"{r['steps']} steps timed ({r['seconds']:.1f} s, {r['events']} "
                             f"events) on one host thread",
                   "host": host_info()}
    kernel = "k_deliver_tiled" if info["delivery_name"] == "tiled" else "k_deliver_atomic"
    point = {"workload": WORKLOAD, "settle_steps": SETTLE_STEPS, "warmup": Wb,
             "steps": K, "sim_steps_per_step": SIM_STEPS, "events": p_events, "spikes": p_spikes,
             "delivery": info["delivery_name"], "tiles": info["tiles"], "window": W,
             "delivery_launches": prof["deliver_launches"]}
    traffic = measured_traffic(point) if kernel == "k_deliver_tiled" else None
    sim_s = sim_steps * dt_ms * 1e-3
    line(METRIC, events / wall, "events/s", K, Wb, wall * 1e3 / K, "int32",
         {"workload": WORKLOAD,
          "neurons": info["n"], "synapses": info["nnz"], "delay_steps": info["delay"],
          "dt_ms": dt_ms, "sim_steps_per_step": SIM_STEPS,
          "step": "one run of the workload as configured: 1,000 simulation steps (0.1 s "
                  "simulated), continuing the same network",
          "delivery": info["delivery_name"], "window": W,
          "tiles": info["tiles"], "source_weights": bool(info["source_weights"]),
          "settle_steps": SETTLE_STEPS, "parallelism": "single-gpu"},
         wall_s_per_sim_s=wall / sim_s, us_per_sim_step=wall * 1e6 / sim_steps, events=events,
         spikes_delivered=spikes, rate_hz=spikes / info["n"] / sim_s,
         build_s=build_s,
         kernels={"measured_over": f"a stamped pass of the same {sim_steps} steps following the timed region "
                                   f"(every launch stamped by HIP events on the simulator's stream; "
                                   f"{p_events} events)",
                  "deliver_ms_mean": deliver_avg_ms, "deliver_launches": prof["deliver_launches"],
                  "update_ms_mean": prof["update_ms"] / max(1, prof["update_launches"]),
                  "update_launches": prof["update_launches"],
                  "delivery_launches_before_timed": before},
         operating_point=point,
         roofline={"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
                   "bytes_per_launch": bytes_per_launch, "bytes_per_event": b_ev,
                   "bytes_per_spike": b_spk},
         cpu_baseline=cpu)


def bench_stdp(args):
    warm = max(args.warmup, SETTLE_STEPS)  # past the start-up burst
    import torch
    from paper_1912_07423_amd import Network
    from paper_1912_07423_amd import workloads as W
    spec = W.stdp_er()
    steps = args.steps or spec["steps"]
    delivery = args.delivery if args.plasticity == "eager" else "auto"
    net = Network(spec, raster_steps=4096, plasticity=args.plasticity, delivery=delivery)
    net.run(warm)
    net.sync()
    i0 = net.info()   # with lazy plasticity this brings every row current
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.run(steps)    # launches replayed from captured HIP graphs, no per-launch timing
    i1 = net.info()   # the timed region ends with every row current (weights, touches)
    wall = time.perf_counter() - t0
    events, touches = i1["events"] - i0["events"], i1["touches"] - i0["touches"]
    # kernel durations: a second pass of the same length, every launch stamped
    net.set_profiling(True)
    net.reset_profile()
    j0 = net.info()
    net.run(steps)
    j1 = net.info()
    prof = net.profile()
    net.set_profiling(False)
    spikes = j1["spikes"] - j0["spikes"]
    p_events = j1["events"] - j0["events"]
    dmean = prof["deliver_ms"] / max(1, prof["deliver_launches"])
    smean = prof["stdp_ms"] / max(1, prof["stdp_launches"])
    b_ev, b_spk = delivery_bytes(i1)
    dbytes = (p_events * b_ev + spikes * b_spk) / max(1, prof["deliver_launches"])
    # add throughput: one int32 add per synaptic event (device-scope atomics in global
    # memory for the atomic delivery, in LDS for the tiled one).  The run's rate inside
    # the delivery kernel, against the same kernel saturated by one step of 20,000 spikes
    # (about 4e7 events) over the same rows
    import numpy as np
    ids = np.random.default_rng(7).choice(i1["n"], 20_000, replace=False).astype(np.uint32)
    ms_sat, ev_sat = net.time_delivery(ids, reps=5, steps=1)
    achieved = p_events / (prof["deliver_ms"] * 1e-3) if prof["deliver_ms"] > 0 else 0.0
    saturated = ev_sat / (ms_sat * 1e-3) if ms_sat > 0 else 0.0
    tiled = i1["delivery_name"] == "tiled"
    dkernel = "k_deliver_tiled" if tiled else "k_deliver_atomic"
    line("STDP network: synaptic events/sec, STDP synapse touches/sec, 1 GPU", events / wall, "events/s",
         steps, warm, wall * 1e3 / steps, "fp32",
         {"workload": "stdp_er_100k_p0.02_d10_poisson10hz", "neurons": i1["n"], "synapses": i1["nnz"],
          "delay_steps": i1["delay"], "delivery": i1["delivery_name"], "plasticity": args.plasticity,
          "parallelism": "single-gpu"},
         touches_per_s=touches / wall, events=events, touches=touches,
         kernels={"measured_over": f"a stamped pass of the same {steps} steps following the timed region",
                  "deliver_ms_mean": dmean, "stdp_ms_mean": smean,
                  "update_ms_mean": prof["update_ms"] / max(1, prof["update_launches"]),
                  "launches_per_kernel": prof["deliver_launches"]},
         roofline={"bound": "hbm", "achieved": dbytes / (dmean * 1e-3) / 1e9 if dmean > 0 else 0.0,
                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": dbytes / (dmean * 1e-3) / 1e9 / HBM_PEAK_GBS if dmean > 0 else 0.0,
                   "traffic": None, "kernel": dkernel},
         atomics={"kernel": dkernel,
                  "per_event": "one int32 add in LDS" if tiled else "one device-scope int32 add",
                  "achieved_per_s": achieved, "saturated_per_s": saturated,
                  "frac": achieved / saturated if saturated > 0 else None,
                  "saturated_by": f"one step of {len(ids)} spikes ({ev_sat} events)"})
    net.close()


def bench_sweep(args):
    warm = max(args.warmup, SETTLE_STEPS)  # past the start-up burst
    import numpy as np
    import torch
    from paper_1912_07423_amd import Batch, Network
    from paper_1912_07423_amd import workloads as W
    specs = W.sweep()
    steps = args.steps or specs[0]["steps"]
    tb = time.perf_counter()
    b = Batch(specs, raster_steps=max(16, min(steps, 5000)))
    build_s = time.perf_counter() - tb
    tuning = b.autotune(trial_steps=100)
    print(f"[bench] sweep built in {build_s:.1f}s; tuning {tuning}", file=sys.stderr, flush=True)
    b.run(warm)
    b.sync()
    ev0 = sum(b.network(k).events for k in range(len(specs)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(steps)
    b.sync()
    wall = time.perf_counter() - t0
    events = sum(b.network(k).events for k in range(len(specs))) - ev0
    neurons = sum(b.network(k).n for k in range(len(specs)))
    synapses = sum(b.network(k).info()["nnz"] for k in range(len(specs)))
    b.close()
    # the plain per-network simulator on a stratified sample (every 8th network by size)
    order = np.argsort([s["pops"][0]["size"] + s["pops"][1]["size"] for s in specs])
    sample = order[::8]
    seq = 0.0
    for k in sample:
        g = Network(specs[k], raster_steps=16)
        g.run(warm)
        g.sync()
        t1 = time.perf_counter()
        g.run(steps)
        g.sync()
        seq += time.perf_counter() - t1
        g.close()
    seq_all = seq * len(specs) / len(sample)
    line("batched sweep: synaptic events/sec over 512 independent networks, 1 GPU", events / wall,
         "events/s", steps, warm, wall * 1e3 / steps, "int32",
         {"workload": "sweep_512_cuba_lif_1k-20k_p0.01-0.05", "networks": len(specs), "neurons": neurons,
          "synapses": synapses, "parallelism": "single-gpu"},
         network_steps_per_s=len(specs) * steps / wall, wall_s=wall, build_s=build_s, tuning=tuning,
         plain_sequential_s_estimate=seq_all,
         plain_sample=f"{len(sample)} networks (every 8th by size) run one after another with the plain "
                      f"simulator for {steps} steps: {seq:.2f} s, scaled by {len(specs) / len(sample):.0f}",
         speedup_vs_plain=seq_all / wall)


def bench_bptt(args):
    import numpy as np
    import torch
    from paper_1912_07423_amd import workloads as W
    from paper_1912_07423_amd.bptt import RecurrentLIF
    d = W.bptt_inputs()
    B, T, C = d["x"].shape
    H, O = d["w_out"].shape
    plan = RecurrentLIF(d["mask_in"], d["mask_rec"], O, B, T, checkpoint=25, dt_ms=d["dt_ms"])
    v_in, v_rec = plan.csr_values(d["w_in"], d["w_rec"])
    dev = plan.device
    x = torch.tensor(d["x"], device=dev)
    y = torch.tensor(d["labels"].astype(np.int32), device=dev)
    w_in = torch.tensor(v_in, device=dev, requires_grad=True)
    w_rec = torch.tensor(v_rec, device=dev, requires_grad=True)
    w_out = torch.tensor(d["w_out"], device=dev, requires_grad=True)
    iters = max(1, args.steps)

    def fwd_bwd():
        w_in.grad = w_rec.grad = w_out.grad = None
        plan.loss(x, w_in, w_rec, w_out, y).backward()

    def fwd():
        with torch.no_grad():
            plan.forward(x, w_in, w_rec, w_out, y)

    def timed(fn, n):
        for _ in range(max(3, min(10, args.warmup))):  # untimed iterations
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    t_fb = timed(fwd_bwd, iters)
    t_f = timed(fwd, iters)

    # dense PyTorch reference of the same model on the same GPU (float32, autograd with a
    # surrogate spike function)
    class Spike(torch.autograd.Function):
        @staticmethod
        def forward(ctx, z):
            ctx.save_for_backward(z)
            return (z >= 0).float()

        @staticmethod
        def backward(ctx, g):
            (z,) = ctx.saved_tensors
            return g / (1.0 + 25.0 * z.abs()) ** 2

    beta = math.exp(-d["dt_ms"] / 20.0)
    mi = torch.tensor(d["mask_in"], device=dev, dtype=torch.float32)
    mr = torch.tensor(d["mask_rec"], device=dev, dtype=torch.float32)
    Wi = torch.tensor(d["w_in"], device=dev, requires_grad=True)
    Wr = torch.tensor(d["w_rec"], device=dev, requires_grad=True)
    Wo = torch.tensor(d["w_out"], device=dev, requires_grad=True)
    yl = y.long()

    def dense():
        Wi.grad = Wr.grad = Wo.grad = None
        wi, wr = Wi * mi, Wr * mr
        v = torch.zeros(B, H, device=dev)
        s = torch.zeros(B, H, device=dev)
        u = torch.zeros(B, O, device=dev)
        m = None
        for t in range(T):
            v = beta * v + x[:, t] @ wi + s @ wr - s.detach()
            s = Spike.apply(v - 1.0)
            u = beta * u + s @ Wo
            m = u if m is None else torch.maximum(m, u)
        torch.nn.functional.cross_entropy(m, yl).backward()

    t_dense = timed(dense, max(1, iters // 4))
    line("surrogate-gradient BPTT: training iterations/sec (forward + adjoint), 1 GPU", 1.0 / t_fb,
         "iterations/s", iters, args.warmup, t_fb * 1e3, "fp32",
         {"workload": "bptt_rlif_b64_t250_in700_h1024_out20", "batch": B, "steps_per_sequence": T,
          "synapses": plan.nnz_in + plan.nnz_rec, "checkpoint": 25, "parallelism": "single-gpu"},
         forward_ms=t_f * 1e3, forward_backward_ms=t_fb * 1e3, dense_torch_ms=t_dense * 1e3,
         speedup_vs_dense_torch=t_dense / t_fb)
    plan.close()


def summarize_pmc(fetch_dir, write_dir, lines, copy_mib, command):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) of
    the same bench command into HBM bytes per tiled-delivery launch of its stamped pass,
    each counter scaled by what it reads for the plain device copy of `copy_mib` MiB in
    the same run.  `lines` are the two runs' JSON lines: they must report the same
    operating point (the simulation is deterministic), which is recorded with the
    summary, and they say how many delivery dispatches the stamped pass made (the run's
    last ones)."""
    import csv
    import glob

    recs = [json.loads(open(f).read().strip().splitlines()[-1]) for f in lines]
    points = [r["operating_point"] for r in recs]
    if points[0] != points[1]:
        raise SystemExit(f"the two runs differ: {points}")
    timed = points[0]["delivery_launches"]

    def read(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r.get("Counter_Name") == counter:
                        rows.append((int(r.get("Dispatch_Id", 0) or 0), r["Kernel_Name"], float(r["Counter_Value"])))
        if not rows:
            raise SystemExit(f"no {counter} rows under {d}")
        rows.sort()
        return [(k, v) for _, k, v in rows]

    out = {"kernel_source_sha": kernel_source_sha(), "operating_point": points[0], "command": command,
           "copy_mib": copy_mib}
    known = copy_mib * (1 << 20)
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = read(d, counter)
        # the three calibration copies are the largest copy dispatches of the run (the
        # runtime's copy kernel also serves the small copies of the simulator's setup)
        copies = sorted((v for k, v in rows if "copy" in k.lower()), reverse=True)[:3]
        deliver = [v for k, v in rows if "k_deliver_tiled" in k]
        if len(copies) < 3 or len(deliver) < timed:
            raise SystemExit(f"{counter}: need 3 copy and {timed} k_deliver_tiled dispatches, "
                             f"found {len(copies)} and {len(deliver)}")
        # the stamped pass is the run's last delivery work (launches replayed from graphs
        # before it may or may not be listed, so the count from the end is what is sure)
        deliver = deliver[len(deliver) - timed:]
        copy_kib = copies[1]
        factor = known / (copy_kib * 1024.0)
        out[f"{key}_copy_kib"] = copy_kib
        out[f"{key}_factor"] = factor
        # the per-dispatch counts summarised (min, mean, max KiB): the record stays short
        out[f"{key}_kib_per_dispatch"] = {"min": min(deliver), "mean": sum(deliver) / len(deliver),
                                          "max": max(deliver)}
        out[f"{key}_bytes_per_launch"] = sum(deliver) / len(deliver) * 1024.0 * factor
        out[f"{key}_dispatches"] = len(deliver)
    out["bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(out, indent=1))


def bench_scaling(args):
    """Eq. 1 size sweep (Sec. IV, the runtime-vs-synapses comparison): both models grown
    with their weights scaled so that the firing regime is kept."""
    warm = max(args.warmup, SETTLE_STEPS)  # past the start-up burst
    import torch
    from paper_1912_07423_amd import Network
    from paper_1912_07423_amd import workloads as W
    steps = args.steps
    points = []
    for model, sizes in (("vogels", (4000, 16000, 64000, 128000)),
                         ("brunel", (20000, 50000, 100000, 200000, 400000))):
        for n in sizes:
            spec = W.vogels_scaled(n) if model == "vogels" else W.brunel_scaled(n)
            net = Network(spec, raster_steps=max(16, steps))
            net.run(warm)
            net.sync()
            i0 = net.info()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            net.run(steps)
            net.sync()
            wall = time.perf_counter() - t0
            i1 = net.info()
            spikes = int(net.raster(warm, warm + steps).sum())
            dt = spec["params"]["dt_ms"] * 1e-3
            # the delivery kernel's roofline, from a separate profiled pass (HIP events
            # between the launches, which the timed run above does without)
            net.set_profiling(True)
            net.reset_profile()
            ip = net.info()
            net.run(min(steps, 300))
            net.sync()
            prof = net.profile()
            iq = net.info()
            net.set_profiling(False)
            b_ev, b_spk = delivery_bytes(iq)
            launches = max(1, prof["deliver_launches"])
            d_ms = prof["deliver_ms"] / launches
            d_bytes = ((iq["events"] - ip["events"]) * b_ev + (iq["spikes"] - ip["spikes"]) * b_spk) / launches
            d_gbs = d_bytes / (d_ms * 1e-3) / 1e9 if d_ms > 0 else 0.0
            p = {"model": model, "neurons": n, "synapses": i1["nnz"], "c": W.eq1_scale(model, n),
                 "wall_s_per_sim_s": wall / (steps * dt), "events_per_s": (i1["events"] - i0["events"]) / wall,
                 "rate_hz": spikes / n / (steps * dt), "delivery": i1["delivery_name"],
                 "deliver_us_mean": d_ms * 1e3, "deliver_gbs": d_gbs, "deliver_hbm_frac": d_gbs / HBM_PEAK_GBS}
            points.append(p)
            print(f"[bench] {json.dumps(p)}", file=sys.stderr, flush=True)
            net.close()
    top = points[-1]
    line("Eq. 1 size sweep: wall time per simulated second and synaptic events/sec vs synapse count, 1 GPU",
         top["events_per_s"], "events/s", steps, warm, top["wall_s_per_sim_s"] * 0.1, "int32",
         {"workload": "eq1_size_sweep_vogels_4k-128k_brunel_20k-400k", "parallelism": "single-gpu"},
         points=points)


def bench_layout(args):
    """Adjacency-layout A/B on the headline network (Sec. III-A.2 and Table I): CSR rows of
    5,000 targets (20,000 B, so row starts fall anywhere inside a 128-byte line) against
    rows of 5,024 targets (20,096 B = 157 lines: every row starts on a 128-byte boundary,
    the geometry of the paper's aligned 2-D adjacency array), each with one weight per
    source (4 B per synapse) and with a weight per synapse (8 B), through the tiled and
    the atomic delivery.  Reported: each delivery's algorithmic bytes per second."""
    warm = max(args.warmup, SETTLE_STEPS)  # past the start-up burst
    from paper_1912_07423_amd import Network
    from paper_1912_07423_amd import workloads as W
    steps = min(args.steps, 300)
    points = []
    for k in (5000, 5024):
        spec = W.brunel_fixed_out(n=200_000, k=k, delay_steps=15, rate_hz=20.0, n_ext=1000,
                                  j_mV=0.1, g=5.0, seed=2, steps=steps)
        for weights in ("auto", "per_synapse"):
            net = Network(spec, raster_steps=16, synapse_weights=weights)
            for delivery in ("tiled", "atomic"):
                net.set_delivery(delivery)
                net.run(warm)
                net.sync()
                i0 = net.info()
                net.set_profiling(True)
                net.reset_profile()
                net.run(steps)
                net.sync()
                prof = net.profile()
                i1 = net.info()
                net.set_profiling(False)
                b_ev, b_spk = delivery_bytes(i1)
                events, spikes = i1["events"] - i0["events"], i1["spikes"] - i0["spikes"]
                launches = max(1, prof["deliver_launches"])
                ms = prof["deliver_ms"] / launches
                gbs = (events * b_ev + spikes * b_spk) / launches / (ms * 1e-3) / 1e9
                p = {"row_targets": k, "row_bytes": 4 * k, "rows_128b_aligned": (4 * k) % 128 == 0,
                     "weights": "per_source" if i1["source_weights"] else "per_synapse",
                     "delivery": delivery, "deliver_us_mean": ms * 1e3, "launches": launches,
                     "events": events, "algorithmic_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
                points.append(p)
                print(f"[bench] {json.dumps(p)}", file=sys.stderr, flush=True)
            net.close()
    best = max(points, key=lambda p: p["algorithmic_gbs"])
    line("delivery bandwidth by adjacency layout (CSR vs 128-B aligned rows; 4 vs 8 B per synapse), 1 GPU",
         best["algorithmic_gbs"], "GB/s", steps, warm, None, "int32",
         {"workload": "layout_ab_brunel_200k_k5000_vs_k5024_d15", "parallelism": "single-gpu"},
         points=points)


def bench_setup(args):
    """Setup time vs network size (Sec. IV, the setup-time benchmark): Brunel networks,
    which carry no synapse state, so that setup is dominated by graph construction.  Each
    size is built three times back to back: the first build takes fresh device memory, the
    later ones reuse the blocks the caching allocator kept from the previous build (only
    growth allocates).  Reported per build: host wall time of the whole setup, and the
    device time of the row-length pass, the synapse fill and the delivery index, with the
    fill's write bandwidth (target ids, 4 B per synapse, and per-synapse weights when
    stored) against the HBM peak.  The headline network is built once more with the
    library's own device-memory cache instead of torch's allocator."""
    import torch
    from paper_1912_07423_amd import Network
    from paper_1912_07423_amd import workloads as W
    points = []
    from paper_1912_07423_amd import memory_cache_release
    cases = [("brunel_k5000", 200_000, W.brunel_fixed_out(), "torch")]
    cases += [("brunel_eq1", n, W.brunel_scaled(n), "torch") for n in (10_000, 20_000, 50_000, 100_000, 200_000, 400_000)]
    # the library's own device-memory cache (no torch allocator): hipMalloc on the first
    # build, reuse on the next ones
    cases += [("brunel_k5000", 200_000, W.brunel_fixed_out(), "library")]
    memory_cache_release()
    for name, n, spec, alloc in cases:
        for rep in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            net = Network(spec, raster_steps=16, torch_memory=(alloc == "torch"))
            torch.cuda.synchronize()
            wall_ms = (time.perf_counter() - t0) * 1e3
            i = net.info()
            net.close()
            written = i["nnz"] * (4 if i["source_weights"] else 8)
            p = {"model": name, "neurons": n, "synapses": i["nnz"], "allocator": alloc,
                 "build": "cold" if rep == 0 else "warm",
                 "setup_ms": wall_ms, "library_ms": i["build_ms"], "rows_ms": i["gen_rows_ms"],
                 "fill_ms": i["gen_fill_ms"], "index_ms": i["index_ms"],
                 "fill_write_gbs": written / (i["gen_fill_ms"] * 1e-3) / 1e9 if i["gen_fill_ms"] > 0 else None,
                 "synapses_per_s": i["nnz"] / (wall_ms * 1e-3)}
            points.append(p)
            print(f"[bench] {json.dumps(p)}", file=sys.stderr, flush=True)
    memory_cache_release()
    head = [p for p in points if p["model"] == "brunel_k5000" and p["build"] == "warm" and p["allocator"] == "torch"]
    best = min(head, key=lambda p: p["setup_ms"])
    line("network setup: synapses generated/sec (whole setup, warm allocator), 1 GPU",
         best["synapses_per_s"], "synapses/s", 1, 0, best["setup_ms"], "int32",
         {"workload": "setup_brunel_200k_k5000_and_eq1_brunel_10k-400k", "parallelism": "single-gpu"},
         fill_write_gbs=best["fill_write_gbs"],
         fill_hbm_frac=best["fill_write_gbs"] / HBM_PEAK_GBS if best["fill_write_gbs"] else None,
         points=points)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (Brunel workload: bench steps of 1,000 simulation steps, "
                         "default 5; other workloads: their own unit and default)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps after the fixed 300-step settle period (Brunel: bench "
                         "steps, default 1)")
    ap.add_argument("--plasticity", default="eager", choices=["eager", "lazy"],
                    help="STDP form of the plastic workload")
    ap.add_argument("--cpu-steps", type=int, default=1500,
                    help="steps of the CPU-oracle sample (0 disables it)")
    ap.add_argument("--delivery", default="auto")
    ap.add_argument("--synapse-weights", default="auto", choices=["auto", "per_synapse"])
    ap.add_argument("--workload", default="brunel", choices=["brunel", "stdp", "sweep", "bptt", "scaling", "setup", "layout"])
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run 3 plain device copies of this size first (HBM counter scaling)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "FETCH_LINE", "WRITE_LINE"),
                    help="write the traffic summary of two rocprofv3 --pmc runs (their output "
                         "directories and the JSON lines they printed) and exit")
    ap.add_argument("--pmc-command", default="", help="the profiled command, recorded in the summary")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.summarize_pmc:
        f, w, fl, wl = args.summarize_pmc
        summarize_pmc(f, w, [fl, wl], args.copy_calibration_mib, args.pmc_command)
        return
    if args.cpu_baseline_child:
        cpu_baseline_child(args.cpu_steps)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} (WORLD_SIZE {world}) is not "
              "supported: multi-GPU execution is not implemented (its sharding design is "
              "documented only)", file=sys.stderr, flush=True)
        sys.exit(2)
    # per-workload defaults of (timed steps, warm-up steps); 0 timed steps means the
    # workload's own length
    defaults = {"brunel": (5, 1), "stdp": (0, 0), "sweep": (0, 0), "bptt": (20, 10),
                "scaling": (1000, 15), "setup": (1000, 15), "layout": (1000, 15)}[args.workload]
    if args.steps is None:
        args.steps = defaults[0]
    if args.warmup is None:
        args.warmup = defaults[1]
    if args.copy_calibration_mib > 0:
        copy_calibration(args.copy_calibration_mib)
    {"brunel": bench_brunel, "stdp": bench_stdp, "sweep": bench_sweep, "bptt": bench_bptt,
     "scaling": bench_scaling, "setup": bench_setup, "layout": bench_layout}[args.workload](args)


if __name__ == "__main__":
    main()
