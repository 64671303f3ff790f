"""GPU parity at the full workload sizes, in the launch configuration the benchmark
times: the whole HIP path against the oracle's complete run of the same network.

  * 4,000-neuron CUBA network (ER p = 0.02, no delays): all 10,000 steps.
  * 200,000-neuron Brunel network (fixed out-degree 5,000, 1e9 synapses, 15-step
    delay, Poisson drive): the benchmark's 300-step settle period, its warm-up bench step
    and one timed bench step (1,000 simulation steps each), with the tiled delivery, 348
    base tiles (2-byte boundaries), one weight per source, and the device-side schedule,
    exactly as benchmarked.
  * 100,000-neuron plastic network (ER p = 0.02, 2e8 synapses, STDP on E->E, 10-step
    delay): all 2,000 steps, final FP32 weights of every synapse compared bit for bit,
    eagerly with the tiled delivery (the default) and with the atomic one, and lazily.
  * the largest Eq. 1 Brunel network (400,000 neurons, 1.6e10 synapses): sampled rows,
    and two steps' deliveries (after 300 steps) recomputed by the oracle from the GPU's own spikes.

Spike rasters, refractory counters, pending Q16 inputs and event/touch counts must be
identical, and binary32 state (V, traces, weights) bit-identical.  The oracle builds
these networks in host memory (8 GB for the 1e9-synapse one)."""
import numpy as np
import pytest

import oracle
from paper_1912_07423_amd import workloads as W
from gpu_compare import compare_net, compare_run, net

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    return gpu_available


def test_cuba_4k_all_10000_steps():
    spec = W.cuba_lif_4k()
    print(f"[full] cuba_lif_4k {spec['steps']} steps", flush=True)
    rg, inf = compare_run(spec, spec["steps"])
    n_spk = int(np.unpackbits(rg.view(np.uint8)).sum())
    print(f"[full] cuba_lif_4k: {n_spk} spikes, {inf['events']} events", flush=True)
    assert n_spk > 10_000


def test_brunel_200k_1e9_synapses():
    spec = W.brunel_fixed_out()
    steps = 300 + 2 * 1000
    print(f"[full] brunel_fixed_out n=200000 k=5000: {steps} steps", flush=True)
    rg, inf = compare_run(spec, steps, raster_steps=4096)
    assert inf["nnz"] == 200_000 * 5000
    assert inf["delivery"] == 2 and inf["tiles"] == 348 and inf["window"] == 15 and inf["source_weights"] == 1
    assert inf["tile_offset_bytes"] == 2
    print(f"[full] brunel: {int(np.unpackbits(rg.view(np.uint8)).sum())} spikes, "
          f"{inf['events']} events", flush=True)
    assert inf["events"] > 0


def test_brunel_200k_sampled_rows_match_generator():
    """Rows drawn one by one by the oracle's generator, including the first and last
    neuron and both sides of the excitatory/inhibitory boundary."""
    spec = W.brunel_fixed_out()
    g = net(spec, raster_steps=16)
    rng = np.random.default_rng(7)
    rows = [0, 1, 159_999, 160_000, 199_998, 199_999] + list(rng.integers(0, 200_000, 26))
    for i in rows:
        col, w = g.row(int(i))
        ocol, owq, _ = oracle.gen_row(spec, int(i))
        assert np.array_equal(col, ocol), f"row {i}"
        assert np.array_equal(w, owq), f"row {i}"
        assert len(col) == 5000 and int(i) not in set(col.tolist())


def test_stdp_100k_all_2000_steps_eager_and_lazy():
    """Both forms of Update Synapses on the 2e8-synapse plastic network against one run
    of the oracle: raster, V, traces, every weight and the touch count after 2,000 steps;
    eager with the tiled delivery (the default at this size) and with the atomic one."""
    spec = W.stdp_er()
    T = spec["steps"]
    print(f"[full] stdp_er n=100000 p=0.02: {T} steps, oracle", flush=True)
    o = oracle.OracleNet(spec, raster_cap=T)
    o.run(T)
    for mode, delivery, want in (("eager", "auto", 2), ("eager", "atomic", 1), ("lazy", "auto", 1)):
        print(f"[full] stdp {mode} {delivery}", flush=True)
        g = net(spec, raster_steps=T, plasticity=mode, delivery=delivery)
        g.run(T)
        rg, inf = compare_net(g, o, T)
        assert inf["plastic"] and inf["touches"] > 0 and inf["plasticity"] == (mode == "lazy")
        assert inf["delivery"] == want
        print(f"[full] stdp {mode} {delivery}: {int(np.unpackbits(rg.view(np.uint8)).sum())} spikes, "
              f"{inf['events']} events, {inf['touches']} touches", flush=True)
        g.close()


def _ids(row_words, n):
    return np.nonzero(np.unpackbits(np.ascontiguousarray(row_words).view(np.uint8), bitorder="little")[:n])[0]


def test_eq1_brunel_400k_1_6e10_synapses():
    """The largest network of the Eq. 1 size sweep (400,000 neurons, out-degree 40,000,
    1.6e10 synapses, 64 GB), too large for the oracle to hold: sampled rows against the
    oracle's row generator, and after 20 windows the pending input of two arrival
    steps against the oracle delivering the GPU's own spikes of their emission steps
    row by row; every delivered spike counts exactly 40,000 events."""
    n, k = 400_000, 40_000
    spec = W.brunel_scaled(n)
    g = net(spec, raster_steps=64)
    inf = g.info()
    assert inf["nnz"] == n * k and inf["delivery"] == 2
    rng = np.random.default_rng(11)
    for i in [0, 319_999, 320_000, 399_999] + [int(x) for x in rng.integers(0, n, 4)]:
        col, w = g.row(i)
        ocol, owq, _ = oracle.gen_row(spec, i)
        assert np.array_equal(col, ocol) and np.array_equal(w, owq), f"row {i}"
    d = inf["delay"]
    steps = 20 * inf["window"]  # past the start-up burst
    print(f"[full] brunel_scaled n={n}: {steps} steps", flush=True)
    g.run(steps)
    inf = g.info()
    assert inf["events"] == k * inf["spikes"] and inf["spikes"] > 0
    s = g.state()
    raster = g.raster_bits(steps - d, steps)
    for e in (steps - d, steps - 1):
        ids = _ids(raster[e - (steps - d)], n)
        ref, ev = oracle.deliver_generated(spec, ids, n)
        assert ev == k * len(ids)
        assert np.array_equal(s["input"][(e + d) % inf["input_buffers"]], ref), f"emission step {e}"
        print(f"[full] step {e}: {len(ids)} spikes delivered identically", flush=True)
