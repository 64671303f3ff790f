"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by
element on the same seeded inputs.  Spike rasters, integer state, Q16 accumulators and
synapse tables must be bit-identical; binary32 state (V, traces, plastic weights) is
compared bit for bit as well (same operations in the same order, no contraction), which
is stricter than the 1e-6 relative bar."""
import numpy as np
import pytest

import oracle
from paper_1912_07423_amd import workloads as W
from gpu_compare import bits as _bits, compare_net as _compare_net, compare_run as _compare_run, net as _net

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    return gpu_available


def _small_specs():
    return {
        "cuba_4k": W.cuba_lif_4k(steps=2000),
        "cuba_ragged": W.cuba_lif_4k(n_exc=777, n_inh=190, p=0.05, steps=600),
        "brunel_d15": W.brunel_fixed_out(n=3000, k=300, delay_steps=15, steps=400),
        "brunel_d4_ragged": W.brunel_fixed_out(n=1111, k=97, delay_steps=4, steps=300),
        "stdp_d10": W.stdp_er(n=2000, p=0.05, delay_steps=10, steps=400),
    }


@pytest.mark.parametrize("n_ext,rate", [(1000, 20.0), (1000, 10.0), (200, 200.0), (1, 10000.0), (0, 0.0)])
def test_drive_table_matches_oracle(n_ext, rate):
    spec = W.cuba_lif_4k(n_exc=64, n_inh=16)
    spec["params"].update(n_ext=n_ext, rate_ext_hz=rate, w_ext_mV=0.1)
    g = _net(spec)
    o = oracle.OracleNet(spec)
    assert np.array_equal(g.drive_table(), o.table())


@pytest.mark.parametrize("name", list(_small_specs()))
def test_generated_synapses_match_oracle(name):
    spec = _small_specs()[name]
    print(f"[gen] {name}", flush=True)
    g = _net(spec)
    o = oracle.OracleNet(spec)
    rp, col, w = g.synapses()
    assert np.array_equal(rp, o.row_ptr())
    assert np.array_equal(col, o.col())
    if o.const.plastic:
        assert np.array_equal(_bits(w), _bits(o.w_f32()))
    else:
        assert np.array_equal(w, o.w_q16())


@pytest.mark.parametrize("k", [4095, 4096, 5102, 5103, 5104, 5120, 6001, 12000])
def test_long_fixed_rows_match_oracle(k):
    """Networks of fixed out-degree projections only, with rows from just below the
    length where a workgroup shares each row (4,096 targets) to rows past a wavefront's
    own gap cache (5,104 gaps): every row byte-identical."""
    spec = W.brunel_fixed_out(n=max(6400, k + 400), k=k, delay_steps=3, steps=10)
    print(f"[gen] fixed out-degree k={k}", flush=True)
    g = _net(spec, raster_steps=16)
    o = oracle.OracleNet(spec)
    rp, col, _ = g.synapses()
    assert np.array_equal(rp, o.row_ptr())
    assert np.array_equal(col, o.col())
    i = g.info()
    assert i["build_ms"] > 0 and i["gen_fill_ms"] > 0 and i["gen_rows_ms"] > 0 and i["index_ms"] >= 0


def test_rows_of_several_fixed_projections():
    """Rows made of several fixed out-degree segments filled by workgroups: excitatory
    rows hold 4,500 targets among the excitatory neurons, then 37 among the inhibitory
    ones (shorter than the four wavefronts), then 4,100 among both populations."""
    spec = W.brunel_fixed_out(n=7500, k=4100, delay_steps=3, steps=10)
    spec["projs"] = [
        {"from": 0, "to": 0, "to_span": 1, "kind": "fixed", "p": 0.0, "k": 4500, "w_mV": 0.1, "plastic": 0},
        {"from": 0, "to": 1, "to_span": 1, "kind": "fixed", "p": 0.0, "k": 37, "w_mV": 0.1, "plastic": 0},
        {"from": 1, "to": 0, "to_span": 2, "kind": "fixed", "p": 0.0, "k": 4100, "w_mV": -0.5, "plastic": 0}]
    print("[gen] several fixed segments per row", flush=True)
    g = _net(spec, raster_steps=16)
    o = oracle.OracleNet(spec)
    rp, col, _ = g.synapses()
    assert np.array_equal(rp, o.row_ptr())
    assert np.array_equal(col, o.col())


@pytest.mark.parametrize("k", [4500, 5300])
def test_fixed_rows_beside_er_projections(k):
    """A network with an ER projection besides its fixed out-degree ones keeps one
    wavefront per row; at k = 5,300 its rows also pass the wavefront's gap cache."""
    spec = W.brunel_fixed_out(n=8000, k=k, delay_steps=3, steps=10)
    spec["projs"][1]["to_span"] = 1  # inhibitory rows: k fixed targets among the excitatory
    spec["projs"].append({"from": 1, "to": 1, "to_span": 1, "kind": "er", "p": 0.05, "k": 0,
                          "w_mV": -0.2, "plastic": 0})
    print(f"[gen] fixed k={k} with an ER projection", flush=True)
    g = _net(spec, raster_steps=16)
    o = oracle.OracleNet(spec)
    rp, col, _ = g.synapses()
    assert np.array_equal(rp, o.row_ptr())
    assert np.array_equal(col, o.col())


def test_spacing_gaps_on_every_input():
    """The fill's gap evaluation (a table estimate, the defined binary64 logarithm where
    the estimate is near an integer) against the oracle's gaps (Fig. 2, step (b)) on all
    2^24 distinct inputs; the word's low 8 bits, which the definition drops, vary."""
    import ctypes as C
    import torch
    from paper_1912_07423_amd import _lib as L
    j = np.arange(1 << 24, dtype=np.uint32)
    words = (j << np.uint32(8)) | (j * np.uint32(2654435761) >> np.uint32(24))
    S, _ = oracle.spacing_core((j.astype(np.float64) + 1.0) * 2.0 ** -24, spare=0)
    want = np.diff(S).astype(np.uint32)
    assert want.max() < (1 << 29) and want[-1] == 0
    d_words = torch.from_numpy(words.view(np.int32)).cuda()
    d_gaps = torch.full((1 << 24,), -1, dtype=torch.int32, device="cuda")
    lib = L.load()
    st = lib.snn_spacing_gaps(C.c_void_p(d_words.data_ptr()), 1 << 24, C.c_void_p(d_gaps.data_ptr()),
                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.SNN_OK
    got = d_gaps.cpu().numpy().view(np.uint32)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} gaps differ, first at j = {bad[:5]}: {got[bad[:5]]} vs {want[bad[:5]]}"
    # a ragged count, and n = 0 with NULL pointers
    d_gaps.fill_(-1)
    st = lib.snn_spacing_gaps(C.c_void_p(d_words.data_ptr()), 1001, C.c_void_p(d_gaps.data_ptr()),
                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    got = d_gaps.cpu().numpy().view(np.uint32)
    assert st == L.SNN_OK and np.array_equal(got[:1001], want[:1001]) and np.all(got[1001:] == 0xFFFFFFFF)
    assert lib.snn_spacing_gaps(None, 0, None, None) == L.SNN_OK
    assert lib.snn_spacing_gaps(None, 5, C.c_void_p(d_gaps.data_ptr()), None) == L.SNN_E_INVALID


@pytest.mark.parametrize("name", list(_small_specs()))
def test_initial_state_matches_oracle(name):
    spec = _small_specs()[name]
    g = _net(spec)
    o = oracle.OracleNet(spec)
    s = g.state()
    assert np.array_equal(_bits(s["v"]), _bits(o.v()))
    assert not s["ref"].any() and not s["input"].any()


@pytest.mark.parametrize("name", list(_small_specs()))
def test_raster_and_state_parity(name):
    spec = _small_specs()[name]
    print(f"[run] {name} steps={spec['steps']}", flush=True)
    rg, inf = _compare_run(spec, spec["steps"])
    print(f"[run] {name}: spikes={int(np.unpackbits(rg.view(np.uint8)).sum())} "
          f"events={inf['events']} delivery={inf['delivery']} window={inf['window']}", flush=True)
    assert rg.any()


@pytest.mark.parametrize("delivery,window", [("atomic", 1), ("atomic", 7), ("atomic", 15),
                                             ("tiled", 1), ("tiled", 6), ("tiled", 15)])
def test_schedule_variants_identical(delivery, window):
    spec = W.brunel_fixed_out(n=2500, k=250, delay_steps=15, steps=200)
    print(f"[variant] {delivery} window={window}", flush=True)
    _compare_run(spec, 200, delivery=delivery, window=window)


@pytest.mark.parametrize("delay", [20, 40, 64])
def test_tiled_long_windows(delay):
    """Windows of 17 to 64 steps (64 is the longest): the tile schedule's search then
    scores each candidate bound over 32 or 64 lanes, one per step."""
    spec = W.brunel_fixed_out(n=3000, k=300, delay_steps=delay, steps=400)
    print(f"[window] tiled, d = window = {delay}", flush=True)
    _, inf = _compare_run(spec, 400, delivery="tiled", window=delay)
    assert inf["window"] == delay and inf["delivery"] == 2


def test_tiled_tile_counts():
    spec = W.brunel_fixed_out(n=2500, k=250, delay_steps=15, steps=120)
    for tiles in (1, 3, 17, 39, 120):
        print(f"[tiles] {tiles}", flush=True)
        _, inf = _compare_run(spec, 120, delivery="tiled", tiles=tiles)
        assert inf["tile_offset_bytes"] == 2


def test_tiled_wide_tile_offsets():
    """A 66,000-neuron population as an ER target: a row may then reach 65,536
    synapses, so the tile boundaries are stored as 4-byte offsets."""
    spec = W.cuba_lif_4k(n_exc=66_000, n_inh=4_000, p=0.001, steps=100)
    print("[tiles] 4-byte boundaries, n=70000", flush=True)
    rg, inf = _compare_run(spec, 100, delivery="tiled", tiles=70)
    assert inf["tile_offset_bytes"] == 4 and inf["tiles"] == 70
    assert rg.any()


def test_step_by_step_equals_graph_run():
    spec = W.brunel_fixed_out(n=2000, k=150, delay_steps=3, steps=300)
    a = _net(spec, raster_steps=300)
    b = _net(spec, raster_steps=300)
    a.run(300)                       # graph replays + eager remainder
    for _ in range(300):
        b.step()                     # one-step windows
    assert np.array_equal(a.raster_bits(0, 300), b.raster_bits(0, 300))
    assert np.array_equal(_bits(a.state()["v"]), _bits(b.state()["v"]))
    assert a.events == b.events


def test_ping_pong_listing1_gpu():
    spec = {"params": W.params(tau_m_ms=1e12, v_rest_mV=0.0, v_bg_mV=0.0, v_th_mV=0.5,
                               v_reset_mV=0.0, t_ref_ms=0.0, v0_lo_mV=0.0, v0_hi_mV=0.0,
                               delay_steps=1, seed=21),
            "pops": [{"size": 100, "excitatory": 1}, {"size": 100, "excitatory": 1}],
            "projs": [{"from": 0, "to": 1, "kind": "er", "p": 0.03, "w_mV": 1.0},
                      {"from": 1, "to": 0, "kind": "er", "p": 0.03, "w_mV": 1.0}]}
    g = _net(spec, raster_steps=30)
    o = oracle.OracleNet(spec, raster_cap=30)
    v0 = np.zeros(200, np.float32)
    v0[:100] = 1.0
    g.set_state(v=v0)
    o.v()[:] = v0
    g.run(30)
    o.run(30)
    assert np.array_equal(g.raster_bits(0, 30), o.raster_words()[:30])
    assert g.raster(0, 30)[29].any()


def test_fifo_single_spike_gpu():
    D, t0 = 5, 7
    spec = W.ei_er(40, 10, 0.2, 0.1, -0.1, delay_steps=D, tau_m_ms=1e6, v_bg_mV=0.0,
                   v0_lo_mV=-60.0, v0_hi_mV=-60.0, seed=5)
    g = _net(spec, raster_steps=64)
    o = oracle.OracleNet(spec, raster_cap=64)
    g.run(t0)
    o.run(t0)
    v = g.state()["v"]
    v[3] = -40.0
    g.set_state(v=v)
    o.v()[3] = -40.0
    g.run(2 * D + 3)
    o.run(2 * D + 3)
    assert np.argwhere(g.raster(0, t0 + 2 * D + 3)).tolist() == [[t0, 3]]
    assert np.array_equal(_bits(g.state()["v"]), _bits(o.v()))
    assert g.events == o.events == len(oracle.gen_row(spec, 3)[0])   # both delivered by now


def test_time_delivery_counts_events():
    spec = W.brunel_fixed_out(n=3000, k=200, delay_steps=15)
    for delivery in ("atomic", "tiled"):
        g = _net(spec, delivery=delivery)
        ids = np.arange(0, 3000, 7, dtype=np.uint32)
        ms, ev = g.time_delivery(ids, reps=3, steps=1)
        assert ev == 200 * len(ids) and ms > 0
        ms, ev = g.time_delivery(ids, reps=2, step_counts=[len(ids) - 50, 0, 50])
        assert ev == 200 * len(ids) and ms > 0
        assert g.t == 0 and g.events == 0


def test_invalid_parameters_rejected_gpu():
    from paper_1912_07423_amd import SnnError
    bad = W.brunel_fixed_out(n=50, k=50, delay_steps=1, n_ext=0)
    with pytest.raises(SnnError):
        _net(bad)
    bad = W.cuba_lif_4k(n_exc=10, n_inh=10)
    bad["params"]["delay_steps"] = 0
    with pytest.raises(SnnError):
        _net(bad)
    g = _net(W.cuba_lif_4k(n_exc=10, n_inh=10), raster_steps=4)
    g.run(10)
    with pytest.raises(SnnError):
        g.raster_bits(0, 10)          # no longer held by the 4-step ring
    with pytest.raises(SnnError):
        g.raster_bits(8, 12)          # beyond the simulated steps


@pytest.mark.parametrize("delivery", ["atomic", "tiled"])
@pytest.mark.parametrize("synapse_weights", ["auto", "per_synapse"])
def test_weight_layouts_identical(delivery, synapse_weights):
    """One weight per source population (4 B per synapse) and a weight per synapse give
    the oracle's results with either delivery kernel."""
    spec = W.brunel_fixed_out(n=2500, k=250, delay_steps=15, steps=200)
    print(f"[weights] {delivery} {synapse_weights}", flush=True)
    rg, inf = _compare_run(spec, 200, delivery=delivery, synapse_weights=synapse_weights)
    assert inf["source_weights"] == (1 if synapse_weights == "auto" else 0)


def test_mixed_weights_of_one_source_population_use_per_synapse_weights():
    spec = W.cuba_lif_4k(n_exc=900, n_inh=225, p=0.05, steps=400)
    spec["projs"][1]["w_mV"] = 0.5          # E->I differs from E->E
    rg, inf = _compare_run(spec, 400)
    assert inf["source_weights"] == 0
    assert rg.any()


def test_delivery_switched_between_windows_keeps_parity():
    """Changing the delivery variant and tiling between runs leaves the results equal
    to the oracle's (the input ring holds exactly the pending arrivals at a window
    boundary, whichever variant filled it)."""
    spec = W.brunel_fixed_out(n=2500, k=250, delay_steps=15, steps=150)
    g = _net(spec, raster_steps=150, delivery="tiled")
    g.run(45)
    g.set_delivery("atomic")
    g.run(45)
    g.set_delivery("tiled", tiles=7, block=1024, grid=64)
    g.run(30)
    g.set_delivery("auto")
    g.run(30)
    o = oracle.OracleNet(spec, raster_cap=150)
    o.run(150)
    assert np.array_equal(g.raster_bits(0, 150), o.raster_words()[:150])
    assert np.array_equal(_bits(g.state()["v"]), _bits(o.v()))


def test_autotune_delivery_keeps_state_and_parity():
    spec = W.brunel_fixed_out(n=4000, k=400, delay_steps=15, steps=150)
    g = _net(spec, raster_steps=150)
    g.run(60)
    before = g.state()
    t = g.autotune_delivery(reps=2)
    print(f"[autotune] {t}", flush=True)
    assert t["delivery"] in ("atomic", "tiled") and t["ms_per_launch"] > 0 and t["events_per_launch"] > 0
    after = g.state()
    assert np.array_equal(_bits(before["v"]), _bits(after["v"]))
    assert np.array_equal(before["input"], after["input"]) and g.t == 60
    g.run(90)
    o = oracle.OracleNet(spec, raster_cap=150)
    o.run(150)
    assert np.array_equal(g.raster_bits(0, 150), o.raster_words()[:150])
    assert np.array_equal(_bits(g.state()["v"]), _bits(o.v()))


def _plastic_specs():
    return {
        "d10": W.stdp_er(n=2000, p=0.05, delay_steps=10, steps=400),
        "d1_ragged": W.stdp_er(n=777, p=0.08, delay_steps=1, rate_hz=40.0, seed=23, steps=350),
        "d3_fast": W.stdp_er(n=600, p=0.1, delay_steps=3, rate_hz=400.0, n_ext=200, seed=21, steps=300),
        "d64": W.stdp_er(n=1000, p=0.05, delay_steps=64, rate_hz=40.0, seed=24, steps=400),
    }


@pytest.mark.parametrize("tiles", [0, 1, 7])
@pytest.mark.parametrize("name", list(_plastic_specs()))
def test_plastic_tiled_delivery(name, tiles):
    """Eager STDP with the tiled delivery (one step per launch): FP32 weights streamed in
    16-byte groups and rounded to Q16 as the atomic kernel rounds them, the traces
    advanced by the launch's extra workgroup.  Raster, V, traces, every weight and the
    touch count equal the oracle's."""
    spec = _plastic_specs()[name]
    print(f"[plastic tiled] {name} tiles={tiles}", flush=True)
    rg, inf = _compare_run(spec, spec["steps"], delivery="tiled", tiles=tiles)
    assert inf["delivery"] == 2 and inf["plastic"] and inf["touches"] > 0
    assert rg.any()


def test_plastic_delivery_switched_between_steps():
    """A plastic network switched from the atomic delivery (which adds into the input
    accumulator the update cleared) to the tiled one (which overwrites it) and back."""
    spec = W.stdp_er(n=2000, p=0.05, delay_steps=10, steps=300)
    g = _net(spec, raster_steps=300, delivery="atomic")
    g.run(100)
    g.set_delivery("tiled", tiles=5)
    assert g.info()["delivery"] == 2
    g.run(100)
    g.set_delivery("atomic")
    g.run(100)
    o = oracle.OracleNet(spec, raster_cap=300)
    o.run(300)
    _compare_net(g, o, 300)


def test_autotune_plastic_delivery_keeps_state_and_parity():
    """The autotuner on an eagerly plastic network times both deliveries (the tiled one
    with FP32 weights) on scratch buffers: weights, traces and the run that follows
    stay the oracle's."""
    spec = W.stdp_er(n=3000, p=0.05, delay_steps=10, steps=200)
    g = _net(spec, raster_steps=200)
    g.run(60)
    before = g.state(weights=True)
    t = g.autotune_delivery(reps=2)
    print(f"[autotune plastic] {t}", flush=True)
    assert t["delivery"] in ("atomic", "tiled") and t["ms_per_launch"] > 0 and t["events_per_launch"] > 0
    after = g.state(weights=True)
    for k in ("v", "x_pre", "x_post", "w_f32"):
        assert np.array_equal(_bits(before[k]), _bits(after[k])), k
    assert np.array_equal(before["input"], after["input"]) and g.t == 60
    g.run(140)
    o = oracle.OracleNet(spec, raster_cap=200)
    o.run(200)
    _compare_net(g, o, 200)


@pytest.mark.parametrize("delivery", ["atomic", "tiled"])
def test_network_without_synapses(delivery):
    """p = 0: every row is empty; the drive alone makes the neurons fire."""
    spec = W.cuba_lif_4k(n_exc=700, n_inh=190, p=0.0, steps=200)
    spec["params"].update(n_ext=500, rate_ext_hz=40.0, w_ext_mV=0.4)
    print(f"[edge] no synapses, {delivery}", flush=True)
    rg, inf = _compare_run(spec, 200, delivery=delivery)
    assert inf["nnz"] == 0 and rg.any() and inf["events"] == 0


@pytest.mark.parametrize("delivery", ["atomic", "tiled"])
def test_delay_of_one_step(delivery):
    """d = 1: one-step windows, every spike delivered by the very next update."""
    spec = W.brunel_fixed_out(n=1500, k=120, delay_steps=1, steps=300)
    print(f"[edge] d = 1, {delivery}", flush=True)
    _, inf = _compare_run(spec, 300, delivery=delivery)
    assert inf["window"] == 1


def test_two_single_neuron_populations():
    """The smallest network: two populations of one neuron, all-to-all between them."""
    spec = W.cuba_lif_4k(n_exc=1, n_inh=1, p=1.0, steps=300)
    spec["params"].update(n_ext=50, rate_ext_hz=500.0, w_ext_mV=0.6)
    print("[edge] 1 + 1 neurons", flush=True)
    rg, inf = _compare_run(spec, 300)
    assert inf["nnz"] == 2


@pytest.mark.parametrize("n", [400, 4500])
def test_fixed_out_degree_to_every_other_neuron(n):
    """K = n - 1 over all n neurons: no spare slot, every row is every other neuron
    (the spacing generator's degenerate case); at n = 4,500 a workgroup shares each row."""
    spec = W.brunel_fixed_out(n=n, k=n - 1, delay_steps=3, steps=150)
    print(f"[edge] K = n - 1, n = {n}", flush=True)
    g = _net(spec)
    o = oracle.OracleNet(spec)
    rp, col, _ = g.synapses()
    assert np.array_equal(rp, o.row_ptr())
    assert np.array_equal(col, o.col())
    _compare_run(spec, 150)


def test_memory_cache_reuses_blocks_with_identical_results():
    """Without torch's allocator, device memory comes from the library's cache: after a
    network is destroyed its blocks are kept, a rebuild of the same spec is served from
    them entirely (no hipMalloc), and the run on reused memory is the oracle's."""
    from paper_1912_07423_amd import memory_cache_release, memory_cache_stats
    spec = W.brunel_fixed_out(n=3000, k=300, delay_steps=15, steps=200)
    memory_cache_release()
    assert memory_cache_stats()["bytes"] == 0
    a = _net(spec, torch_memory=False, raster_steps=200)
    a.run(200)
    first = a.raster_bits(0, 200)
    held = a.info()["device_bytes"]
    a.close()
    st0 = memory_cache_stats()
    assert st0["bytes"] >= held and st0["blocks"] > 0
    b = _net(spec, torch_memory=False, raster_steps=200)
    st1 = memory_cache_stats()
    assert st1["misses"] == st0["misses"] and st1["hits"] >= st0["hits"] + st0["blocks"]
    assert st1["bytes"] == 0
    o = oracle.OracleNet(spec, raster_cap=200)
    b.run(200)
    o.run(200)
    from gpu_compare import compare_net
    compare_net(b, o, 200)
    assert np.array_equal(b.raster_bits(0, 200), first)
    b.close()
    memory_cache_release()
    assert memory_cache_stats()["bytes"] == 0
