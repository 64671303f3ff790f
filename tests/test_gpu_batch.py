"""GPU parity of the batched form: every member of a batch, stepped by the persistent
batch kernel, against the oracle's run of the same network (raster, V, refractory
counters, pending Q16 inputs, event counts), for heterogeneous batches (sizes below
one wavefront, ragged sizes, delays 1-5, with and without Poisson drive), across
several run calls, for every launch shape the autotuner may pick, and at the full
sweep size: every one of the 512 networks after 5,000 steps."""
import numpy as np
import pytest

import oracle
from paper_1912_07423_amd import workloads as W
from gpu_compare import bits, compare_net

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    return gpu_available


def _mixed_specs():
    specs = [
        W.cuba_lif_4k(n_exc=800, n_inh=200, p=0.05, seed=11),
        W.cuba_lif_4k(n_exc=777, n_inh=190, p=0.03, seed=12),
        W.cuba_lif_4k(n_exc=50, n_inh=13, p=0.2, seed=13),          # one partial wavefront
        W.cuba_lif_4k(n_exc=3200, n_inh=800, p=0.02, seed=14),
        W.brunel_fixed_out(n=2000, k=100, delay_steps=3, seed=15),  # drive + delay ring
        W.brunel_fixed_out(n=1500, k=40, delay_steps=1, seed=16),
        W.brunel_fixed_out(n=999, k=250, delay_steps=5, rate_hz=30.0, seed=17),
        W.ei_er(300, 75, 0.1, 0.4, -4.5, v_bg_mV=11.0, delay_steps=2, seed=18),
    ]
    mixed = W.ei_er(500, 125, 0.08, 0.3, -4.5, v_bg_mV=11.0, seed=19)
    mixed["projs"][1]["w_mV"] = 0.45         # a weight per synapse for this member
    specs.append(mixed)
    return specs


def _batch(specs, **kw):
    from paper_1912_07423_amd import Batch
    return Batch(specs, **kw)


def _check_members(b, specs, steps, which=None):
    for k in (range(len(specs)) if which is None else which):
        print(f"[batch] member {k} n={b.network(k).n}", flush=True)
        o = oracle.OracleNet(specs[k], raster_cap=steps)
        o.run(steps)
        compare_net(b.network(k), o, steps)


def test_batch_members_match_oracle_over_several_runs():
    specs = _mixed_specs()
    steps = 400
    b = _batch(specs, raster_steps=steps)
    for chunk in (1, 99, 300):
        b.run(chunk)
    b.sync()
    _check_members(b, specs, steps)
    assert all(b.network(k).t == steps for k in range(len(specs)))


@pytest.mark.parametrize("block,degree_div", [(256, 1), (512, 16), (1024, 4), (1024, 1)])
def test_batch_every_launch_shape_identical(block, degree_div):
    specs = _mixed_specs()[:5]
    b = _batch(specs, raster_steps=200)
    b.set_tuning(block, degree_div)
    t = b.tuning()
    assert t["block"] == block and t["degree_div"] == degree_div and t["per_lane"] * block >= 4000
    b.run(200)
    _check_members(b, specs, 200)


def test_autotune_leaves_state_unchanged():
    specs = _mixed_specs()
    b = _batch(specs, raster_steps=300)
    b.run(100)
    before = [b.network(k).state() for k in range(len(specs))]
    ev = [b.network(k).events for k in range(len(specs))]
    t = b.autotune(trial_steps=50)
    assert t["block"] in (256, 512, 1024) and t["ms_per_step"] > 0
    for k in range(len(specs)):
        s = b.network(k).state()
        assert np.array_equal(bits(s["v"]), bits(before[k]["v"]))
        assert np.array_equal(s["ref"], before[k]["ref"])
        assert np.array_equal(s["input"], before[k]["input"])
        assert b.network(k).events == ev[k] and b.network(k).t == 100
    b.run(200)
    _check_members(b, specs, 300)


def test_batch_member_equals_single_network_run():
    from paper_1912_07423_amd import Network
    specs = _mixed_specs()[4:6]
    b = _batch(specs, raster_steps=250)
    b.run(250)
    for k, spec in enumerate(specs):
        g = Network(spec, raster_steps=250)
        g.run(250)
        assert np.array_equal(b.network(k).raster_bits(0, 250), g.raster_bits(0, 250))
        assert np.array_equal(bits(b.network(k).state()["v"]), bits(g.state()["v"]))
        assert b.network(k).events == g.events


def test_batch_set_state_and_member_guards():
    from paper_1912_07423_amd import SnnError
    D, t0 = 3, 5
    spec = W.ei_er(40, 10, 0.2, 0.1, -0.1, delay_steps=D, tau_m_ms=1e6, v_bg_mV=0.0,
                   v0_lo_mV=-60.0, v0_hi_mV=-60.0, seed=5)
    b = _batch([spec, W.cuba_lif_4k(n_exc=100, n_inh=25)], raster_steps=64)
    m = b.network(0)
    with pytest.raises(SnnError):
        m.step()
    with pytest.raises(SnnError):
        m.run(3)
    b.run(t0)
    v = m.state()["v"]
    v[3] = -40.0
    m.set_state(v=v)
    o = oracle.OracleNet(spec, raster_cap=64)
    o.run(t0)
    o.v()[3] = -40.0
    b.run(2 * D + 3)
    o.run(2 * D + 3)
    assert np.argwhere(m.raster(0, t0 + 2 * D + 3)).tolist() == [[t0, 3]]
    assert np.array_equal(bits(m.state()["v"]), bits(o.v()))
    assert m.events == o.events == len(oracle.gen_row(spec, 3)[0])


def test_batch_rejects_what_it_cannot_run():
    from paper_1912_07423_amd import SnnError
    with pytest.raises(SnnError, match="member 1"):
        _batch([W.cuba_lif_4k(n_exc=80, n_inh=20), W.stdp_er(n=500, p=0.05)])
    with pytest.raises(SnnError, match="member 0"):
        _batch([W.cuba_lif_4k(n_exc=20000, n_inh=5000, p=0.001)])
    with pytest.raises(SnnError):
        _batch([])


def _compare_member(g, o, steps):
    """One batch member against the oracle's run of its network, both advanced by
    `steps` steps from step 0: every raster row, V bit for bit, refractory counters,
    the pending Q16 input and the event count (with delay 1 both have delivered every
    spike emitted before the last step)."""
    inf = g.info()
    assert inf["t"] == steps and inf["input_buffers"] == 1
    rg = g.raster_bits(0, steps)
    ro = o.raster_words()[:steps]
    if not np.array_equal(rg, ro):
        bad = np.nonzero((rg != ro).any(axis=1))[0]
        raise AssertionError(f"raster differs first at step {bad[0]} ({len(bad)} steps differ)")
    s = g.state()
    assert np.array_equal(bits(s["v"]), bits(o.v()))
    assert np.array_equal(s["ref"], o.ref())
    assert np.array_equal(s["input"][0], o.input())
    assert inf["events"] == o.events
    return int(np.unpackbits(rg.view(np.uint8)).sum())


def test_sweep_512_networks_5000_steps_every_member():
    """The full parameter sweep in the benchmarked launch configuration (autotuned, one
    persistent launch per run): all 512 networks after 5,000 steps against the oracle's
    runs, one network per host thread, each compared as soon as its run ends."""
    import os
    from concurrent.futures import ThreadPoolExecutor, as_completed
    specs = W.sweep()
    steps = specs[0]["steps"]
    print(f"[sweep] building {len(specs)} networks", flush=True)
    b = _batch(specs, raster_steps=steps)
    t = b.autotune(trial_steps=100)
    print(f"[sweep] tuning {t}", flush=True)
    b.run(steps)
    b.sync()

    def oracle_run(k):
        o = oracle.OracleNet(specs[k], raster_cap=steps)
        o.run(steps)
        return k, o

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    done, spikes = 0, 0
    with ThreadPoolExecutor(workers) as ex:
        futs = [ex.submit(oracle_run, k) for k in range(len(specs))]
        for f in as_completed(futs):
            k, o = f.result()
            try:
                spikes += _compare_member(b.network(k), o, steps)
            except AssertionError as e:
                raise AssertionError(f"member {k} (n={b.network(k).n}): {e}") from None
            finally:
                o.close()
            done += 1
            if done % 64 == 0:
                print(f"[sweep] {done}/{len(specs)} members identical", flush=True)
    total_events = sum(b.network(k).events for k in range(len(specs)))
    print(f"[sweep] all {len(specs)} members identical: {spikes} spikes, {total_events} events", flush=True)
    assert done == len(specs) and spikes > 0 and total_events > 0
