"""The delivery-timing entry point that allocates no device memory
(snn_time_delivery_static, include/snn.h) against the allocating one
(snn_time_delivery): the same events per launch on the same spike lists, for the tiled
and the atomic delivery, with explicit step counts and round-robin ids, on two calls in
a row (the second smaller), on a static and on an eagerly plastic network; the
network's own state untouched (a run afterwards still matches the oracle); a window too
large for the fixed array refused with SNN_E_INVALID."""
import numpy as np
import pytest

import oracle
from paper_1912_07423_amd import _lib as L
from paper_1912_07423_amd import workloads as W
from gpu_compare import compare_net, net as _net

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    return gpu_available


def _expected_events(row_ptr, ids):
    deg = np.diff(row_ptr.astype(np.int64))
    return int(deg[np.asarray(ids, dtype=np.int64)].sum())


def _spike_lists(n, steps, rng):
    """Two windows of spike ids: a busy one and a smaller one (fewer steps busy)."""
    big = [rng.choice(n, int(c), replace=False) for c in rng.integers(0, n // 4, steps)]
    small = [rng.choice(n, int(c), replace=False) for c in rng.integers(0, 40, steps)]
    return big, small


@pytest.mark.parametrize("delivery", ["tiled", "atomic"])
def test_static_scratch_matches_allocating_timing(delivery):
    spec = W.brunel_fixed_out(n=20_000, k=600, delay_steps=15, steps=60, seed=7)
    print(f"[no-alloc] brunel 20k k600 d15, {delivery}", flush=True)
    g = _net(spec, raster_steps=64, delivery=delivery)
    o = oracle.OracleNet(spec, raster_cap=64)
    assert g.info()["delivery_name"] == delivery
    row_ptr = g.synapses()[0]
    rng = np.random.default_rng(11)
    steps = g.info()["window"]
    for lists in _spike_lists(g.info()["n"], steps, rng):
        counts = np.array([len(x) for x in lists], dtype=np.uint32)
        ids = np.concatenate(lists).astype(np.uint32)
        want = _expected_events(row_ptr, ids)
        ms_a, ev_a = g.time_delivery(ids, reps=3, step_counts=counts)
        ms_s, ev_s = g.time_delivery_static(ids, reps=3, step_counts=counts)
        assert ev_a == ev_s == want
        assert ms_a > 0 and ms_s > 0
        # ids dealt round-robin over the steps
        ms_a, ev_a = g.time_delivery(ids, reps=2)
        ms_s, ev_s = g.time_delivery_static(ids, reps=2)
        assert ev_a == ev_s == want
    # an empty window
    ms_s, ev_s = g.time_delivery_static(np.zeros(0, np.uint32), reps=1)
    assert ev_s == 0
    # the network's own state is untouched: a run still matches the oracle bit for bit
    g.run(60)
    o.run(60)
    compare_net(g, o, 60)
    g.close()


@pytest.mark.parametrize("delivery", ["tiled", "atomic"])
def test_static_scratch_plastic_network(delivery):
    """An eagerly plastic network (one-step windows, FP32 weights): the same events as
    the allocating call, weights and traces untouched."""
    spec = W.stdp_er(n=3000, p=0.05, delay_steps=10, steps=80)
    print(f"[no-alloc] stdp 3k p0.05 d10, {delivery}", flush=True)
    g = _net(spec, raster_steps=80, delivery=delivery)
    assert g.info()["delivery_name"] == delivery and g.info()["window"] == 1
    g.run(40)
    before = g.state(weights=True)
    row_ptr = g.synapses()[0]
    rng = np.random.default_rng(13)
    for count in (400, 25):
        ids = rng.choice(g.info()["n"], count, replace=False).astype(np.uint32)
        want = _expected_events(row_ptr, ids)
        _, ev_a = g.time_delivery(ids, reps=2)
        _, ev_s = g.time_delivery_static(ids, reps=2)
        assert ev_a == ev_s == want
    after = g.state(weights=True)
    for k in ("v", "x_pre", "x_post", "w_f32"):
        assert np.array_equal(np.asarray(before[k]).view(np.uint32), np.asarray(after[k]).view(np.uint32)), k
    g.run(40)
    o = oracle.OracleNet(spec, raster_cap=80)
    o.run(80)
    compare_net(g, o, 80)
    g.close()


def test_static_scratch_rejects_oversized_window():
    # 15 input buffers of 1.2e6 neurons alone need 72 MB of the 64 MiB array
    spec = W.brunel_fixed_out(n=1_200_000, k=8, delay_steps=15, steps=15, seed=9)
    print("[no-alloc] brunel 1.2M k8 d15: oversized window", flush=True)
    g = _net(spec, raster_steps=16, delivery="atomic")
    ids = np.arange(100, dtype=np.uint32)
    with pytest.raises(L.SnnError, match="static scratch") as err:
        g.time_delivery_static(ids, reps=1)
    assert err.value.status == L.SNN_E_INVALID
    # the allocating form still serves it, and the static form still serves a smaller one
    _, ev = g.time_delivery(ids, reps=1)
    assert ev == 100 * 8
    small = _net(W.brunel_fixed_out(n=20_000, k=50, delay_steps=15, steps=15, seed=9), raster_steps=16)
    _, ev = small.time_delivery_static(ids, reps=1)
    assert ev == 100 * 50
    small.close()
    g.close()
