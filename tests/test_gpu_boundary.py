"""The C ABI's contracts on the GPU (include/snn.h): the timestamped spike download as
sorted (step, id) pairs against the oracle's raster, its required-count contract on
overflow and its range checks, allocator failure reported as SNN_E_OOM with every block
handed back, and a refused delivery reconfiguration that leaves the network running as
before."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1912_07423_amd import _lib as L
from paper_1912_07423_amd import workloads as W
from gpu_compare import bits, compare_net, net as _net

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    return gpu_available


def _oracle_pairs(o, t0, t1):
    """(steps, ids) of the oracle's raster rows [t0, t1), sorted by step then id."""
    t, i = np.nonzero(o.raster_bool(t0, t1))
    return (t + t0).astype(np.uint32), i.astype(np.uint32)


def _get_raster(g, t0, t1, cap, steps=None, ids=None):
    n = C.c_uint64(12345)
    st = g._lib.snn_get_raster(g._h, t0, t1, None if steps is None else C.c_void_p(steps.ctypes.data),
                               None if ids is None else C.c_void_p(ids.ctypes.data), cap, C.byref(n))
    return st, n.value


def test_spike_download_cuba_4k_10000_steps():
    spec = W.cuba_lif_4k()
    T = spec["steps"]
    print(f"[raster] cuba_lif_4k {T} steps", flush=True)
    g = _net(spec, raster_steps=T)
    o = oracle.OracleNet(spec, raster_cap=T)
    g.run(T)
    o.run(T)
    steps, ids = g.spikes(0, T)
    ws, wi = _oracle_pairs(o, 0, T)
    assert len(steps) > 10_000
    assert np.array_equal(steps, ws) and np.array_equal(ids, wi)
    # sorted by step, then by id, and every pair a spike of the bit raster
    key = steps.astype(np.uint64) * (1 << 32) + ids
    assert np.all(np.diff(key.astype(np.int64)) > 0)
    # a sub-range is the matching slice
    s2, i2 = g.spikes(4321, 4400)
    sel = (ws >= 4321) & (ws < 4400)
    assert np.array_equal(s2, ws[sel]) and np.array_equal(i2, wi[sel])
    # an empty range
    s3, i3 = g.spikes(500, 500)
    assert len(s3) == 0 and len(i3) == 0


def test_spike_download_brunel_window():
    """One 15-step window of a delayed, driven network (20,000 neurons, out-degree 1,000,
    tiled delivery) after 300 steps."""
    spec = W.brunel_fixed_out(n=20_000, k=1000, delay_steps=15, steps=315)
    g = _net(spec, raster_steps=64, delivery="tiled")
    o = oracle.OracleNet(spec, raster_cap=64)
    g.run(315)
    o.run(315)
    steps, ids = g.spikes(300, 315)
    ws, wi = _oracle_pairs(o, 300, 315)
    assert len(steps) > 0
    assert np.array_equal(steps, ws) and np.array_equal(ids, wi)
    assert np.array_equal(bits(g.state()["v"]), bits(o.v()))


def test_spike_download_overflow_reports_required_count():
    spec = W.cuba_lif_4k(steps=300)
    g = _net(spec, raster_steps=300)
    g.run(300)
    st, need = _get_raster(g, 0, 300, 0)
    assert st == L.SNN_E_OVERFLOW and need > 0
    steps = np.full(need, 0xFFFFFFFF, np.uint32)
    ids = np.full(need, 0xFFFFFFFF, np.uint32)
    st, n = _get_raster(g, 0, 300, need - 1, steps, ids)
    assert st == L.SNN_E_OVERFLOW and n == need
    assert np.all(steps == 0xFFFFFFFF) and np.all(ids == 0xFFFFFFFF), "nothing is written on overflow"
    st, n = _get_raster(g, 0, 300, need, steps, ids)
    assert st == L.SNN_OK and n == need
    o = oracle.OracleNet(spec, raster_cap=300)
    o.run(300)
    ws, wi = _oracle_pairs(o, 0, 300)
    assert np.array_equal(steps, ws) and np.array_equal(ids, wi)


def test_spike_download_rejects_ranges_outside_the_ring():
    g = _net(W.cuba_lif_4k(steps=200), raster_steps=64)
    g.run(200)
    buf = np.zeros(1 << 16, np.uint32)
    for t0, t1 in ((150, 140),      # t_end < t_begin
                   (190, 201),      # past the simulated steps
                   (100, 150),      # no longer held by the 64-step ring
                   (135, 200)):     # one step too old: the ring holds [136, 200)
        st, _ = _get_raster(g, t0, t1, len(buf), buf, buf.copy())
        assert st == L.SNN_E_INVALID, (t0, t1)
    st, n = _get_raster(g, 136, 200, len(buf), buf, buf.copy())   # the oldest step held
    assert st == L.SNN_OK
    if n:
        st, _ = _get_raster(g, 136, 200, len(buf), None, None)
        assert st == L.SNN_E_INVALID, "NULL outputs while the range holds spikes"
    st, n = _get_raster(g, 137, 137, 0, None, None)
    assert st == L.SNN_OK and n == 0


class _CountingAllocator:
    """Device memory from torch's caching allocator, failing every request from the
    `fail_at`-th on; records what is outstanding."""

    def __init__(self, fail_at):
        import torch
        self.fail_at, self.calls, self.live = fail_at, 0, {}
        dev = torch.cuda.current_device()

        def _alloc(nbytes, s, ctx):
            self.calls += 1
            if self.calls >= self.fail_at:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), dev)
            self.live[p] = int(nbytes)
            return p

        def _free(ptr, nbytes, s, ctx):
            assert self.live.pop(ptr) == int(nbytes)
            torch.cuda.caching_allocator_delete(ptr)

        self.fns = (L.ALLOC_FN(_alloc), L.FREE_FN(_free))
        self.struct = L.Allocator(self.fns[0], self.fns[1], None)


@pytest.mark.parametrize("fail_at", [1, 2, 5, 12, 19])
def test_allocator_failure_is_oom_and_releases_everything(fail_at):
    from paper_1912_07423_amd.network import _structs
    spec = W.brunel_fixed_out(n=3000, k=200, delay_steps=15)
    p, pops, projs, n_projs = _structs(spec, raster_steps=64)
    a = _CountingAllocator(fail_at)
    lib = L.load()
    h = C.c_void_p()
    st = lib.snn_build_network(C.byref(p), pops, len(spec["pops"]), projs, n_projs, C.byref(a.struct),
                               None, C.byref(h))
    assert st == L.SNN_E_OOM, st
    assert not h.value
    assert b"NULL" in lib.snn_last_error(None)
    assert a.calls == fail_at and a.live == {}, "every block taken before the failure is handed back"


def test_refused_delivery_change_keeps_the_network_usable():
    """A configuration with an impossible workgroup size is refused, on an atomic and on
    a tiled network; each keeps reporting and running the delivery it had (the tiled one
    with its own tile index), with the oracle's results."""
    from paper_1912_07423_amd import SnnError
    spec = W.brunel_fixed_out(n=2500, k=250, delay_steps=15, steps=150)
    g = _net(spec, raster_steps=150, delivery="atomic")
    g.run(30)
    with pytest.raises(SnnError):
        g.set_delivery("tiled", block=300)
    inf = g.info()
    assert inf["delivery"] == 1 and inf["tiles"] == 1 and inf["tile_offset_bytes"] == 0
    assert inf["target_bytes"] == 4
    g.run(45)
    g.set_delivery("tiled", tiles=7, block=512)
    g.run(30)
    held = g.info()["device_bytes"]
    with pytest.raises(SnnError):
        g.set_delivery("tiled", tiles=3, block=300)
    inf = g.info()
    assert inf["delivery"] == 2 and inf["tiles"] == 7 and inf["tile_offset_bytes"] == 2
    assert inf["device_bytes"] == held
    g.run(45)
    o = oracle.OracleNet(spec, raster_cap=150)
    o.run(150)
    compare_net(g, o, 150)
