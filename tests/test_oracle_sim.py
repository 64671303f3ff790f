"""Pins of the oracle's simulation against closed forms, dense brute force and the
paper's ping-pong example (Sec. III-A.1, Fig. 1, Listing 1)."""
import math

import numpy as np
import pytest

import oracle
from paper_1912_07423_amd import workloads as W


def _single_pop(n, **prm):
    p = W.params(**prm)
    return {"params": p, "pops": [{"size": n, "excitatory": 1}], "projs": []}


def _dense_q16(net):
    """W[i, j] = Q16 weight of edge i->j (int64), from the oracle's CSR."""
    n = net.n
    rp = net.row_ptr().astype(np.int64)
    dense = np.zeros((n, n), dtype=np.int64)
    w = net.w_q16() if net.const.plastic == 0 else None
    col = net.col()
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            dense[i, col[e]] += w[e]
    return dense


def test_closed_form_lif_silent():
    """No input (the literal 4,000-neuron configuration with zero background): every
    neuron relaxes as V_k = V_inf + (V_0 - V_inf) alpha^k.  binary32 rounding adds at
    most ~1.5 ulp(|V|) per step, damped geometrically: |err| <= 1.5 ulp / (1 - alpha)."""
    spec = W.cuba_lif_4k(v_bg_mV=0.0, steps=3000)
    net = oracle.OracleNet(spec, raster_cap=8)
    v0 = net.v().astype(np.float64).copy()
    alpha = float(np.float32(net.const.alpha))
    assert alpha == float(np.float32(math.exp(-0.1 / 20.0)))
    net.run(3000)
    v_inf = -60.0
    expect = v_inf + (v0 - v_inf) * alpha ** 3000
    bound = 1.5 * 2.0**-18 / (1 - alpha)
    assert np.max(np.abs(net.v() - expect)) <= bound
    assert net.events == 0 and np.all(net.input() == 0) and np.all(net.ref() == 0)


def test_closed_form_constant_input_is_added_before_leak():
    """p_ext = 1 makes the drive k = n_ext each step, i.e. a constant input c.  With the
    input added before the leak, V* = V_inf + c alpha / (1 - alpha) and
    V_k = V* + (V_0 - V*) alpha^k (leak-then-add would give V_inf + c / (1 - alpha))."""
    spec = _single_pop(64, n_ext=1, rate_ext_hz=10000.0, w_ext_mV=0.025, v0_lo_mV=-60.0,
                       v0_hi_mV=-52.0)
    net = oracle.OracleNet(spec)
    v0 = net.v().astype(np.float64).copy()
    alpha = float(net.const.alpha)
    c = 1638 * 2.0**-16                     # Q16 of 0.025 mV
    assert net.const.w_ext_q16 == 1638
    v_star = -60.0 + c * alpha / (1 - alpha)
    for k in (1, 10, 500, 2000):
        net.run(k - (net.t))
        expect = v_star + (v0 - v_star) * alpha ** k
        assert np.max(np.abs(net.v() - expect)) <= 1.5 * 2.0**-18 / (1 - alpha)
    assert net.events == 0


def _first_crossing(alpha, v_inf, v_start, v_th):
    k, v = 0, v_start
    while True:
        k += 1
        v = v_inf + (v_start - v_inf) * alpha ** k
        if v >= v_th:
            return k, v


def test_tonic_firing_period_with_refractoriness():
    """A lone neuron above threshold asymptote fires periodically: from V_reset it needs
    k updates to cross V_th, then holds for t_ref/dt = 50 steps and integrates again
    at the 51st step after its spike."""
    spec = _single_pop(1, v_bg_mV=11.0, v0_lo_mV=-60.0, v0_hi_mV=-60.0)
    net = oracle.OracleNet(spec, raster_cap=5000)
    alpha = float(net.const.alpha)
    k, v_cross = _first_crossing(alpha, -49.0, -60.0, -50.0)
    # margins so that binary32 rounding cannot move the crossing
    assert v_cross - (-50.0) > 1e-3
    assert -50.0 - (-49.0 - 11.0 * alpha ** (k - 1)) > 1e-3
    assert net.const.ref_steps == 50
    net.run(5000)
    spikes = np.nonzero(net.raster_bool(0, 5000)[:, 0])[0]
    period = 50 + k
    assert list(spikes) == list(range(k - 1, 5000, period))


def test_drive_statistics():
    """Binomial(n_ext, rate dt) virtual inputs per step: with alpha = 1, V_inf = 0 and
    w_ext = 2^-16 mV, V accumulates exactly sum_t k_t * 2^-16."""
    n, steps = 2000, 100
    spec = _single_pop(n, n_ext=1000, rate_ext_hz=20.0, w_ext_mV=2.0**-16, tau_m_ms=1e12,
                       v_rest_mV=0.0, v_bg_mV=0.0, v0_lo_mV=0.0, v0_hi_mV=0.0, v_th_mV=1e9)
    net = oracle.OracleNet(spec)
    assert net.const.alpha == 1.0
    net.run(steps)
    k = net.v().astype(np.float64) * 2**16
    assert np.all(k == np.round(k))
    lam, var = 1000 * 0.002, 1000 * 0.002 * 0.998
    assert abs(k.mean() / steps - lam) < 5 * math.sqrt(var / (n * steps))
    per_neuron_var = k.var() / steps
    assert abs(per_neuron_var - var) < 0.15 * var


@pytest.mark.parametrize("delay", [1, 3])
def test_dense_bruteforce_propagation(delay):
    """Before every update the input accumulators equal the dense product
    I = W_q^T s_{t-D} (int64, wrapped to int32), and the event counter equals the sum
    of out-degrees of all delivered spikes."""
    spec = W.ei_er(240, 60, 0.1, 0.27, -1.0, delay_steps=delay, v_bg_mV=9.0, n_ext=200,
                   rate_ext_hz=200.0, w_ext_mV=0.5, seed=11)
    T = 400
    net = oracle.OracleNet(spec, raster_cap=T)
    dense = _dense_q16(net)
    outdeg = np.diff(net.row_ptr().astype(np.int64))
    events = 0
    n_spikes = 0
    for t in range(T):
        net.run(1)
        s = net.raster_bool(t, t + 1)[0]
        n_spikes += s.sum()
        src = t + 1 - delay
        if src >= 0:
            sv = net.raster_bool(src, src + 1)[0].astype(np.int64)
            expect = (sv @ dense).astype(np.int64)
            expect = ((expect + 2**31) % 2**32 - 2**31).astype(np.int32)
            events += int(outdeg[sv.astype(bool)].sum())
        else:
            expect = np.zeros(net.n, np.int32)
        assert np.array_equal(net.input(), expect), t
        assert net.events == events
    assert n_spikes > 200          # the network is active


def test_ping_pong_listing1():
    """Listing 1 as a LIF special case (alpha = 1, V_inf = 0, V_th = 0.5, V_reset = 0,
    w = 1 mV, no refractoriness, D = 1): the first population starts at V = 1, and
    the set that spikes at t+1 is exactly the set of targets of the spikes at t."""
    spec = {"params": W.params(tau_m_ms=1e12, v_rest_mV=0.0, v_bg_mV=0.0, v_th_mV=0.5,
                               v_reset_mV=0.0, t_ref_ms=0.0, v0_lo_mV=0.0, v0_hi_mV=0.0,
                               delay_steps=1, seed=21),
            "pops": [{"size": 100, "excitatory": 1}, {"size": 100, "excitatory": 1}],
            "projs": [{"from": 0, "to": 1, "kind": "er", "p": 0.03, "w_mV": 1.0},
                      {"from": 1, "to": 0, "kind": "er", "p": 0.03, "w_mV": 1.0}]}
    T = 30
    net = oracle.OracleNet(spec, raster_cap=T)
    net.v()[:100] = 1.0
    adj = _dense_q16(net) > 0
    net.run(T)
    r = net.raster_bool(0, T)
    assert np.array_equal(r[0], np.arange(200) < 100)
    for t in range(T - 1):
        assert np.array_equal(r[t + 1], adj[r[t]].any(axis=0)), t
    assert r[T - 1].any()


def test_fifo_single_spike_arrives_after_exactly_d_steps():
    """One injected spike at step t0 with D = 5: the input accumulators stay zero except
    after step t0 + D - 1 (delivery), when they hold exactly the spiker's row; the
    targets' potentials change only at the update of step t0 + D."""
    D, t0 = 5, 7
    spec = W.ei_er(40, 10, 0.2, 0.1, -0.1, delay_steps=D, tau_m_ms=1e6, v_bg_mV=0.0,
                   v0_lo_mV=-60.0, v0_hi_mV=-60.0, seed=5)
    net = oracle.OracleNet(spec, raster_cap=64)
    dense = _dense_q16(net)
    src = 3
    net.run(t0)
    net.v()[src] = -40.0
    history = []
    for t in range(t0, t0 + 2 * D + 3):
        v_before = net.v().copy()
        net.run(1)
        history.append((t, net.input().copy(), net.v() - v_before))
    r = net.raster_bool(0, t0 + 2 * D + 3)
    assert np.argwhere(r).tolist() == [[t0, src]]
    targets = dense[src] != 0
    assert targets.any()
    for t, inp, dv in history:
        if t == t0 + D - 1:
            assert np.array_equal(inp, dense[src].astype(np.int32))
        else:
            assert not inp.any()
        moved = (dv != 0)
        moved[src] = False
        if t == t0 + D:
            assert np.array_equal(moved, targets)
        else:
            assert not moved.any()
    assert net.events == int(targets.sum())


def _stdp_pair_spec(delay, w0=0.01, t_ref_ms=0.0):
    prm = W.params(delay_steps=delay, tau_m_ms=1e6, v_bg_mV=0.0, v0_lo_mV=-60.0,
                   v0_hi_mV=-60.0, t_ref_ms=t_ref_ms, tau_plus_ms=20.0, tau_minus_ms=15.0,
                   a_plus=0.01, a_minus=0.012, w_max_mV=0.5, seed=3)
    return {"params": prm, "pops": [{"size": 2, "excitatory": 1}],
            "projs": [{"from": 0, "to": 0, "kind": "er", "p": 1.0, "w_mV": w0, "plastic": 1}]}


def _run_with_forced_spikes(net, forced, T):
    """forced: {step: [neuron ids]}; the neurons are pushed above threshold right
    before the update of that step."""
    for t in range(T):
        for i in forced.get(t, []):
            net.v()[i] = -40.0
        net.run(1)


@pytest.mark.parametrize("t0,t1", [(10, 20), (10, 13), (10, 12), (10, 10), (20, 10), (30, 5)])
def test_stdp_pair_closed_form(t0, t1):
    """Neuron 0 fires at t0 and neuron 1 at t1, D = 3.  Synapse 0->1 sees its
    presynaptic event at arrival a = t0 + D: LTP A+ beta+^(t1-a) if t1 >= a, otherwise
    LTD -A- beta-^(a-t1).  Synapse 1->0 likewise with the roles swapped."""
    D, w0 = 3, 0.1
    net = oracle.OracleNet(_stdp_pair_spec(D, w0=w0), raster_cap=64)
    forced = {}
    forced.setdefault(t0, []).append(0)
    forced.setdefault(t1, []).append(1)
    _run_with_forced_spikes(net, forced, 60)
    r = net.raster_bool(0, 60)
    assert list(np.nonzero(r[:, 0])[0]) == [t0] and list(np.nonzero(r[:, 1])[0]) == [t1]
    bp, bm = float(net.const.beta_plus), float(net.const.beta_minus)
    ap, am = float(net.const.a_plus), float(net.const.a_minus)

    def dw(t_pre, t_post):
        a = t_pre + D
        return ap * bp ** (t_post - a) if t_post >= a else -am * bm ** (a - t_post)

    w = net.w_f32()          # row 0: edge 0->1, row 1: edge 1->0
    assert abs(w[0] - (w0 + dw(t0, t1))) <= 1e-6
    assert abs(w[1] - (w0 + dw(t1, t0))) <= 1e-6
    assert net.touches == 4


def test_stdp_clipping():
    net = oracle.OracleNet(_stdp_pair_spec(2, w0=0.001), raster_cap=64)
    _run_with_forced_spikes(net, {10: [1], 11: [0]}, 30)   # 0->1: post before arrival
    assert net.w_f32()[0] == 0.0                              # LTD larger than w, clipped
    net = oracle.OracleNet(_stdp_pair_spec(2, w0=0.499), raster_cap=64)
    _run_with_forced_spikes(net, {10: [0], 12: [1]}, 30)    # 0->1: post at arrival
    assert net.w_f32()[0] == np.float32(0.5)


def test_stdp_all_pairs_sum():
    """All-to-all traces: with no clipping the total change of a synapse is the sum over
    all (arrival a, post spike t) pairs of A+ beta+^(t-a) (t >= a) or -A- beta-^(a-t)."""
    D = 4
    pre = [5, 9, 30, 31, 50]
    post = [8, 12, 13, 33, 49, 60]
    net = oracle.OracleNet(_stdp_pair_spec(D, w0=0.25), raster_cap=128)
    forced = {}
    for t in pre:
        forced.setdefault(t, []).append(0)
    for t in post:
        forced.setdefault(t, []).append(1)
    _run_with_forced_spikes(net, forced, 80)
    bp, bm = float(net.const.beta_plus), float(net.const.beta_minus)
    ap, am = float(net.const.a_plus), float(net.const.a_minus)
    total = 0.0
    for tp in pre:
        a = tp + D
        for tq in post:
            total += ap * bp ** (tq - a) if tq >= a else -am * bm ** (a - tq)
    assert abs(net.w_f32()[0] - (0.25 + total)) <= 1e-5
