"""Seeded synthetic workloads: network descriptions as plain dicts.

This module holds only inputs -- population sizes, connection rules, physical
constants, seeds -- and no arithmetic of the simulation method.  The GPU library and
the CPU oracle each derive their own constants from these numbers.  It imports
nothing from the rest of the package.

The paper's benchmark models (Vogels-Abbott, Brunel, Brunel with STDP; Sec. IV) are
LIF networks of an excitatory and an inhibitory population (4:1).  The functions
below build networks of that shape at the sizes used for measurement.

Spec layout (shared by the library binding and the oracle wrapper):
    {"params": {dt_ms, delay_steps, n_ext, tau_m_ms, v_rest_mV, v_bg_mV, v_th_mV,
                v_reset_mV, t_ref_ms, v0_lo_mV, v0_hi_mV, rate_ext_hz, w_ext_mV,
                tau_plus_ms, tau_minus_ms, a_plus, a_minus, w_max_mV, seed},
     "pops":  [{"size", "excitatory"}, ...],
     "projs": [{"from", "to", "to_span", "kind": "er"|"fixed", "p", "k", "w_mV",
                "plastic"}, ...],
     "steps": number of simulation steps of the workload}
"""
import math

import numpy as np

LIF_DEFAULTS = dict(tau_m_ms=20.0, v_rest_mV=-60.0, v_bg_mV=0.0, v_th_mV=-50.0,
                    v_reset_mV=-60.0, t_ref_ms=5.0, v0_lo_mV=-60.0, v0_hi_mV=-50.0)
NO_STDP = dict(tau_plus_ms=20.0, tau_minus_ms=20.0, a_plus=0.0, a_minus=0.0, w_max_mV=0.0)


def params(**kw):
    p = dict(dt_ms=0.1, delay_steps=1, n_ext=0, rate_ext_hz=0.0, w_ext_mV=0.0, seed=1)
    p.update(LIF_DEFAULTS)
    p.update(NO_STDP)
    p.update(kw)
    return p


def ei_er(n_exc, n_inh, p, w_exc_mV, w_inh_mV, plastic_ee=False, **kw):
    """Two populations, Erdos-Renyi connectivity (no self-loops) between all four
    population pairs with one probability; weights set by the source population."""
    pops = [{"size": n_exc, "excitatory": 1}, {"size": n_inh, "excitatory": 0}]
    projs = []
    for a, w in ((0, w_exc_mV), (1, w_inh_mV)):
        for b in (0, 1):
            projs.append({"from": a, "to": b, "to_span": 1, "kind": "er", "p": p, "k": 0,
                          "w_mV": w, "plastic": int(plastic_ee and a == 0 and b == 0)})
    return {"params": params(**kw), "pops": pops, "projs": projs}


def cuba_lif_4k(v_bg_mV=11.0, seed=1, steps=10_000, n_exc=3200, n_inh=800, p=0.02):
    """Current-based LIF network of 4,000 neurons (3,200 exc. / 800 inh.), ER p=0.02,
    exc. weight +0.27 mV, inh. weight -4.5 mV, no delay (one step), dt 0.1 ms, 1 s of
    activity.  A constant background voltage drives the network (Vogels-Abbott style,
    Sec. IV); v_bg_mV = 0 gives the literal, silent configuration."""
    s = ei_er(n_exc, n_inh, p, 0.27, -4.5, v_bg_mV=v_bg_mV, seed=seed, delay_steps=1)
    s["steps"] = steps
    return s


def brunel_fixed_out(n=200_000, k=5000, delay_steps=15, rate_hz=20.0, n_ext=1000,
                     j_mV=0.1, g=5.0, seed=2, steps=1000):
    """Brunel-style network: 4:1 exc./inh., every neuron projects to exactly k targets
    drawn uniformly (without replacement, no self-loop) from all neurons; exc. weight
    J, inh. weight -gJ; uniform delay; independent Poisson drive of n_ext virtual
    inputs per neuron at rate_hz with weight J."""
    n_exc = (4 * n) // 5
    pops = [{"size": n_exc, "excitatory": 1}, {"size": n - n_exc, "excitatory": 0}]
    projs = [{"from": 0, "to": 0, "to_span": 2, "kind": "fixed", "p": 0.0, "k": k,
              "w_mV": j_mV, "plastic": 0},
             {"from": 1, "to": 0, "to_span": 2, "kind": "fixed", "p": 0.0, "k": k,
              "w_mV": -g * j_mV, "plastic": 0}]
    prm = params(delay_steps=delay_steps, n_ext=n_ext, rate_ext_hz=rate_hz, w_ext_mV=j_mV,
                 seed=seed)
    return {"params": prm, "pops": pops, "projs": projs, "steps": steps}


def stdp_er(n=100_000, p=0.02, delay_steps=10, rate_hz=10.0, n_ext=1000, seed=3, steps=2000,
            w_exc_mV=0.1, w_inh_mV=-0.5):
    """Plastic network: 4:1 exc./inh., ER p, FP32 weights (exc. 0.1 mV, inh. -0.5 mV),
    additive pair STDP on exc->exc synapses (tau+-=20 ms, A+=0.01, A-=0.012, clip
    [0, 0.5] mV), 1 ms delay, Poisson drive of 1,000 inputs at 10 Hz x 0.1 mV."""
    n_exc = (4 * n) // 5
    s = ei_er(n_exc, n - n_exc, p, w_exc_mV, w_inh_mV, plastic_ee=True,
              delay_steps=delay_steps, n_ext=n_ext, rate_ext_hz=rate_hz, w_ext_mV=0.1,
              tau_plus_ms=20.0, tau_minus_ms=20.0, a_plus=0.01, a_minus=0.012, w_max_mV=0.5,
              seed=seed)
    s["steps"] = steps
    return s


def eq1_scale(model, n):
    """Synaptic weight scale c of Eq. 1 (Sec. IV): 16e6 / N^2 for the Vogels model and
    20,000 / N for the Brunel model, so that both keep their firing regime when N grows
    (c = 1 at the models' original sizes of 4,000 and 20,000 neurons)."""
    if model == "vogels":
        return 16e6 / float(n) ** 2
    if model == "brunel":
        return 20000.0 / float(n)
    raise ValueError(model)


def vogels_scaled(n, steps=1000, seed=31):
    """The 4,000-neuron CUBA network grown to n neurons (4:1, ER p = 0.02) with its
    weights scaled by Eq. 1."""
    c = eq1_scale("vogels", n)
    n_exc = (4 * n) // 5
    s = ei_er(n_exc, n - n_exc, 0.02, 0.27 * c, -4.5 * c, v_bg_mV=11.0, seed=seed, delay_steps=1)
    s["steps"] = steps
    return s


def brunel_scaled(n, steps=1000, seed=32):
    """A Brunel network of n neurons (4:1) with fixed out-degree 0.1 n (uniform targets),
    J = 0.1 mV and g = 5 scaled by Eq. 1, a 1.5 ms delay and the 20 Hz Poisson drive."""
    s = brunel_fixed_out(n=n, k=max(1, n // 10), j_mV=0.1 * eq1_scale("brunel", n), seed=seed,
                         steps=steps)
    s["params"]["w_ext_mV"] = 0.1
    return s


def sweep(n_nets=512, seed=4, steps=5000, n_lo=1000, n_hi=20_000, p_lo=0.01, p_hi=0.05,
          w_lo=0.1, w_hi=0.4):
    """Independent CUBA LIF networks of uneven size for a parameter sweep: N
    log-uniform in [n_lo, n_hi], p uniform in [p_lo, p_hi], exc. weight uniform in
    [w_lo, w_hi] mV, inh. weight -4.5 mV, background 11 mV, one seed per network."""
    rng = np.random.default_rng(seed)
    u_n = rng.random(n_nets)
    u_p = rng.random(n_nets)
    u_w = rng.random(n_nets)
    seeds = rng.integers(1, 2**63 - 1, size=n_nets, dtype=np.int64)
    nets = []
    for m in range(n_nets):
        n = int(math.floor(n_lo * (n_hi / n_lo) ** u_n[m]))
        n_exc = (4 * n) // 5
        s = ei_er(n_exc, n - n_exc, float(p_lo + (p_hi - p_lo) * u_p[m]),
                  float(w_lo + (w_hi - w_lo) * u_w[m]), -4.5, v_bg_mV=11.0,
                  seed=int(seeds[m]), delay_steps=1)
        s["steps"] = steps
        nets.append(s)
    return nets


def bptt_inputs(batch=64, steps=250, n_in=700, n_hidden=1024, n_out=20, p_in=0.2, p_rec=0.1,
                rate_lo=0.0, rate_hi=50.0, dt_ms=1.0, seed=5):
    """Inputs of the surrogate-gradient recurrent SNN: Poisson input spike trains
    [batch, steps, n_in] (rates uniform in [rate_lo, rate_hi] Hz per channel), sparse
    ER masks for input->hidden (p_in) and hidden->hidden (p_rec, no self-loops),
    Gaussian weights N(0, 1/fan_in) on the masks, dense hidden->readout weights and
    random labels.  All arrays are numpy, from one seeded generator."""
    rng = np.random.default_rng(seed)
    rates = rng.uniform(rate_lo, rate_hi, size=n_in)
    prob = rates * dt_ms * 1e-3
    x = (rng.random((batch, steps, n_in)) < prob[None, None, :]).astype(np.float32)
    m_in = rng.random((n_in, n_hidden)) < p_in
    m_rec = rng.random((n_hidden, n_hidden)) < p_rec
    np.fill_diagonal(m_rec, False)
    fan_in = n_in * p_in + n_hidden * p_rec
    w_in = (rng.standard_normal((n_in, n_hidden)) / math.sqrt(fan_in)).astype(np.float32) * m_in
    w_rec = (rng.standard_normal((n_hidden, n_hidden)) / math.sqrt(fan_in)).astype(np.float32) * m_rec
    w_out = (rng.standard_normal((n_hidden, n_out)) / math.sqrt(n_hidden)).astype(np.float32)
    labels = rng.integers(0, n_out, size=batch)
    return {"x": x, "w_in": w_in.astype(np.float32), "mask_in": m_in,
            "w_rec": w_rec.astype(np.float32), "mask_rec": m_rec, "w_out": w_out,
            "labels": labels, "dt_ms": dt_ms}
