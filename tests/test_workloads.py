"""Input recipes (no GPU): the Eq. 1 weight scaling of Sec. IV, the sweep table's ranges,
and the spec structure every builder expects."""
import math

import numpy as np
import pytest

from paper_1912_07423_amd import workloads as W


def test_eq1_scale_is_one_at_the_original_sizes_and_follows_the_equation():
    assert W.eq1_scale("vogels", 4000) == 1.0
    assert W.eq1_scale("brunel", 20000) == 1.0
    assert W.eq1_scale("vogels", 8000) == pytest.approx(0.25)
    assert W.eq1_scale("brunel", 200000) == pytest.approx(0.1)
    with pytest.raises(ValueError):
        W.eq1_scale("other", 10)


def test_scaled_networks_carry_the_scaled_weights():
    v = W.vogels_scaled(16000)
    c = 16e6 / 16000 ** 2
    assert [p["w_mV"] for p in v["projs"]] == pytest.approx([0.27 * c, 0.27 * c, -4.5 * c, -4.5 * c])
    b = W.brunel_scaled(100000)
    assert b["projs"][0]["k"] == 10000 and b["projs"][0]["w_mV"] == pytest.approx(0.1 * 0.2)
    assert b["projs"][1]["w_mV"] == pytest.approx(-5 * 0.1 * 0.2)
    assert b["params"]["w_ext_mV"] == 0.1          # the drive is not scaled


def test_sweep_table_ranges():
    nets = W.sweep()
    assert len(nets) == 512
    n = np.array([s["pops"][0]["size"] + s["pops"][1]["size"] for s in nets])
    p = np.array([s["projs"][0]["p"] for s in nets])
    w = np.array([s["projs"][0]["w_mV"] for s in nets])
    assert n.min() >= 1000 and n.max() <= 20000
    assert 0.01 <= p.min() and p.max() <= 0.05 and 0.1 <= w.min() and w.max() <= 0.4
    # log-uniform sizes: log N roughly uniform over [log 1000, log 20000]
    u = (np.log(n) - math.log(1000)) / math.log(20)
    assert abs(u.mean() - 0.5) < 0.05
    assert len({s["params"]["seed"] for s in nets}) == 512


def test_specs_are_complete():
    for spec in (W.cuba_lif_4k(), W.brunel_fixed_out(n=1000, k=50), W.stdp_er(n=500, p=0.05),
                 W.vogels_scaled(8000), W.brunel_scaled(30000)):
        assert {"params", "pops", "projs", "steps"} <= set(spec)
        for q in spec["projs"]:
            assert 0 <= q["from"] < len(spec["pops"]) and 0 <= q["to"] < len(spec["pops"])
