"""GPU parity of lazy plasticity (Sec. III-A.1: potentiation kept pending per row and
replayed in registers when the row transmits or its oldest pending step would leave
the 64-step spike history) against the oracle, which applies every STDP event eagerly.
Spike raster, V, traces, every plastic weight and the touch count must be identical:
for delays 1 to 64, ragged sizes, neurons that spike on consecutive steps (no
refractory period), runs interrupted by state reads (which bring every row current)
and by state writes of weights and traces; and the lazy and eager forms on the GPU
against each other."""
import numpy as np
import pytest

import oracle
from paper_1912_07423_amd import workloads as W
from gpu_compare import bits, compare_net, compare_run, net as _net

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    return gpu_available


def _specs():
    fast = W.stdp_er(n=600, p=0.1, delay_steps=3, rate_hz=400.0, n_ext=200, seed=21, steps=300)
    fast["params"]["t_ref_ms"] = 0.0   # spikes on consecutive steps
    strong = W.stdp_er(n=1500, p=0.05, delay_steps=10, rate_hz=80.0, seed=22, steps=500)
    strong["params"].update(a_plus=0.05, a_minus=0.01)  # many clipped potentiations
    return {
        "d10": W.stdp_er(n=2000, p=0.05, delay_steps=10, steps=400),
        "d1_ragged": W.stdp_er(n=777, p=0.08, delay_steps=1, rate_hz=40.0, seed=23, steps=350),
        "d64": W.stdp_er(n=1000, p=0.05, delay_steps=64, rate_hz=40.0, seed=24, steps=400),
        "no_refractory": fast,
        "strong_ltp": strong,
    }


@pytest.mark.parametrize("name", list(_specs()))
def test_lazy_matches_oracle(name):
    spec = _specs()[name]
    print(f"[lazy] {name}: {spec['steps']} steps", flush=True)
    rg, inf = compare_run(spec, spec["steps"], plasticity="lazy")
    assert inf["plasticity"] == 1 and inf["touches"] > 0
    assert int(np.unpackbits(rg.view(np.uint8)).sum()) > 0


def test_lazy_state_reads_and_writes_mid_run():
    """State reads bring every row current (a flush); a state write of weights and
    presynaptic traces rebuilds the rows' traces at age.  Both mid-run, on both sides."""
    spec = _specs()["d10"]
    g = _net(spec, raster_steps=400, plasticity="lazy")
    o = oracle.OracleNet(spec, raster_cap=400)
    g.run(97)
    o.run(97)
    s = g.state(weights=True)
    assert np.array_equal(bits(s["w_f32"]), bits(o.w_f32()))
    assert g.info()["touches"] == o.touches
    g.run(60)
    o.run(60)
    # set some weights and presynaptic traces on both sides
    rng = np.random.default_rng(5)
    w = g.state(weights=True)["w_f32"]
    xp = g.state()["x_pre"]
    idx = rng.choice(len(w), 500, replace=False)
    w[idx] = np.float32(0.25)
    neu = rng.choice(len(xp), 50, replace=False)
    xp[neu] = xp[neu] + np.float32(0.75)
    g.set_state(w_f32=w, x_pre=xp)
    o.w_f32()[idx] = np.float32(0.25)
    o.x_pre()[neu] = o.x_pre()[neu] + np.float32(0.75)
    g.run(243)
    o.run(243)
    compare_net(g, o, 400)


def test_lazy_equals_eager_on_the_gpu():
    spec = W.stdp_er(n=20_000, p=0.02, delay_steps=10, rate_hz=20.0, seed=25, steps=600)
    print("[lazy] 20,000 neurons, 600 steps: lazy against eager", flush=True)
    runs = {}
    for mode in ("eager", "lazy"):
        g = _net(spec, raster_steps=600, plasticity=mode)
        g.run(600)
        runs[mode] = (g.raster_bits(0, 600), g.state(weights=True), g.info())
        g.close()
    (re, se, ie), (rl, sl, il) = runs["eager"], runs["lazy"]
    assert np.array_equal(re, rl)
    for k in ("v", "x_pre", "x_post", "w_f32"):
        assert np.array_equal(bits(se[k]), bits(sl[k])), k
    assert ie["touches"] == il["touches"] and ie["events"] == il["events"]


def test_lazy_refuses_delivery_changes_and_long_delays():
    from paper_1912_07423_amd import SnnError
    spec = W.stdp_er(n=500, p=0.05, delay_steps=10, steps=20)
    g = _net(spec, plasticity="lazy")
    with pytest.raises(SnnError):
        g.set_delivery("atomic")
    with pytest.raises(SnnError):
        g.set_delivery("tiled")
    with pytest.raises(SnnError, match="lazy"):
        _net(spec, plasticity="lazy", delivery="tiled")
    spec = W.stdp_er(n=500, p=0.05, delay_steps=65, steps=20)
    with pytest.raises(SnnError, match="delay"):
        _net(spec, plasticity="lazy")
