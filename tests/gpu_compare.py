"""Helpers shared by the GPU parity tests: build a network through the C ABI and
compare a run with the oracle's run of the same spec element by element."""
import numpy as np

import oracle


def net(spec, **kw):
    from paper_1912_07423_amd import Network
    return Network(spec, **kw)


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def compare_run(spec, steps, **kw):
    g = net(spec, **{"raster_steps": steps, **kw})
    o = oracle.OracleNet(spec, raster_cap=steps)
    g.run(steps)
    o.run(steps)
    return compare_net(g, o, steps)


def compare_net(g, o, steps):
    """A GPU network and the oracle's network of the same spec, both advanced by
    `steps` steps from step 0: raster, state and counters must agree exactly."""
    inf = g.info()
    assert inf["t"] == steps
    rg = g.raster_bits(0, steps)
    ro = o.raster_words()[:steps]
    if not np.array_equal(rg, ro):
        bad = np.nonzero((rg != ro).any(axis=1))[0]
        raise AssertionError(f"raster differs first at step {bad[0]} ({len(bad)} steps differ)")
    s = g.state(weights=bool(inf["plastic"]))
    assert np.array_equal(bits(s["v"]), bits(o.v()))
    assert np.array_equal(s["ref"], o.ref())
    assert np.array_equal(s["input"][steps % inf["input_buffers"]], o.input())
    # events: out-degree sums over the delivered emission steps.  A spike of step e is
    # delivered once the update of step e + d - B has run (B input buffers), so after
    # T steps the GPU has delivered e < T - d + B and the oracle (B = 1) e < T - d + 1.
    outdeg = np.diff(o.row_ptr().astype(np.int64))
    spk = o.raster_bool(0, steps)
    def delivered(upto):
        return int(outdeg[np.nonzero(spk[:max(upto, 0)])[1]].sum())
    assert o.events == delivered(steps - inf["delay"] + 1)
    assert inf["events"] == delivered(steps - inf["delay"] + inf["input_buffers"])
    if inf["plastic"]:
        assert np.array_equal(bits(s["x_pre"]), bits(o.x_pre()))
        assert np.array_equal(bits(s["x_post"]), bits(o.x_post()))
        assert np.array_equal(bits(s["w_f32"]), bits(o.w_f32()))
        assert inf["touches"] == o.touches
    return rg, inf


