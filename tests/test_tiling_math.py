"""Arithmetic the tiled delivery relies on, restated on the host (binary64 and integer
operations round here as they do on the GPU):

  * a target t of a range [lo, lo + L), L <= 65,536, is recovered from its low 16 bits
    as lo + ((t16 - lo) mod 2^16), so the delivery can read a 16-bit copy of the targets;
  * the window schedule (ranges per step from a searched work bound) never needs more
    workgroups than the grid, cuts every step's tiles into ranges of 1 to 32 tiles that
    cover them exactly, and balances a steady window to within 12% of ideal;
  * the tile boundaries of a sorted row, written by one streaming pass from the tile
    changes between consecutive targets, equal their definition (the first target
    >= p * tile_size)."""
import numpy as np
import pytest



def test_low_16_bits_identify_a_target_in_its_range():
    rng = np.random.default_rng(11)
    for L in (1, 2299, 18392, 65535, 65536):
        lo = rng.integers(0, 2**31 - 70000, 2000, dtype=np.int64)
        t = lo + rng.integers(0, L, 2000, dtype=np.int64)
        t16 = t & 0xFFFF
        assert np.array_equal((t16 - lo) & 0xFFFF, t - lo)
    # a range of 65,537 targets would alias its first and last target
    lo, t = 5, 5 + 65536
    assert ((t & 0xFFFF) - lo) & 0xFFFF == 0


M = 32  # base tiles a range may hold (the LDS accumulators)


def _schedule(c, P, G):
    """The window schedule's arithmetic in binary32, as the delivery's wave 0 computes
    it: ranges per step r_w = clamp(ceil(c_w P / X), r_min, P) for a bound X found by
    two 64-way rounds (X_lb 2^(j/4), then 64 even steps below the first feasible one)."""
    f = np.float32
    steps = len(c)
    r_min = -(-P // M)
    p_f = f(P)

    def ranges_at(work, inv):
        q = np.ceil(f(work) * f(inv), dtype=np.float32)
        return int(min(max(q, f(r_min)), f(P)))

    def need(inv):
        return sum(ranges_at(f(cw) * p_f, inv) for cw in c)

    total = int(sum(c))
    inv_best = f(0)
    if total > 0 and G > steps * r_min:
        x_lb = f(f(total) * p_f) / f(G)
        x1 = [f(x_lb * np.exp2(f(0.25) * f(j), dtype=np.float32)) for j in range(64)]
        ok1 = [need(f(1) / x) <= G for x in x1]
        if any(ok1):
            j = ok1.index(True)
            hi = x1[j]
            lo = x1[j - 1] if j else f(0)
            x2 = [hi if k == 63 else f(lo + f(f(hi - lo) * f(f(k + 1) * f(1 / 64)))) for k in range(64)]
            inv2 = [f(1) / x for x in x2]
            ok2 = [need(v) <= G for v in inv2]
            inv_best = inv2[ok2.index(True) if any(ok2) else 63]
    return [ranges_at(f(cw) * p_f, inv_best) for cw in c]


@pytest.mark.parametrize("seed", range(4))
def test_schedule_fits_the_grid_and_covers_every_tile(seed):
    rng = np.random.default_rng(seed)
    cases = [([373] * 15, 348, 256), ([0] * 15, 348, 256), ([5000] + [0] * 14, 348, 256),
             ([1] * 64, 5, 320), ([7, 0, 3], 1, 3), ([200000] * 15, 348, 256)]
    for _ in range(60):
        steps = int(rng.integers(1, 65))
        P = int(rng.integers(1, 2000))
        G = steps * -(-P // M) + int(rng.integers(0, 600))
        c = list(rng.integers(0, 3000, steps) * (rng.random(steps) < 0.9))
        cases.append((c, P, G))
    for c, P, G in cases:
        r = _schedule(c, P, G)
        assert sum(r) <= G
        for w, rw in enumerate(r):
            assert -(-P // M) <= rw <= P
            edges = [j * P // rw for j in range(rw + 1)]
            assert edges[0] == 0 and edges[-1] == P
            sizes = np.diff(edges)
            assert sizes.min() >= 1 and sizes.max() <= M


def test_schedule_balances_a_steady_window():
    # step counts of a steady-state window of the 1e9-synapse network (about 373 spikes
    # per step, the busiest near 1.5x the mean), 348 base tiles, 256 workgroups
    rng = np.random.default_rng(5)
    for _ in range(20):
        c = [int(x) for x in rng.integers(250, 560, 15)]
        r = _schedule(c, 348, 256)
        work = max(cw * -(-348 // rw) for cw, rw in zip(c, r))  # largest range of any step
        ideal = sum(c) * 348 / 256
        assert work / ideal < 1.12, (c, r)


def _boundaries_by_definition(row, tiles, ts):
    return [int(np.searchsorted(row, p * ts, side="left")) for p in range(tiles)] + [len(row)]


def _boundaries_by_tile_changes(row, tiles, ts):
    """The index pass's formulation: element e is the boundary of every tile p in
    (tile(e - 1), tile(e)] (tile(-1) = -1); the entries past the last element's tile get
    the row length."""
    out = [None] * (tiles + 1)
    prev = -1
    for e, t in enumerate(row):
        tl = int(t) // ts
        for p in range(prev + 1, tl + 1):
            out[p] = e
        prev = tl
    for p in range(prev + 1, tiles + 1):
        out[p] = len(row)
    return out


@pytest.mark.parametrize("seed", range(3))
def test_tile_boundaries_from_tile_changes(seed):
    rng = np.random.default_rng(100 + seed)
    for n, k, tiles in [(2500, 250, 3), (2500, 250, 120), (70000, 70, 40), (200000, 5000, 87), (1000, 0, 7),
                        (1000, 5, 300), (64, 63, 64)]:
        ts = -(-n // tiles)
        tiles = -(-n // ts)
        for _ in range(5):
            row = np.sort(rng.choice(n, size=k, replace=False)) if k else np.zeros(0, dtype=np.int64)
            assert _boundaries_by_tile_changes(row, tiles, ts) == _boundaries_by_definition(row, tiles, ts)
    # every target in one tile, and targets only in the last tile
    row = np.arange(10, 20)
    assert _boundaries_by_tile_changes(row, 4, 25) == _boundaries_by_definition(row, 4, 25)
    row = np.arange(80, 100)
    assert _boundaries_by_tile_changes(row, 4, 25) == _boundaries_by_definition(row, 4, 25)
