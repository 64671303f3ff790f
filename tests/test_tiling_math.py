"""Arithmetic the tiled delivery relies on, restated on the host (binary64 and integer
operations round here as they do on the GPU):

  * a target t of a range [lo, lo + L), L <= 65,536, is recovered from its low 16 bits
    as lo + ((t16 - lo) mod 2^16), so the delivery can read a 16-bit copy of the targets;
  * the schedule's range size m = clamp(floor(x * inv), 1, 8) with inv = (1 + 2^-40) / c
    equals clamp(floor(x / c), 1, 8) for every count c < 2^32, in particular at the
    candidate bounds x = c * m, which must not round down to m - 1;
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


def _m(x, c, M=8):
    inv = (1.0 + 2.0**-40) / c
    return int(min(max(x * inv, 1.0), float(M)))


@pytest.mark.parametrize("seed", range(4))
def test_schedule_quotient_is_exact(seed):
    rng = np.random.default_rng(seed)
    cs = list(rng.integers(1, 2**32, 3000)) + [1, 2, 3, 7, 2**31 - 1, 2**32 - 1, 3720, 5581]
    for c in cs:
        c = int(c)
        for m in range(1, 10):
            for x in (c * m - 1, c * m, c * m + 1):
                if x < 0:
                    continue
                assert _m(x, c) == min(max(x // c, 1), 8), (c, m, x)


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
