"""Arithmetic the tiled delivery relies on, restated on the host (binary64 and integer
operations round here as they do on the GPU):

  * a target t of a range [lo, lo + L), L <= 65,536, is recovered from its low 16 bits
    as lo + ((t16 - lo) mod 2^16), so the delivery can read a 16-bit copy of the targets;
  * the schedule's range size m = clamp(floor(x * inv), 1, 8) with inv = (1 + 2^-40) / c
    equals clamp(floor(x / c), 1, 8) for every count c < 2^32, in particular at the
    candidate bounds x = c * m, which must not round down to m - 1."""
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
