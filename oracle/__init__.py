"""CPU oracle of the clock-driven work-queue SNN simulation (test infrastructure only).

Plain, slow, single-threaded reference: only tests, the smoke check and the
benchmark's CPU-baseline leg may use it.  It shares no code with the GPU library.
"""
from .oracle import (OracleNet, binom_table, deliver_generated, gen_row, neg_log,  # noqa: F401
                     philox4x32_10, spacing_core)
