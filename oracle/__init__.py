"""CPU oracle for the compositing hot path.  TEST INFRASTRUCTURE ONLY.

Importable only by the tests, the smoke check and the benchmark's CPU-baseline
leg.  It shares no code with the HIP library; the product never calls it.
"""

from .composite import (OUTPUTS, Multiset, OracleRangeError, accumulate, batch,
                        narrow, overlap_histogram, replay_session, window)

__all__ = ["OUTPUTS", "Multiset", "OracleRangeError", "accumulate", "batch",
           "narrow", "overlap_histogram", "replay_session", "window"]
