"""CPU oracle (plain FP64 numpy) for the NOLSM hot path.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
