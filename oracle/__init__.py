"""CPU oracle of the MAM hot path (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the HIP library never does.
"""
