"""CPU oracle of the per-step vehicle update -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It wraps the plain C reference in ``moss_oracle.c``
through ctypes and shares nothing with the HIP simulator except the scenario
generator that feeds both.
"""
from .oracle import OracleSim, philox4x32_10, idm, lib, max_threads, mlp_forward, mlp_candidates  # noqa: F401
