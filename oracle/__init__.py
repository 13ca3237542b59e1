"""FP64 CPU oracle of the coupled lattice Boltzmann step (test infrastructure).

Importable only from the test-suite, the smoke entry point and the CPU-baseline
leg of the benchmark. The HIP library never imports it.
"""
from .oracle import (Oracle, feq, geq, lib, segment_extent, set_threads, tau_g_from_D,  # noqa: F401
                     threads)
