"""MI355X-native coupled lattice Boltzmann step (D2Q9 fluid + D2Q5 compound)
after Tanaka & Iber, arXiv:1307.4703.

The compute path is the HIP library libgg.so (C ABI in include/gg.h); this
package binds it (``Lattice``) and provides the seeded synthetic workloads.
"""
from .lattice import Batch, Lattice, make_phases  # noqa: F401
from . import workloads  # noqa: F401

__all__ = ["Batch", "Lattice", "make_phases", "workloads"]
