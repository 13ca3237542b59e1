"""gg_diagnostics_noalloc (the diagnostics with the reduction in the
library's fixed device array, for callers that cannot allocate) against
gg_diagnostics on the same state: two calls in a row, the second on a
smaller lattice, called through the C ABI."""
import ctypes

import numpy as np
import pytest

from paper_1307_4703_amd import _abi as A
from paper_1307_4703_amd import workloads as W
from tests.parity_util import log, make_lattice, seeded_init

pytestmark = pytest.mark.gpu


def _noalloc(lat):
    d = A.gg_diag()
    A.call("gg_diagnostics_noalloc", lat.handle, ctypes.byref(d))
    return d


def _check(d, ref):
    # FP64 totals in another summation order: the FP64 parity bar
    for k in ("mass", "solute"):
        assert getattr(d, k) == pytest.approx(ref[k], rel=1e-12), k
    # maxima, counts, time and boundary fluxes: the same values
    for k in ("t", "n_fluid", "n_nonfinite", "max_u", "max_u_region", "max_pe_region",
              "mass_in", "mass_out", "solute_in", "solute_out"):
        assert getattr(d, k) == ref[k], k
    assert np.array_equal(np.array(d.seg_mass[:]), ref["seg_mass"])
    assert np.array_equal(np.array(d.seg_solute[:]), ref["seg_solute"])


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_noalloc_diagnostics_equal_allocating_ones(storage):
    # first a lattice with more 64 x 4 tiles than the reduction's 2048
    # work-groups (each folds several tiles), then a smaller one
    big = W.all_fluid_channel(nx=1024, ny=1024, storage=storage)
    small = W.gradient_generator(nx=300, ny=150, half_period=7, storage=storage)
    for wl, steps in ((big, 6), (small, 9)):
        lat = make_lattice(wl, storage, seeded_init(wl, 3))
        lat.step(steps)
        log(f"noalloc diagnostics, {wl.name} {storage}")
        ref = lat.diagnostics()
        d = _noalloc(lat)
        _check(d, ref)
        assert d.n_fluid == wl.n_fluid and d.t == steps
        lat.close()
