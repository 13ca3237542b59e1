"""Degenerate lattices on the GPU: no fluid at all, a single fluid row, a
single periodic column, the smallest periodic box; each against the oracle
where there is something to compare."""
import numpy as np
import pytest

from paper_1307_4703_amd import workloads as W
from tests.parity_util import field_errors, log, make_lattice, make_oracle, seeded_init

pytestmark = pytest.mark.gpu


def test_no_fluid_nodes():
    mask = np.ones((16, 16), np.uint8)
    wl = W.Workload("walls", mask, tau_f=0.8, D=0.01)
    lat = make_lattice(wl, "f32", {})
    lat.step(10)
    lat.set_velocity_field(0)
    lat.cde_step(4)
    d = lat.diagnostics()
    assert d["n_fluid"] == 0 and d["t"] == 14 and d["mass"] == 0.0
    rho = lat.read()[0]
    assert np.all(np.isnan(rho))


@pytest.mark.parametrize("mask_kind", ["one_row", "one_column", "box_2x2"])
def test_thin_lattices_against_oracle(mask_kind):
    if mask_kind == "one_row":      # walls above and below one row, periodic in x
        mask = np.ones((3, 40), np.uint8)
        mask[1, :] = 0
        periodic = (True, False)
    elif mask_kind == "one_column":  # one column, periodic in x, walls in y
        mask = np.zeros((12, 1), np.uint8)
        mask[0, 0] = mask[-1, 0] = 1
        periodic = (True, False)
    else:                            # 2 x 2, periodic both ways
        mask = np.zeros((2, 2), np.uint8)
        periodic = (True, True)
    wl = W.Workload(mask_kind, mask, tau_f=0.7, D=0.02, periodic=periodic)
    init = seeded_init(wl, 9)
    log(f"degenerate lattice {mask_kind}")
    lat = make_lattice(wl, "f64", init, chunk=8)
    lat.step(37)
    o = make_oracle(wl)
    o.init(**init)
    o.step(37)
    err = field_errors(lat, o, mask == 0)
    log(f"{mask_kind}: {err}")
    for k in ("rho", "C", "f", "g"):
        assert err[k] < 1e-12, (k, err)
