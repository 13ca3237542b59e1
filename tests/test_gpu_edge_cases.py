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


def test_three_segments_on_a_vertical_node_pair():
    """A corner where a bottom inlet (4) and two left segments (2, 3) meet:
    each fluid node links to at most two segments, but the nodes (1, 1) and
    (1, 2) link to three between them, which one walking-strip flux record
    cannot hold: fuse 2 is refused, the row-parallel tiles run and match the
    oracle, fluxes per segment included."""
    from paper_1307_4703_amd._abi import GGError, GG_ERR_ARG
    mask = np.ones((12, 16), np.uint8)
    mask[1:-1, 1:-1] = 0
    mask[0, 1:-1] = 4
    mask[1:3, 0] = 2
    mask[3:-1, 0] = 3
    segs = [W.Segment(2, "inlet", (-1, 0), u_max=0.02, c_in=1.0),
            W.Segment(3, "outlet", (-1, 0)),
            W.Segment(4, "inlet", (0, -1), u_max=0.01, c_in=0.5)]
    wl = W.Workload("corner", mask, tau_f=0.8, D=0.02, segments=segs)
    init = seeded_init(wl, 12, amp_u=0.005)
    lat = make_lattice(wl, "f64", init, chunk=8)
    with pytest.raises(GGError) as e:
        lat.set_two_step(2, 8)
    assert e.value.status == GG_ERR_ARG
    lat.set_two_step(3, 6)
    lat.step(40)
    o = make_oracle(wl)
    o.init(**init)
    o.step(40)
    err = field_errors(lat, o, mask == 0)
    log(f"three segments at a corner: {err}")
    for k in ("rho", "u", "C"):
        assert err[k] < 1e-12, (k, err)
    d = lat.diagnostics()
    for s in segs:
        assert d["seg_mass"][s.id - 2] == pytest.approx(o.flux_mass[s.id], rel=1e-10, abs=1e-12)
        assert d["seg_solute"][s.id - 2] == pytest.approx(o.flux_solute[s.id], rel=1e-10, abs=1e-12)
