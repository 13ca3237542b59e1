"""The monitor (FP64 diagnostics reduced every K steps inside gg_step,
without waiting) and the profiled step (plain launches with events around
the dominant kernel): the monitor record equals gg_diagnostics taken at the
same step, and neither changes the state, which stays bitwise that of plain
gg_step calls."""
import numpy as np
import pytest

from paper_1307_4703_amd import workloads as W
from paper_1307_4703_amd._abi import GGError, GG_ERR_STATE
from tests.parity_util import log, make_lattice, seeded_init

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage,fuse", [("f64", 3), ("f32", 4), ("f16", 3), ("f32", 1)])
def test_monitor_matches_diagnostics(storage, fuse):
    wl = W.gradient_generator(nx=300, ny=150, half_period=9, storage=storage)
    init = seeded_init(wl, 5)
    a = make_lattice(wl, storage, init, chunk=8)
    b = make_lattice(wl, storage, init, chunk=8)
    for lat in (a, b):
        lat.set_two_step(fuse, 6)
    a.step(3)
    b.step(3)
    with pytest.raises(GGError) as e:
        a.monitor()
    assert e.value.status == GG_ERR_STATE
    a.set_monitor(10)
    log(f"monitor every 10, {storage} fuse {fuse}")
    a.step(17)                 # one reduction, after the 10th step
    a.step(23)                 # three more (20th, 30th, 40th)
    b.step(40)
    m = a.monitor()
    d = b.diagnostics()
    assert m["count"] == 4 and m["t"] == d["t"] == 43
    # the reduction is deterministic (no atomics); the boundary fluxes are
    # FP64 atomic sums whose order varies from run to run
    for k in ("mass", "solute", "max_u", "max_u_region"):
        assert m[k] == d[k], k
    for k in ("mass_in", "mass_out", "solute_in", "solute_out"):
        assert m[k] == pytest.approx(d[k], rel=1e-12, abs=1e-13), k
    assert np.allclose(m["seg_mass"], d["seg_mass"], rtol=1e-12, atol=1e-13)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


@pytest.mark.parametrize("fuse", [1, 3, 4])
def test_profiled_steps_equal_plain_steps(fuse):
    wl = W.gradient_generator(nx=300, ny=150, half_period=7, storage="f32")
    init = seeded_init(wl, 8)
    a = make_lattice(wl, "f32", init, chunk=8)
    b = make_lattice(wl, "f32", init, chunk=8)
    for lat in (a, b):
        lat.set_two_step(fuse, 6)
    a.step(1)
    b.step(1)
    log(f"profiled steps, fuse {fuse}")
    p = a.step_profile(22)     # odd start: 1 single, 5 quads (10 passes), 1 single
    b.step(22)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    # graph chunk 8: one odd step, two replays of 8 steps, the rest plain
    assert p["n_graph"] == 2
    if fuse == 1:
        assert p["n_pass"] == 0 and p["graph_passes"] == 0 and p["graph_singles"] == 16
        assert sum(p["n_single"]) == 6 and p["n_single"] == [3, 3]
    else:
        assert p["graph_passes"] == 8 and p["n_pass"] == 2 and sum(p["n_single"]) == 2
        assert p["pass_fluid"] + p["pass_side_fluid"] == a.info()["n_fluid"]
    assert p["ms_total"] > 0 and p["ms_pass"] >= 0 and p["ms_graph"] > 0
    assert p["ms_pass"] + p["ms_graph"] + sum(p["ms_single"]) <= p["ms_total"] * 1.01
