"""The long-time gradient-formation experiment on the compound-only step:
its machinery (three frozen fields mapped to the four phases of the
paper's valve pattern, the media swap, decay) against the oracle on a
compressed schedule, and one short run of the driver itself."""
import numpy as np
import pytest

from oracle import Oracle
from paper_1307_4703_amd import experiments as E
from paper_1307_4703_amd import workloads as W
from paper_1307_4703_amd.lattice import Lattice
from tests.parity_util import log, seeded_init

pytestmark = pytest.mark.gpu


def _fields(wl, peak=E.GF_U):
    """Stand-ins for the three valve states (left open, right open, closed):
    a Poiseuille profile along the open channel (u_y across its width,
    peaking at the run's U; zero elsewhere, so divergence-free), and rest."""
    out = []
    for (a, b, c, d) in (wl.layout.left_channel, wl.layout.right_channel):
        w = b - a
        s = np.arange(wl.nx) - a + 0.5
        prof = np.where((s > 0) & (s < w), 4.0 * peak * s * (w - s) / w ** 2, 0.0)
        uy = np.zeros(wl.mask.shape)
        uy[c:d, :] = prof[None, :]
        uy[wl.layout.inlet_row, :] = prof
        uy[wl.layout.outlet_row, :] = prof
        out.append((np.zeros(wl.mask.shape), uy))
    z = np.zeros(wl.mask.shape)
    out.append((z, z.copy()))
    return out


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-5)])
def test_valve_pattern_swap_and_decay_against_oracle(storage, tol):
    k = 1e-4
    wl = E.gradient_generator_paper_scale(storage, k_decay=k)
    init = seeded_init(wl, 5)
    init = {"C": np.where(wl.mask == 0, init["C"], 0.0)}
    fields = _fields(wl)
    sched = W.paper_schedule(open_steps=200, closed_steps=1000)
    swapped = W.paper_schedule(open_steps=200, closed_steps=1000, c_source=0.0, c_sink=1.0)
    log(f"gradient formation machinery, {storage}")
    lat = Lattice.from_workload(wl, storage=storage, init=False)
    lat.init(**init)
    lat.set_schedule(sched)
    for slot, f in enumerate(fields):
        lat.set_velocity_field(slot, *f)
    lat.set_phase_fields([0, 2, 1, 2])
    lat.cde_step(2400)
    lat.set_schedule(swapped)
    lat.cde_step(2400)
    C = lat.read()[3]
    d = lat.diagnostics()
    lat.close()
    o = Oracle(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, k_decay=k, segments=wl.segments,
               schedule=sched)
    o.init(**init)
    o.cde_step(2400, fields, phase_field=[0, 2, 1, 2])
    o.schedule = swapped
    o.cde_step(2400, fields, phase_field=[0, 2, 1, 2])
    Co = o.fields()[3]
    fl = wl.mask == 0
    err = float(np.abs(C[fl] - Co[fl]).max() / max(1.0, np.abs(Co[fl]).max()))
    log(f"max |C - oracle| {err:.3e}")
    assert err < tol
    for sid in (2, 3, 4, 5):
        assert d["seg_solute"][sid - 2] == pytest.approx(o.flux_solute[sid], rel=max(tol, 1e-11) * 100,
                                                        abs=1e-9)


def test_driver_short_run():
    """Four minutes of the experiment (two valve periods, the swap after
    the first): finite, bounded, both runs stepped."""
    r = E.gradient_formation(hours=4 / 60, samples_per_hour=30, flow_steps=4000)
    s = E.gradient_formation_summary(r)
    log(f"summary {s}")
    for label in ("decay", "no_decay"):
        assert r[label]["n_nonfinite"] == 0
        assert len(r[label]["t_hours"]) == 2
        for p in r["monitor_points"]:
            assert all(-0.2 < v < 1.2 for v in r[label][p])
    assert r["scale"] * r["u_max_flow"] == pytest.approx(E.GF_U)
