"""GPU parity of the pressure boundary (the paper's do-nothing plus
rescaling, Eq. 10) against the oracle, through the C ABI: a pressure-driven
channel and a gradient generator whose channels are driven by pressure,
with valves switching, graphs, odd leftovers, the compound-only step, and
the calls that refuse such lattices."""
import numpy as np
import pytest

from oracle import Oracle
from paper_1307_4703_amd import Batch, Lattice
from paper_1307_4703_amd import workloads as W
from paper_1307_4703_amd._abi import GGError, GG_ERR_STATE
from tests.parity_util import field_errors, log, seeded_init

pytestmark = pytest.mark.gpu

TOL = {"f64": {"rho": 1e-12, "u": 1e-12, "C": 1e-12},
       "f32": {"rho": 1e-6, "u": 2e-5, "C": 2e-5},
       "f16": {"rho": 3e-4, "u": 8e-3, "C": 1e-2}}


def _channel(storage, schedule=None):
    nx, ny = 130, 34
    mask = np.zeros((ny, nx), np.uint8)
    mask[0, :] = 1
    mask[-1, :] = 1
    mask[1:-1, 0] = 2
    mask[1:-1, -1] = 3
    segs = [W.Segment(2, "pressure", (-1, 0), rho=1.003, c_in=1.0, fix_c=True),
            W.Segment(3, "pressure", (1, 0), rho=0.997)]
    return W.Workload("pressure_channel", mask, tau_f=0.8, D=0.02, segments=segs,
                      schedule=schedule, storage=storage)


def _pressure_gg(storage, half_period=7):
    wl = W.gradient_generator(nx=300, ny=150, half_period=half_period, storage=storage)
    wl.segments = [W.Segment(2, "pressure", (0, -1), rho=1.002, c_in=1.0, fix_c=True),
                   W.Segment(3, "pressure", (0, 1), rho=0.998),
                   W.Segment(4, "pressure", (0, -1), rho=1.002, c_in=0.0, fix_c=True),
                   W.Segment(5, "pressure", (0, 1), rho=0.998)]
    return wl


def _oracle(wl):
    return Oracle(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, k_decay=wl.k_decay,
                  segments=wl.segments, schedule=wl.schedule, t_origin=wl.t_origin)


def _run_pair(wl, storage, steps, seed, chunk=8, two_step=None):
    init = seeded_init(wl, seed)
    lat = Lattice.from_workload(wl, storage=storage, init=False)
    lat.set_launch(64, 4, chunk)
    if two_step is not None:
        lat.set_two_step(*two_step)
    lat.init(**init)
    o = _oracle(wl)
    o.init(**init)
    for n in steps:
        lat.step(n)
        o.step(n)
    return lat, o


def _check(lat, o, wl, storage, label):
    err = field_errors(lat, o, wl.mask == 0)
    log(f"{label}: {err}")
    for k, tol in TOL[storage].items():
        assert err[k] < tol, (k, err)
    d = lat.diagnostics()
    ftol = 1e-10 if storage == "f64" else 1e-3
    for s in wl.segments:
        assert d["seg_mass"][s.id - 2] == pytest.approx(o.flux_mass[s.id], rel=ftol, abs=1e-9)
        assert d["seg_solute"][s.id - 2] == pytest.approx(o.flux_solute[s.id], rel=ftol, abs=1e-9)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_pressure_channel(storage):
    wl = _channel(storage)
    log(f"pressure channel {storage}")
    lat, o = _run_pair(wl, storage, (37, 200, 63), seed=1)
    _check(lat, o, wl, storage, f"pressure channel {storage}")
    rho = lat.read()[0]
    tol = {"f64": 1e-14, "f32": 1e-6, "f16": 1e-3}[storage]
    assert np.abs(rho[1:-1, 1] - 1.003).max() < tol


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_pressure_gradient_generator_valves(storage):
    """Channels driven by pressure, valves switching every 7 steps, with the
    row-parallel two-step pass (the first rescaling of each pass in
    registers, the second as the rescaling kernel)."""
    wl = _pressure_gg(storage)
    log(f"pressure gradient generator {storage}")
    lat, o = _run_pair(wl, storage, (8, 3, 29, 60), seed=4, two_step=(3, 6))
    _check(lat, o, wl, storage, f"pressure gg {storage}")


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_pressure_passes_equal_single_steps(storage):
    """Every two-step form that covers pressure segments (row-parallel
    tiles with the boundary kernel apart or in one kernel, 6 or 14 rows)
    leaves the state single steps leave, bit for bit, and the same fluxes;
    the walking strips fall back to single steps."""
    wl = _pressure_gg(storage, half_period=5)
    init = seeded_init(wl, 11)
    lats = []
    for form in ((1, 6), (3, 6), (3, 14), (4, 6), (4, 14), (2, 8)):
        lat = Lattice.from_workload(wl, storage=storage, init=False)
        lat.set_launch(64, 4, 8)
        lat.set_two_step(*form)
        lat.init(**init)
        for n in (8, 3, 29, 60):
            lat.step(n)
        lats.append((form, lat))
    f0, g0 = lats[0][1].populations()
    d0 = lats[0][1].diagnostics()
    for form, lat in lats[1:]:
        f, g = lat.populations()
        log(f"pressure pass {form} {storage}: max |df| {np.nanmax(np.abs(f - f0)):.3e}")
        assert np.array_equal(f, f0, equal_nan=True) and np.array_equal(g, g0, equal_nan=True), form
        d = lat.diagnostics()
        for k in ("seg_mass", "seg_solute"):
            np.testing.assert_allclose(d[k], d0[k], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_pressure_compound_only_passes_equal_single_steps(storage):
    """The compound-only step with pressure segments (inlets holding C_in):
    single steps and the two-step passes of 6 and 14 rows leave the same
    compound bit for bit, from an even and from an odd step, valves
    switching."""
    wl = _pressure_gg(storage, half_period=5)
    init = seeded_init(wl, 13)
    out = []
    for rows in (0, 6, 14):
        lat = Lattice.from_workload(wl, storage=storage, init=False)
        lat.set_launch(64, 4, 8)
        lat.init(**init)
        lat.step(9)
        lat.set_velocity_field(0)
        lat.set_cde_launch(rows)
        for n in (2, 8, 30, 64):
            lat.cde_step(n)
        out.append((rows, lat.populations()[1], lat.diagnostics()["seg_solute"]))
    for rows, g, sol in out[1:]:
        log(f"pressure compound-only pass {rows} rows {storage}: max |dg| "
            f"{np.nanmax(np.abs(g - out[0][1])):.3e}")
        assert np.array_equal(g, out[0][1], equal_nan=True), rows
        np.testing.assert_allclose(sol, out[0][2], rtol=1e-12, atol=1e-12)


def test_pressure_closed_valves_conserve():
    wl = _channel("f64", schedule=[W.Phase(100, frozenset())])
    lat, o = _run_pair(wl, "f64", (51,), seed=3)
    _check(lat, o, wl, "f64", "closed pressure valves")
    d = lat.diagnostics()
    assert not np.any(d["seg_mass"]) and not np.any(d["seg_solute"])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_pressure_compound_only(storage):
    wl = _pressure_gg(storage, half_period=9)
    init = seeded_init(wl, 6)
    lat = Lattice.from_workload(wl, storage=storage, init=False)
    lat.set_launch(64, 4, 8)
    lat.init(**init)
    o = _oracle(wl)
    o.init(**init)
    lat.step(11)
    o.step(11)
    lat.set_velocity_field(0)
    _, ux, uy, _ = o.fields()
    lat.cde_step(40)
    o.cde_step(40, [(np.nan_to_num(ux), np.nan_to_num(uy))])
    fl = wl.mask == 0
    C = lat.read()[3]
    Co = o.fields()[3]
    err = float(np.abs(C[fl] - Co[fl]).max() / max(1.0, np.abs(Co[fl]).max()))
    log(f"compound only with pressure boundaries {storage}: {err:.3e}")
    assert err < TOL[storage]["C"]


def test_calls_that_refuse_pressure_boundaries():
    wl = _channel("f32")
    lat = Lattice.from_workload(wl)
    w = np.ones((wl.ny, wl.nx))
    for call in (lambda: lat.adjoint(4, w, w), lambda: lat.step_timed(2),
                 lambda: lat.step2_timed(1), lambda: Batch([lat])):
        with pytest.raises(GGError) as e:
            call()
        assert e.value.status == GG_ERR_STATE
    lat.step(4)
    assert lat.info()["t"] == 4


def test_boundary_comparison_runs():
    from paper_1307_4703_amd import experiments as E
    r = E.boundary_comparison(steps=4000, rate_steps=64)
    log(f"boundary comparison (short) {r}")
    for label in ("velocity_inlet", "pressure", "pressure_paper_walls"):
        assert np.isfinite(r[label]["profile_error_vs_local_gradient"])
        assert r[label]["gg2048_f32_mlups"] > 0
        assert 0 < r[label]["no_slip_points"][0] < 1.5
    g = r["gradient_generator_2048"]
    for label in ("velocity_inlet", "pressure", "pressure_paper_walls"):
        assert np.isfinite(g[label]["max_u_chamber"]) and g[label]["u_centre_source_channel"] > 0
