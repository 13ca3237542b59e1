"""GPU parity: the HIP coupled step against the FP64 oracle, element by
element, on the same seeded inputs (through the C ABI)."""
import numpy as np
import pytest

from paper_1307_4703_amd import workloads as W
from tests.parity_util import field_errors, log, make_lattice, make_oracle, seeded_init

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
# FP32 / FP16-shifted storage: one storage rounding per population per step
# (unit roundoff 6e-8 for FP32, 4.9e-4 for FP16, relative to the deviations
# from rest that are stored) accumulating over the run, with headroom of
# about ten over what the run shows; u is relative to the run's max |u|.
F32_TOL = {"rho": 1e-6, "u": 2e-5, "C": 2e-5}
F16_TOL = {"rho": 3e-4, "u": 8e-3, "C": 1e-2}


def _run(wl, storage, steps, seed=0, tile=None, chunk=None, form=None):
    init = seeded_init(wl, seed)
    log(f"{wl.name} storage={storage} steps={steps} tile={tile} chunk={chunk} form={form}")
    lat = make_lattice(wl, storage, init, tile=tile, chunk=chunk)
    if form is not None:
        lat.set_two_step(*form)
    lat.step(steps)
    lat.sync()
    o = make_oracle(wl)
    o.init(**init)
    o.step(steps)
    return lat, o


def _ragged_gg(**kw):
    # 300 x 150: neither dimension a multiple of the 64 x 4 tile
    return W.gradient_generator(nx=300, ny=150, **kw)


def test_f64_straight_channel_full_run():
    """Straight channel 128x64, FP64, 1000 steps: GPU == oracle to 1e-12."""
    wl = W.straight_channel()
    lat, o = _run(wl, "f64", 1000)
    err = field_errors(lat, o, wl.mask == 0)
    log(f"errors {err}")
    for k in ("rho", "u", "C", "f", "g"):
        assert err[k] < F64_TOL, (k, err)
    d = lat.diagnostics()
    m, s = o.totals()
    assert d["mass"] == pytest.approx(m, rel=1e-13)
    assert d["solute"] == pytest.approx(s, rel=1e-12)
    assert d["mass_in"] == pytest.approx(o.flux_mass[2], rel=1e-12)
    assert d["mass_out"] == pytest.approx(o.flux_mass[3], rel=1e-12)
    assert d["solute_in"] == pytest.approx(o.flux_solute[2], rel=1e-12)
    assert d["solute_out"] == pytest.approx(o.flux_solute[3], rel=1e-10, abs=1e-12)
    assert d["t"] == 1000 and d["n_fluid"] == 126 * 62


@pytest.mark.parametrize("steps", [1, 2, 3, 301])
def test_f64_gradient_generator_valves(steps):
    """Ragged 300x150 gradient generator with the valves toggling every 7
    steps (phase switches on odd and even steps), FP64."""
    wl = _ragged_gg(half_period=7, storage="f64")
    lat, o = _run(wl, "f64", steps, seed=steps)
    err = field_errors(lat, o, wl.mask == 0)
    log(f"errors {err}")
    for k in ("rho", "u", "C", "f", "g"):
        assert err[k] < F64_TOL, (k, err)
    d = lat.diagnostics()
    for sid in (2, 3, 4, 5):
        assert d["seg_mass"][sid - 2] == pytest.approx(o.flux_mass[sid], rel=1e-11, abs=1e-12)
        assert d["seg_solute"][sid - 2] == pytest.approx(o.flux_solute[sid], rel=1e-11, abs=1e-12)


@pytest.mark.parametrize("periodic", [(True, False), (False, True), (True, True), (False, False)])
def test_f64_random_masks(periodic):
    mask = W.random_mask(133, 71, seed=7, periodic=periodic)
    wl = W.Workload("random", mask, tau_f=0.7, D=0.03, periodic=periodic)
    lat, o = _run(wl, "f64", 40, seed=3)
    err = field_errors(lat, o, mask == 0)
    log(f"errors {err}")
    for k in ("rho", "u", "C", "f", "g"):
        assert err[k] < F64_TOL, (k, err)


def test_f64_paper_d2q4_source_decay():
    """w0 = 0 (the paper's D2Q4 compound lattice), a source patch and decay."""
    wl = _ragged_gg(half_period=11, storage="f64", w0=0.0)
    wl.k_decay = 1e-3
    rng = np.random.default_rng(2)
    R = np.zeros(wl.mask.shape)
    R[60:90, 100:140] = 1e-3 * rng.random((30, 40))
    init = seeded_init(wl, 5)
    log("paper D2Q4 + source + decay")
    lat = make_lattice(wl, "f64", init)
    lat.set_source(R)
    lat.step(60)
    from oracle import Oracle
    o = Oracle(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=0.0, k_decay=1e-3,
               segments=wl.segments, schedule=wl.schedule, R=R)
    o.init(**init)
    o.step(60)
    err = field_errors(lat, o, wl.mask == 0)
    log(f"errors {err}")
    for k in ("rho", "u", "C", "f", "g"):
        assert err[k] < F64_TOL, (k, err)


@pytest.mark.parametrize("tile,chunk", [((64, 4), 0), ((256, 1), 16), ((32, 8), 5),
                                        ((8, 8), 0), ((128, 4), 3), ((16, 32), 7)])
def test_launch_shape_and_graphs_bitwise_identical(tile, chunk):
    """Tile shape, XCD ordering and graph replay change only the order in
    which nodes are processed; AA in-place streaming must give bitwise the
    same state (race check)."""
    wl = _ragged_gg(half_period=5, storage="f32")
    init = seeded_init(wl, 9)
    log(f"reference run, tile {tile} chunk {chunk}")
    ref = make_lattice(wl, "f32", init, tile=(64, 4), chunk=0)
    ref.step(37)
    f0, g0 = ref.populations()
    lat = make_lattice(wl, "f32", init, tile=tile, chunk=chunk)
    lat.step(37)
    f1, g1 = lat.populations()
    assert np.array_equal(f0, f1) and np.array_equal(g0, g1)


@pytest.mark.parametrize("form", [None, (5, 6)])
@pytest.mark.parametrize("storage,tol", [("f32", F32_TOL), ("f16", F16_TOL)])
def test_reduced_precision_against_f64_oracle(storage, tol, form):
    """300 steps across valve switches; form (5, 6): four-step passes in
    graph replays and plain launches, two-step passes for the last four."""
    wl = _ragged_gg(half_period=50, storage=storage)
    lat, o = _run(wl, storage, 300, seed=4, chunk=None if form is None else 64, form=form)
    err = field_errors(lat, o, wl.mask == 0)
    log(f"{storage} errors {err}")
    for k, v in tol.items():
        assert err[k] < v, (k, err)


def test_save_load_resume_bitwise():
    wl = _ragged_gg(half_period=9, storage="f32")
    init = seeded_init(wl, 1)
    log("save/load")
    a = make_lattice(wl, "f32", init)
    a.step(13)
    snap = a.save()
    a.step(20)
    fa, ga = a.populations()
    b = make_lattice(wl, "f32", init)
    b.load(snap)
    assert b.info()["t"] == 13
    b.step(20)
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    assert a.diagnostics()["mass_in"] == b.diagnostics()["mass_in"]


def test_gradient_generator_full_size_f32():
    """The 2048x1024 FP32 gradient generator in the benchmark's launch
    configuration (the two-step form bench.py records for it, 64 x 4
    single-step tiles, graph chunks of 64), 200 steps across a valve
    switch, against the oracle."""
    import bench
    wl = W.gradient_generator(half_period=100)
    lat, o = _run(wl, "f32", 200, seed=0, tile=(64, 4), chunk=64, form=bench.FORMS["gg2048_f32"])
    err = field_errors(lat, o, wl.mask == 0)
    log(f"full-size f32 errors {err}")
    for k, v in F32_TOL.items():
        assert err[k] < v, (k, err)
    d = lat.diagnostics()
    m, s = o.totals()
    # the deviations from rest round without a systematic bias, and the
    # step's weights sum to one exactly in FP32: no mass is created
    assert d["mass"] == pytest.approx(m, rel=1e-7)
    assert d["solute"] == pytest.approx(s, rel=1e-5)
    ro, uxo, uyo, Co = o.fields()
    sel = (wl.region > 0) & (wl.mask == 0)
    umax_chamber = np.sqrt(uxo[sel] ** 2 + uyo[sel] ** 2).max()
    assert d["max_u_region"] == pytest.approx(umax_chamber, rel=1e-3)
    assert d["max_pe_region"] == pytest.approx(umax_chamber / wl.D, rel=1e-3)


def test_f64_full_size_8192_window():
    """The 8192x4096 gradient generator (the lattice of the FP16 precision
    report) in FP64 on the GPU against the oracle over a 200-step window
    from a seeded state, every fluid node: the FP64 GPU run that the
    reduced-precision runs are measured against is the oracle's run."""
    wl = W.gradient_generator(scale=4.0, storage="f64", half_period=60)
    log("full size 8192x4096 FP64, 200 steps against the oracle")
    lat, o = _run(wl, "f64", 200, seed=11)
    err = field_errors(lat, o, wl.mask == 0)
    log(f"errors {err}")
    for k in ("rho", "u", "C"):
        assert err[k] < F64_TOL, (k, err)
