"""Population layouts (gg_set_layout): the paired layout (f_i and g_i side by
side for i = 0..4) and the plane-major one hold the same state, so every
form of the step must give the same bits in both; switching converts the
stored state exactly, at any step parity, with or without the second plane
set; snapshots of one layout load into a lattice of the other; the
compound-only steps, the adjoint and the batched launch agree across
layouts."""
import numpy as np
import pytest

from paper_1307_4703_amd import Batch, Lattice, workloads as W
from paper_1307_4703_amd._abi import GGError
from tests.parity_util import log, seeded_init

pytestmark = pytest.mark.gpu


def _lattice(wl, storage, init, layout, form=(3, 6), chunk=0):
    lat = Lattice.from_workload(wl, storage=storage, init=False, layout=layout)
    lat.set_launch(64, 4, chunk)
    lat.set_two_step(*form)
    lat.init(**init)
    assert lat.layout == layout
    return lat


def _same(a, b):
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert a.info()["t"] == b.info()["t"]
    if not (np.array_equal(fa, fb) and np.array_equal(ga, gb)):
        bad = np.argwhere(np.any(fa != fb, axis=0) | np.any(ga != gb, axis=0))
        raise AssertionError(f"{len(bad)} nodes differ, first {bad[:5].tolist()}")
    da, db = a.diagnostics(), b.diagnostics()
    for k in ("mass_in", "mass_out", "solute_in", "solute_out"):
        assert db[k] == pytest.approx(da[k], rel=1e-12, abs=1e-12), k


FORMS = [(1, 6), (2, 5), (3, 6), (3, 14), (4, 6), (4, 14), (5, 6)]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("form", FORMS)
def test_both_layouts_give_the_same_steps(storage, form):
    """Ragged 300x150 gradient generator, valves switching every 7 steps,
    stepped in every launch form, graph replays included."""
    wl = W.gradient_generator(nx=300, ny=150, half_period=7, storage=storage)
    init = seeded_init(wl, 11)
    log(f"layouts, gradient generator {storage}, form {form}")
    a = _lattice(wl, storage, init, "planes", form, chunk=8)
    b = _lattice(wl, storage, init, "paired", form, chunk=8)
    for n in (8, 3, 29):
        a.step(n)
        b.step(n)
    _same(a, b)


@pytest.mark.parametrize("form", [(1, 6), (3, 6), (4, 14), (5, 6)])
@pytest.mark.parametrize("periodic", [(True, False), (False, True), (True, True)])
def test_periodic_lattices(periodic, form):
    """Obstacles everywhere, 133x71, periodic axes (the neighbours wrap, so
    the pushes take their addresses from the neighbour table)."""
    mask = W.random_mask(133, 71, seed=7, periodic=periodic)
    wl = W.Workload("random", mask, tau_f=0.7, D=0.03, periodic=periodic, storage="f32")
    init = seeded_init(wl, 3)
    log(f"layouts, random mask periodic {periodic}, form {form}")
    a = _lattice(wl, "f32", init, "planes", form)
    b = _lattice(wl, "f32", init, "paired", form)
    for lat in (a, b):
        lat.step(37)
    _same(a, b)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_pressure_segments_and_paper_walls(storage):
    """Pressure boundaries (rescaling between the pass's steps) and the
    paper's walls (single steps with the wall kernels around them)."""
    nx, ny = 130, 34
    mask = np.zeros((ny, nx), np.uint8)
    mask[0, :] = 1
    mask[-1, :] = 1
    mask[1:-1, 0] = 2
    mask[1:-1, -1] = 3
    segs = [W.Segment(2, "pressure", (-1, 0), rho=1.003, c_in=1.0, fix_c=True),
            W.Segment(3, "pressure", (1, 0), rho=0.997)]
    wl = W.Workload("pressure_channel", mask, tau_f=0.8, D=0.02, segments=segs,
                    storage=storage)
    init = seeded_init(wl, 5)
    for scheme, form in (("bounce_back", (4, 6)), ("equilibrium", (1, 6))):
        log(f"layouts, pressure channel {storage}, walls {scheme}")
        lats = []
        for layout in ("planes", "paired"):
            lat = Lattice.from_workload(wl, storage=storage, init=False, layout=layout)
            lat.set_two_step(*form)
            lat.set_wall_scheme(scheme)
            lat.init(**init)
            lat.step(60)
            lats.append(lat)
        _same(*lats)


@pytest.mark.parametrize("form", [(1, 6), (3, 6)])
@pytest.mark.parametrize("start", [12, 13])
def test_switching_converts_the_state(form, start):
    """Switching at even and odd t, with the second plane set (fuse 3) and
    without it (fuse 1, a buffer of its own), back and forth, equals never
    switching."""
    wl = W.gradient_generator(nx=200, ny=100, half_period=5, storage="f16")
    init = seeded_init(wl, 2)
    ref = _lattice(wl, "f16", init, "paired", form)
    sw = _lattice(wl, "f16", init, "paired", form)
    ref.step(start)
    sw.step(start)
    sw.set_layout("planes")
    assert sw.layout == "planes"
    _same(ref, sw)
    ref.step(9)
    sw.step(9)
    sw.set_layout("paired")
    sw.set_layout("paired")  # (no change)
    ref.step(8)
    sw.step(8)
    _same(ref, sw)


def test_snapshots_load_across_layouts():
    wl = W.gradient_generator(nx=200, ny=100, half_period=5, storage="f32")
    init = seeded_init(wl, 6)
    a = _lattice(wl, "f32", init, "paired")
    a.step(11)
    snap = a.save()
    b = _lattice(wl, "f32", seeded_init(wl, 7), "planes")
    b.load(snap)
    assert b.layout == "planes" and b.info()["t"] == 11
    _same(a, b)
    a.step(10)
    b.step(10)
    _same(a, b)
    c = _lattice(wl, "f32", seeded_init(wl, 8), "paired")
    c.load(b.save())
    assert c.layout == "paired"
    _same(b, c)


def test_compound_only_steps_agree():
    wl = W.gradient_generator(nx=300, ny=150, half_period=9, storage="f32")
    init = seeded_init(wl, 3)
    lats = []
    for layout in ("planes", "paired"):
        lat = _lattice(wl, "f32", init, layout)
        lat.step(40)
        lat.set_velocity_field(0)
        lat.set_cde_launch(14)
        lat.cde_step(30)
        lat.set_cde_launch(0)
        lat.cde_step(8)
        lats.append(lat)
    _same(*lats)


def test_adjoint_agrees():
    wl = W.gradient_generator(nx=160, ny=80, half_period=15, storage="f32")
    init = seeded_init(wl, 3)
    rng = np.random.default_rng(4)
    weight = np.where(wl.mask == 0, rng.random(wl.mask.shape), 0.0)
    target = rng.random(wl.mask.shape)
    res = []
    for layout in ("planes", "paired"):
        lat = _lattice(wl, "f32", init, layout, (4, 6))
        res.append(lat.adjoint(60, weight, target, ckpt_every=7))
    assert res[0]["loss"] == res[1]["loss"]
    assert np.array_equal(res[0]["d_c_in"], res[1]["d_c_in"])
    assert res[0]["d_omega_g"] == res[1]["d_omega_g"]


def test_batch_members_share_the_layout():
    wls = W.batch_instances(4, 4703)
    init = [seeded_init(wl, 10 + k) for k, wl in enumerate(wls)]
    mixed = [_lattice(wl, "f32", i, "paired" if k else "planes") for k, (wl, i) in
             enumerate(zip(wls, init))]
    with pytest.raises(GGError, match="layout"):
        Batch(mixed, tile=(64, 4), graph_chunk=0, fuse=4, rows=6)
    for layout in ("planes", "paired"):
        ref = [_lattice(wl, "f32", i, layout, (4, 6)) for wl, i in zip(wls, init)]
        bat = [_lattice(wl, "f32", i, layout, (4, 6)) for wl, i in zip(wls, init)]
        b = Batch(bat, tile=(64, 4), graph_chunk=0, fuse=4, rows=6)
        b.step(12)
        for lat in ref:
            lat.step(12)
        for x, y in zip(ref, bat):
            _same(x, y)
