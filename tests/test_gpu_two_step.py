"""Two-step pass: the state after stepping with passes of two steps (strips
of 62 columns walked row by row, or row-parallel tiles exchanging through
LDS; a one-node halo collided once more) must be bitwise the state the
single-step kernels give, for every storage type, boundary kind,
periodicity, strip height and schedule phase; boundary fluxes agree to
FP64 rounding (their atomics add in another order). The same for the
four-step pass (fuse 5: 58 x 6 tiles with a three-node halo, runs of 8k
steps; other runs in two-step passes), which lattices with pressure
segments decline for the two-step pass."""
import numpy as np
import pytest

from paper_1307_4703_amd import workloads as W
from tests.parity_util import log, make_lattice, seeded_init

pytestmark = pytest.mark.gpu


def _pair(wl, storage, seed, strip_h, chunk=0, R=None, mode=2):
    init = seeded_init(wl, seed)
    one = make_lattice(wl, storage, init, chunk=chunk)
    one.set_two_step(1)
    two = make_lattice(wl, storage, init, chunk=chunk)
    two.set_two_step(mode, strip_h)
    if R is not None:
        one.set_source(R)
        two.set_source(R)
    return one, two


def _same_state(one, two, steps):
    fa, ga = one.populations()
    fb, gb = two.populations()
    assert one.info()["t"] == two.info()["t"] == steps
    if not (np.array_equal(fa, fb) and np.array_equal(ga, gb)):
        bad = np.argwhere(np.any(fa != fb, axis=0) | np.any(ga != gb, axis=0))
        raise AssertionError(f"{len(bad)} nodes differ, first {bad[:5].tolist()}")
    da, db = one.diagnostics(), two.diagnostics()
    for k in ("mass_in", "mass_out", "solute_in", "solute_out"):
        assert db[k] == pytest.approx(da[k], rel=1e-12, abs=1e-12), k


MODES = [(2, 1), (2, 5), (2, 16), (3, 6), (3, 14), (4, 6), (4, 14), (5, 6), (5, 14)]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("mode,strip_h", MODES)
def test_gradient_generator_valves(storage, mode, strip_h):
    """Ragged 300x150 gradient generator, valves switching every 7 steps
    (on odd and even steps, so inside and between the two steps of a pass)."""
    wl = W.gradient_generator(nx=300, ny=150, half_period=7, storage=storage)
    log(f"two-step vs single, {storage}, mode {mode}, rows {strip_h}")
    one, two = _pair(wl, storage, 11, strip_h, mode=mode)
    for n in (8, 3, 29):  # 40 steps: passes, an odd leftover, odd starts
        one.step(n)
        two.step(n)
    _same_state(one, two, 40)


@pytest.mark.parametrize("mode,strip_h", [(2, 7), (3, 6), (4, 14), (5, 6)])
@pytest.mark.parametrize("periodic", [(True, False), (False, True), (True, True), (False, False)])
def test_random_masks_periodic(periodic, mode, strip_h):
    """Obstacles everywhere, 133x71 (not a multiple of the 62- or 58-column
    tile), every combination of periodic axes (FP32 for the four-step
    pass)."""
    mask = W.random_mask(133, 71, seed=7, periodic=periodic)
    wl = W.Workload("random", mask, tau_f=0.7, D=0.03, periodic=periodic)
    log(f"two-step vs single, random mask, periodic {periodic}, mode {mode}")
    one, two = _pair(wl, "f32" if mode == 5 else "f64", 3, strip_h, mode=mode)
    one.step(40)
    two.step(40)
    _same_state(one, two, 40)


@pytest.mark.parametrize("mode,strip_h", [(2, 4), (3, 14), (5, 6)])
@pytest.mark.parametrize("ny", [24, 5])
def test_narrow_periodic_lattice(mode, strip_h, ny):
    """A periodic lattice narrower than one strip: the halo lanes wrap onto
    the strip's own columns (and, periodic in y with 5 rows, the four-step
    tile's halo rows onto its own rows)."""
    mask = np.zeros((ny, 20), np.uint8)
    if ny > 5:
        mask[0, :] = 1
        mask[-1, :] = 1
    else:
        mask[2, 5:9] = 1
    wl = W.Workload("narrow", mask, tau_f=0.9, D=0.02, periodic=(True, ny <= 5))
    one, two = _pair(wl, "f32", 4, strip_h, mode=mode)
    one.step(24)
    two.step(24)
    _same_state(one, two, 24)


@pytest.mark.parametrize("mode,strip_h", [(2, 16), (3, 6), (4, 6), (5, 6)])
def test_source_decay_d2q4_and_graphs(mode, strip_h):
    """w0 = 0 (D2Q4), decay, a source patch, graph-replayed passes."""
    wl = W.gradient_generator(nx=300, ny=150, half_period=11, storage="f32", w0=0.0)
    wl.k_decay = 1e-3
    rng = np.random.default_rng(2)
    R = np.zeros(wl.mask.shape)
    R[60:90, 100:140] = 1e-3 * rng.random((30, 40))
    one, two = _pair(wl, "f32", 5, strip_h, chunk=8, R=R, mode=mode)
    one.step(50)
    two.step(50)
    _same_state(one, two, 50)


@pytest.mark.parametrize("mode,strip_h,storage", [(2, 16, "f64"), (3, 14, "f64"), (4, 6, "f64"),
                                                   (5, 6, "f32"), (5, 6, "f16")])
def test_straight_channel_inlet_outlet(mode, strip_h, storage):
    """Velocity inlet and pressure outlet on vertical segments (the strip's
    halo lanes sit on the ghost columns)."""
    wl = W.straight_channel(storage=storage)
    one, two = _pair(wl, storage, 0, strip_h, mode=mode)
    one.step(120)
    two.step(120)
    _same_state(one, two, 120)


@pytest.mark.parametrize("storage,steps_per_pass", [("f32", 4), ("f16", 4), ("f64", 4)])
def test_four_step_pass_runs_where_it_applies(storage, steps_per_pass):
    """fuse 5 runs four-step passes (the profile times their interior
    kernel) in every storage type; a
    2048x1024 gradient generator over graph replays of 64 steps and a run
    of 8k + 4 plain-launched steps is still bitwise the single steps'."""
    wl = W.gradient_generator(nx=2048, ny=1024, half_period=50, storage=storage)
    one, two = _pair(wl, storage, 5, 6, chunk=64, mode=5)
    p = two.step_profile(64)
    assert p["steps_per_pass"] == steps_per_pass and p["fuse"] == 5
    assert p["graph_passes"] == 64 // steps_per_pass and p["n_graph"] == 1
    two.step(140)  # two replays, then 8 + 4 steps: two four-step and two two-step passes
    one.step(204)
    _same_state(one, two, 204)


@pytest.mark.parametrize("mode,strip_h", [(2, 16), (3, 6)])
def test_timed_passes_keep_the_state(mode, strip_h):
    """gg_step2_timed advances like gg_step."""
    wl = W.gradient_generator(nx=300, ny=150, half_period=9, storage="f32")
    one, two = _pair(wl, "f32", 8, strip_h, mode=mode)
    one.step(12)
    ms = two.step2_timed(3)
    assert ms > 0.0
    _same_state(one, two, 12)


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_four_step_forms_fall_back_with_pressure_segments(storage):
    """Pressure segments (rescaling between steps) and the paper's walls
    keep the four-step forms out: fuse 5 then steps as fuse 3 (two-step
    passes) or in single steps, and the compound-only rows -6 in two-step
    passes, each bitwise the single steps'."""
    nx, ny = 130, 34
    mask = np.zeros((ny, nx), np.uint8)
    mask[0, :] = 1
    mask[-1, :] = 1
    mask[1:-1, 0] = 2
    mask[1:-1, -1] = 3
    segs = [W.Segment(2, "pressure", (-1, 0), rho=1.003, c_in=1.0, fix_c=True),
            W.Segment(3, "pressure", (1, 0), rho=0.997)]
    wl = W.Workload("pressure_channel", mask, tau_f=0.8, D=0.02, segments=segs, storage=storage)
    for walls in (False, True):
        one, two = _pair(wl, storage, 5, 6, mode=5)
        if walls:
            for lat in (one, two):
                lat.set_wall_scheme("equilibrium")
        log(f"four-step forms with pressure segments, {storage}, paper walls {walls}")
        p = two.step_profile(16)
        assert p["steps_per_pass"] == 2 and p["fuse"] == (1 if walls else 5)
        one.step(16)
        one.step(24)
        two.step(24)
        _same_state(one, two, 40)
        for lat in (one, two):
            lat.set_velocity_field(0)
        one.set_cde_launch(0)
        two.set_cde_launch(-6)
        one.cde_step(24)
        two.cde_step(24)
        fa, ga = one.populations()
        fb, gb = two.populations()
        assert np.array_equal(ga, gb) and np.array_equal(fa, fb)
