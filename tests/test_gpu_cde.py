"""GPU parity of the compound-only step on frozen velocity fields (the
paper's decoupled production path, Results section) against the FP64
oracle's compound-only step, through the C ABI: given fields per schedule
phase, fields captured from the fluid state, odd start times, graph replays
and the full-size gradient generator."""
import numpy as np
import pytest

from oracle import Oracle
from paper_1307_4703_amd import Lattice
from paper_1307_4703_amd import workloads as W
from paper_1307_4703_amd._abi import GGError, GG_ERR_ARG, GG_ERR_STATE
from tests.parity_util import log, make_lattice, make_oracle, seeded_init

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
# C relative to max(1, max C): FP32 / FP16 storage rounding per step (see
# the coupled-step parity tests), the field rounded once to FP32
C_TOL = {"f64": F64_TOL, "f32": 2e-5, "f16": 1e-2}


def _fields(shape, seed, amp=0.04):
    """Two smooth synthetic velocity fields (sums of a few sine modes)."""
    rng = np.random.default_rng(seed)
    ny, nx = shape
    yy, xx = np.mgrid[0:ny, 0:nx]
    out = []
    for _ in range(2):
        comp = []
        for _c in range(2):
            v = np.zeros(shape)
            for _m in range(3):
                kx, ky = rng.integers(1, 5, 2)
                ph = rng.random(2) * 2 * np.pi
                v += np.sin(2 * np.pi * kx * xx / nx + ph[0]) * np.cos(2 * np.pi * ky * yy / ny + ph[1])
            comp.append(amp / 3 * v)
        out.append(tuple(comp))
    return out


def _compare(lat, o, fluid, storage, label):
    _, _, _, C = lat.read()
    _, _, _, Co = o.fields()
    f, g = lat.populations()
    go = np.moveaxis(o.g, 2, 0)
    errC = float(np.abs(C[fluid] - Co[fluid]).max() / max(1.0, np.abs(Co[fluid]).max()))
    errg = float(np.abs(g[:, fluid] - go[:, fluid]).max() / max(1e-300, np.abs(go[:, fluid]).max()))
    log(f"{label}: C err {errC:.3e}, g err {errg:.3e}")
    assert errC < C_TOL[storage], (label, errC)
    if storage == "f64":
        assert errg < F64_TOL, (label, errg)
    return f


@pytest.mark.parametrize("rows", [14, -6])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_given_fields_per_phase(storage, rows):
    """Ragged 300x150 gradient generator, valves switching every 7 steps,
    one field per valve phase, source and decay; 40 steps in graph replays
    of 8 plus plain launches (two- or four-step passes); the fluid
    populations stay as they were."""
    wl = W.gradient_generator(nx=300, ny=150, half_period=7, storage=storage)
    wl.k_decay = 1e-3
    rng = np.random.default_rng(9)
    R = np.zeros(wl.mask.shape)
    R[50:70, 90:130] = 1e-3 * rng.random((20, 40))
    init = seeded_init(wl, 21)
    lat = make_lattice(wl, storage, init, chunk=8)
    lat.set_cde_launch(rows)
    lat.set_source(R)
    fields = _fields(wl.mask.shape, 5)
    for k, (ux, uy) in enumerate(fields):
        lat.set_velocity_field(k, ux, uy)
    lat.set_phase_fields([0, 1])
    f0, _ = lat.populations()
    log(f"cde given fields, {storage}")
    lat.cde_step(18)
    lat.cde_step(22)
    o = Oracle(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, rho0=wl.rho0, k_decay=wl.k_decay,
               segments=wl.segments, schedule=wl.schedule, R=R)
    o.init(**init)
    o.cde_step(40, fields, phase_field=[0, 1])
    fluid = wl.mask == 0
    f = _compare(lat, o, fluid, storage, f"given fields {storage}")
    assert np.array_equal(f, f0)
    d = lat.diagnostics()
    assert d["t"] == 40
    tol = {"f64": 1e-11, "f32": 1e-4, "f16": 2e-2}[storage]
    for sid in (2, 3, 4, 5):
        assert d["seg_mass"][sid - 2] == 0.0
        assert d["seg_solute"][sid - 2] == pytest.approx(o.flux_solute[sid], rel=tol, abs=1e-9)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_captured_field_odd_start_then_coupled(storage):
    """Coupled steps to an odd t, the velocity of that state captured, the
    compound alone for 24 steps, then coupled steps again: the oracle does
    the same with the velocity of its own fluid state."""
    wl = W.gradient_generator(nx=300, ny=150, half_period=9, storage=storage)
    init = seeded_init(wl, 8)
    lat = make_lattice(wl, storage, init, chunk=8)
    o = make_oracle(wl)
    o.init(**init)
    lat.step(13)
    o.step(13)
    lat.set_velocity_field(0, scale=2.0)  # a power of two: the same product on both sides
    _, ux, uy, _ = o.fields()
    log(f"cde captured field, odd start, {storage}")
    lat.cde_step(24)
    o.cde_step(24, [(2.0 * np.nan_to_num(ux), 2.0 * np.nan_to_num(uy))])
    fluid = wl.mask == 0
    _compare(lat, o, fluid, storage, f"captured field {storage}")
    lat.step(7)
    o.step(7)
    _compare(lat, o, fluid, storage, f"coupled after cde {storage}")
    assert lat.info()["t"] == 44


def test_periodic_uniform_field_graphs():
    """Random obstacles on a periodic 133x71 lattice, a uniform field given
    with a scale factor, 64 steps as 4 graph replays of 16, FP64."""
    mask = W.random_mask(133, 71, seed=5, periodic=(True, True))
    wl = W.Workload("random", mask, tau_f=0.7, D=0.03, periodic=(True, True))
    init = seeded_init(wl, 2)
    lat = make_lattice(wl, "f64", init, chunk=16)
    u = (np.full(mask.shape, 0.004), np.full(mask.shape, -0.0024))
    lat.set_velocity_field(3, *u, scale=12.5)  # scaled in FP64, as below
    lat.set_phase_fields([3])
    lat.cde_step(64)
    o = make_oracle(wl)
    o.init(**init)
    o.cde_step(64, [(12.5 * u[0], 12.5 * u[1])])
    _compare(lat, o, mask == 0, "f64", "periodic uniform")


def test_argument_and_state_errors():
    wl = W.gradient_generator(nx=300, ny=150, half_period=7, storage="f32")
    lat = make_lattice(wl, "f32", seeded_init(wl, 1))
    with pytest.raises(GGError) as e:
        lat.cde_step(2)  # no field set
    assert e.value.status == GG_ERR_STATE
    lat.set_velocity_field(0)
    with pytest.raises(GGError) as e:
        lat.cde_step(3)  # odd n would leave the fluid planes in the wrong layout
    assert e.value.status == GG_ERR_ARG
    lat.set_phase_fields([0, 2])
    with pytest.raises(GGError) as e:
        lat.cde_step(2)  # phase 1 names slot 2, never set
    assert e.value.status == GG_ERR_STATE
    with pytest.raises(GGError) as e:
        lat.set_velocity_field(16)
    assert e.value.status == GG_ERR_ARG
    lat.set_phase_fields(None)
    lat.cde_step(2)
    assert lat.info()["t"] == 2


def test_full_size_gradient_generator_f32():
    """The 2048x1024 FP32 gradient generator in the launch form the bench
    times (graph replays of 64 steps): 200 compound-only steps on the
    velocity captured from the initial state against the oracle on the
    whole field, and the solute balance (change = net inflow, no source)."""
    import bench
    wl = W.gradient_generator()
    init = seeded_init(wl, 4703)
    lat = make_lattice(wl, "f32", init)
    lat.set_cde_launch([r for n, _, _, r in bench.CDE_LEG if n == "gg2048_f32"][0])
    lat.set_velocity_field(0)
    d0 = lat.diagnostics()
    log("cde full size 2048x1024 f32, 200 steps")
    lat.cde_step(200)
    d1 = lat.diagnostics()
    o = make_oracle(wl)
    o.init(**init)
    _, ux, uy, _ = o.fields()
    o.cde_step(200, [(np.nan_to_num(ux), np.nan_to_num(uy))])
    _compare(lat, o, wl.mask == 0, "f32", "full size f32")
    net_in = sum(d1["seg_solute"]) - sum(d0["seg_solute"])
    assert d1["solute"] - d0["solute"] == pytest.approx(net_in, rel=1e-5, abs=1e-6 * d0["solute"])
    assert d1["mass"] == d0["mass"]


def _cde_pair(wl, storage, seed, rows, chunk=0, R=None):
    init = seeded_init(wl, seed)
    out = []
    for r in (0, rows):
        lat = make_lattice(wl, storage, init, chunk=chunk)
        if R is not None:
            lat.set_source(R)
        lat.set_cde_launch(r)
        out.append(lat)
    return out


def _same_compound(one, two, t):
    fa, ga = one.populations()
    fb, gb = two.populations()
    assert one.info()["t"] == two.info()["t"] == t
    assert np.array_equal(fa, fb)
    if not np.array_equal(ga, gb):
        bad = np.argwhere(np.any(ga != gb, axis=0))
        raise AssertionError(f"{len(bad)} nodes differ, first {bad[:5].tolist()}")
    da, db = one.diagnostics(), two.diagnostics()
    for a, b in zip(da["seg_solute"], db["seg_solute"]):
        assert b == pytest.approx(a, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("rows", [6, 14, -6, -10])
def test_passes_equal_single_steps(storage, rows):
    """Two (rows > 0) or four (rows < 0) compound-only steps per pass
    against single steps, bit for bit:
    ragged gradient generator, valves switching every 7 steps (inside and
    between the steps of a pass) with a field per phase, a source and decay,
    odd starts and leftovers, graph replays."""
    wl = W.gradient_generator(nx=300, ny=150, half_period=7, storage=storage)
    wl.k_decay = 1e-3
    rng = np.random.default_rng(3)
    R = np.zeros(wl.mask.shape)
    R[40:60, 100:150] = 1e-3 * rng.random((20, 50))
    one, two = _cde_pair(wl, storage, 12, rows, chunk=8, R=R)
    fields = _fields(wl.mask.shape, 7)
    for lat in (one, two):
        for k, (ux, uy) in enumerate(fields):
            lat.set_velocity_field(k, ux, uy)
        lat.set_phase_fields([1, 0])
    log(f"cde passes vs single steps, {storage}, rows {rows}")
    for lat in (one, two):
        lat.step(3)        # odd t
        lat.cde_step(10)   # a single step, two passes, leftovers
        lat.cde_step(30)   # graph replays from an odd t
        lat.step(1)        # even t
        lat.cde_step(22)
    _same_compound(one, two, 66)


@pytest.mark.parametrize("rows", [14, -6])
@pytest.mark.parametrize("periodic", [(True, False), (False, True), (True, True), (False, False)])
def test_passes_random_masks_periodic(periodic, rows):
    mask = W.random_mask(133, 71, seed=7, periodic=periodic)
    wl = W.Workload("random", mask, tau_f=0.7, D=0.03, periodic=periodic)
    one, two = _cde_pair(wl, "f64", 3, rows)
    u = _fields(mask.shape, 2)[0]
    for lat in (one, two):
        lat.set_velocity_field(0, *u)
        lat.cde_step(36)
    _same_compound(one, two, 36)
    o = make_oracle(wl)
    o.init(**seeded_init(wl, 3))
    o.cde_step(36, [u])
    _compare(two, o, mask == 0, "f64", f"passes periodic {periodic}")


def test_autotuner_keeps_the_result(tmp_path):
    """tune_cde times single steps and the four pass forms, applies the
    fastest, and the state it leaves equals single steps over as many steps."""
    from paper_1307_4703_amd import tune
    wl = W.gradient_generator(nx=300, ny=150, half_period=9, storage="f32")
    one, two = _cde_pair(wl, "f32", 6, 14, chunk=8)
    for lat in (one, two):
        lat.set_velocity_field(0)
    res = tune.tune_cde(two, steps=16, path=str(tmp_path / "tune.json"), use_cache=False)
    assert res["rows"] in (0, 6, 14, -6, -10) and len(res["all"]) == 5
    one.cde_step(5 * (4 + 16))  # per candidate: 4 warm-up and 16 timed steps
    _same_compound(one, two, 100)


def test_host_field_beyond_positivity_limit_refused():
    """Host fields whose scaled components exceed c_sg^2 = (1 - w0) / 2 (where
    the compound's linear equilibrium turns negative) are refused; at the
    limit they are taken (the paper's D2Q4 runs at U = 1/2 exactly)."""
    from paper_1307_4703_amd._abi import GGError, GG_ERR_ARG
    mask = np.zeros((16, 32), np.uint8)
    for w0, ok_speed in ((1.0 / 3.0, 1.0 / 3.0), (0.0, 0.5)):
        lat = Lattice(mask, tau_f=0.8, D=0.02, w0=w0, periodic=(True, True), storage="f64")
        ux = np.full(mask.shape, ok_speed)
        uy = np.zeros(mask.shape)
        lat.set_velocity_field(0, ux, uy)
        with pytest.raises(GGError) as e:
            lat.set_velocity_field(1, ux, uy, scale=1.01)
        assert e.value.status == GG_ERR_ARG
        with pytest.raises(GGError):
            lat.set_velocity_field(1, uy, -1.2 * ux)
        lat.close()
