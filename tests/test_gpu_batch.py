"""Batched launch: many uneven lattices in one flat launch per step must give
bitwise the same states as stepping each lattice on its own (same kernels,
same arithmetic, only the work-group to tile assignment differs)."""
import numpy as np
import pytest

from paper_1307_4703_amd import Batch, Lattice, _abi as A, workloads as W
from tests.parity_util import log, seeded_init

pytestmark = pytest.mark.gpu


def _members():
    wls = [W.gradient_generator(nx=256, ny=128, half_period=9, storage="f32"),
           W.gradient_generator(nx=384, ny=192, half_period=14, peclet=1500.0, storage="f32",
                                chamber_width=300),
           W.gradient_generator(nx=300, ny=150, half_period=5, storage="f32"),
           W.straight_channel(96, 40, storage="f32")]
    m = W.random_mask(131, 67, seed=3, periodic=(True, False))
    wls.append(W.Workload("random", m, tau_f=0.7, D=0.02, periodic=(True, False), storage="f32"))
    return wls


def _make(wls, seed0=0):
    lats = []
    for k, wl in enumerate(wls):
        lat = Lattice.from_workload(wl, init=False)
        lat.init(**seeded_init(wl, seed0 + k))
        lats.append(lat)
    return lats


def _states(lats):
    return [lat.populations() for lat in lats]


@pytest.mark.parametrize("tile,persist,chunk", [((64, 4), 0, 8), ((32, 8), 64, 0),
                                                ((128, 2), 512, 16)])
def test_batch_equals_individual(tile, persist, chunk):
    wls = _members()
    log(f"batch tile {tile} persist {persist} chunk {chunk}")
    ref = _make(wls)
    for lat in ref:
        lat.step(53)
    lats = _make(wls)
    b = Batch(lats, tile=tile, persist=persist, graph_chunk=chunk)
    b.step(20)
    b.step(33)
    b.close()
    for (fa, ga), (fb, gb) in zip(_states(ref), _states(lats)):
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    for lat in lats:
        assert lat.info()["t"] == 53


@pytest.mark.parametrize("fuse,rows,chunk", [(4, 6, 8), (3, 6, 0), (3, 14, 16), (5, 6, 8),
                                             (5, 14, 0)])
def test_batch_two_step_equals_individual(fuse, rows, chunk):
    """Two-step passes over all members in one launch (boundary tiles in the
    same kernel, or in their own beside it), or four-step passes with runs
    of 8k + 4 steps ending in two-step ones, == each member on its own, also
    when the batch starts at odd member steps."""
    wls = _members()
    log(f"batch two-step fuse {fuse} rows {rows} chunk {chunk}")
    ref = _make(wls)
    lats = _make(wls)
    for lat in ref + lats:
        lat.step(1)
    for lat in ref:
        lat.set_two_step(1)
        lat.step(45)
    b = Batch(lats, graph_chunk=chunk, fuse=fuse, rows=rows)
    b.step(20)
    b.step(13)
    b.step(12)
    b.close()
    for (fa, ga), (fb, gb) in zip(_states(ref), _states(lats)):
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    for lat in lats:
        assert lat.info()["t"] == 46


def test_batch_two_step_needs_one_parity():
    wls = _members()[:2]
    lats = _make(wls)
    lats[0].step(1)
    b = Batch(lats)
    with pytest.raises(A.GGError) as e:
        b.set_two_step(4, 6)
    assert e.value.status == A.GG_ERR_STATE


def test_batch_four_step_pass_needs_periodic_axes_of_four():
    mask = np.zeros((3, 40), np.uint8)
    wl = W.Workload("thin", mask, tau_f=0.9, D=0.02, periodic=(True, True), storage="f32")
    lats = _make([wl])
    b = Batch(lats)
    with pytest.raises(A.GGError) as e:
        b.set_two_step(5, 6)
    assert e.value.status == A.GG_ERR_ARG
    b.close()


def test_batch_members_at_different_parities():
    wls = _members()
    ref = _make(wls)
    lats = _make(wls)
    for k in (1, 3):
        ref[k].step(1)
        lats[k].step(1)
    for lat in ref:
        lat.step(17)
    b = Batch(lats, graph_chunk=4)
    b.step(17)
    for (fa, ga), (fb, gb) in zip(_states(ref), _states(lats)):
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


def test_batch_refuses_members_stepped_outside():
    wls = _members()[:2]
    lats = _make(wls)
    b = Batch(lats)
    b.step(3)
    lats[0].step(1)
    with pytest.raises(A.GGError) as e:
        b.step(1)
    assert e.value.status == A.GG_ERR_STATE


def test_autotuner_picks_and_caches(tmp_path):
    from paper_1307_4703_amd import tune
    wl = W.gradient_generator(nx=512, ny=256, storage="f32")
    lat = Lattice.from_workload(wl)
    path = str(tmp_path / "tune.json")
    res = tune.tune_lattice(lat, steps=16, tiles=((64, 4), (32, 8), (128, 2)),
                            two_step=((3, 6), (4, 14)), path=path)
    assert tuple(res["tile"]) in ((64, 4), (32, 8), (128, 2))
    assert (res["fuse"], res["rows"]) in ((1, 6), (3, 6), (4, 14))
    assert len(res["all"]) == 5
    again = tune.tune_lattice(lat, steps=16, path=path)
    assert again["tile"] == res["tile"] and again["fuse"] == res["fuse"]
    wls = _members()[:3]
    lats = _make(wls)
    rb = tune.tune_batch(lats, steps=8, tiles=((64, 4), (32, 8)), persist=(0, 256),
                         two_step=((4, 6),), path=path)
    assert len(rb["all"]) == 5 and rb["persist"] in (0, 256) and rb["fuse"] in (1, 4)


def test_batch_refuses_reconfigured_members():
    """A batch copies its members' descriptors; a member reconfigured after
    the batch was made (its second plane set freed and reallocated, its
    schedule or source changed) makes the batch refuse to run."""
    wls = _members()[:2]
    for change in ("two_step", "schedule", "source"):
        lats = _make(wls)
        b = Batch(lats, fuse=3, rows=6)
        b.step(4)
        if change == "two_step":
            lats[1].set_two_step(1)
            lats[1].set_two_step(3, 6)
        elif change == "schedule":
            lats[0].set_schedule(wls[0].schedule)
        else:
            lats[0].set_source(np.zeros(wls[0].mask.shape))
        with pytest.raises(A.GGError) as e:
            b.step(4)
        assert e.value.status == A.GG_ERR_STATE
        with pytest.raises(A.GGError) as e:
            b.set_two_step(4, 6)
        assert e.value.status == A.GG_ERR_STATE
        b.close()


def test_library_autotuner_leaves_members_and_steps_like_them():
    """gg_batch_create with GG_AUTOTUNE: the members come back unchanged
    from the tuning runs, the batch reports a candidate form, and it steps
    the members exactly as they step on their own."""
    wls = _members()
    ref = _make(wls)
    lats = _make(wls)
    before = _states(lats)
    b = Batch(lats, tile=None, graph_chunk=8)
    f = b.form()
    log(f"library autotune picked {f}")
    assert (f["tile_x"], f["tile_y"]) in ((64, 4), (32, 8), (128, 2))
    # (the library's candidates: single steps, the two-step forms, the
    # four-step pass)
    assert (f["fuse"], f["rows"]) in ((1, 6), (3, 6), (3, 14), (4, 6), (4, 14), (5, 6))
    for (fa, ga), (fb, gb) in zip(before, _states(lats)):
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    for lat in lats:
        assert lat.info()["t"] == 0
    b.step(21)
    for lat in ref:
        lat.step(21)
    for (fa, ga), (fb, gb) in zip(_states(ref), _states(lats)):
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    b.close()
