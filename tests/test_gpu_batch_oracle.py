"""Batched launch against the FP64 oracle: every member of a batch of uneven
lattices (gradient generators of different sizes, valve periods and Peclet
numbers, two seeded instances of the 64-instance set, a straight channel and
a periodic random obstacle mask), advanced by gg_batch_step in single steps
(plain and persistent grids, graph replays and plain launches, members at
steps of different parity) and in two-step passes (boundary tiles in their
own kernel or in the one kernel), element by element against the oracle
advanced member by member."""
import numpy as np
import pytest

from paper_1307_4703_amd import Batch, Lattice, workloads as W
from tests.parity_util import field_errors, log, make_oracle, seeded_init
from tests.test_gpu_parity import F32_TOL

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def _members():
    wls = [W.gradient_generator(nx=256, ny=128, half_period=9),
           W.gradient_generator(nx=384, ny=192, half_period=14, peclet=1500.0,
                                chamber_width=300),
           W.gradient_generator(nx=300, ny=150, half_period=5, peclet=150.0),
           W.straight_channel(96, 40)]
    m = W.random_mask(131, 67, seed=3, periodic=(True, False))
    wls.append(W.Workload("random", m, tau_f=0.7, D=0.02, periodic=(True, False)))
    # the two smallest of the seeded 64-instance set (sizes, chamber widths,
    # valve periods and Peclet numbers from its generator)
    inst = sorted(W.batch_instances(64, 4703), key=lambda w: w.nx * w.ny)[:2]
    return wls + inst


def _run(storage, steps, pre, make_batch, split=(None,)):
    wls = _members()
    lats, orcs = [], []
    for k, wl in enumerate(wls):
        init = seeded_init(wl, 40 + k)
        lat = Lattice.from_workload(wl, storage=storage, init=False)
        lat.init(**init)
        o = make_oracle(wl)
        o.init(**init)
        if pre[k % len(pre)]:
            lat.step(pre[k % len(pre)])
            o.step(pre[k % len(pre)])
        lats.append(lat)
        orcs.append(o)
    b = make_batch(lats)
    done = 0
    for n in split:
        n = steps - done if n is None else n
        b.step(n)
        done += n
    b.close()
    for o in orcs:
        o.step(steps)
    errs = []
    for wl, lat, o in zip(wls, lats, orcs):
        e = field_errors(lat, o, wl.mask == 0)
        errs.append((wl.name, e))
        lat.close()
    return errs


@pytest.mark.parametrize("tile,persist,chunk", [((64, 4), 0, 8), ((32, 8), 64, 0)])
def test_batch_single_steps_f64_vs_oracle(tile, persist, chunk):
    log(f"batch vs oracle, single steps, tile {tile} persist {persist} chunk {chunk}")
    errs = _run("f64", 41, pre=(0, 1, 0, 1, 1, 0, 1),
                make_batch=lambda lats: Batch(lats, tile=tile, persist=persist,
                                              graph_chunk=chunk),
                split=(17, None))
    for name, e in errs:
        for k in ("f", "g", "rho", "u", "C"):
            assert e[k] <= F64_TOL, (name, k, e[k])


@pytest.mark.parametrize("fuse,rows,chunk", [(3, 6, 8), (4, 14, 0), (5, 6, 8)])
def test_batch_two_step_f64_vs_oracle(fuse, rows, chunk):
    log(f"batch vs oracle, two-step fuse {fuse} rows {rows} chunk {chunk}")
    errs = _run("f64", 45, pre=(1,),
                make_batch=lambda lats: Batch(lats, graph_chunk=chunk, fuse=fuse, rows=rows),
                split=(20, None))
    for name, e in errs:
        for k in ("f", "g", "rho", "u", "C"):
            assert e[k] <= F64_TOL, (name, k, e[k])


@pytest.mark.parametrize("fuse", [1, 4, 5])
def test_batch_f32_vs_oracle(fuse):
    log(f"batch vs oracle, FP32, fuse {fuse}")
    errs = _run("f32", 60, pre=(0,),
                make_batch=lambda lats: Batch(lats, graph_chunk=8, fuse=fuse, rows=6))
    for name, e in errs:
        for k in ("rho", "u", "C"):
            assert e[k] <= F32_TOL[k], (name, k, e[k])
