"""Race freedom and failure detection on the GPU.

Order: the in-place (AA) step reads and writes every slot from its owner
node only, so the state cannot depend on the order in which work-groups
run; shuffling the launch order of the tiles and strips must give the same
state bit for bit, in single steps and in two-step passes.

Failure: a non-finite population anywhere on the fluid must be reported by
the diagnostics (GG_ERR_NONFINITE, with the count) and spread no further
than the stencil allows."""
import numpy as np
import pytest

from paper_1307_4703_amd import workloads as W
from paper_1307_4703_amd._abi import GGError, GG_ERR_NONFINITE
from tests.parity_util import SNAP_DATA, log, make_lattice, seeded_init, snapshot_header, snapshot_slot

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fuse,rows", [(1, 6), (3, 6), (4, 14), (2, 8), (5, 6)])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_tile_order_does_not_matter(fuse, rows, storage):
    wl = W.gradient_generator(nx=300, ny=150, half_period=7, storage=storage)
    init = seeded_init(wl, 13)
    a = make_lattice(wl, storage, init, chunk=8)
    b = make_lattice(wl, storage, init, chunk=8)
    for lat in (a, b):
        lat.set_two_step(fuse, rows)
    b.permute_tiles(4703)
    log(f"tile order, fuse {fuse}, {storage}")
    for n in (8, 3, 29):
        a.step(n)
        b.step(n)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


def test_nonfinite_population_is_reported():
    wl = W.gradient_generator(nx=300, ny=150, half_period=7, storage="f32")
    lat = make_lattice(wl, "f32", seeded_init(wl, 2))
    lat.step(4)
    assert lat.diagnostics()["n_nonfinite"] == 0
    snap = bytearray(lat.save())
    # node (x, y) at node0 + y * pitch + x; f_0 of it poisoned
    h = snapshot_header(snap)
    ys, xs = np.nonzero(wl.mask == 0)
    x, y = int(xs[len(xs) // 2]), int(ys[len(ys) // 2])
    off = SNAP_DATA + 4 * snapshot_slot(h, 0, h["node0"] + y * h["pitch"] + x)
    snap[off:off + 4] = np.array([np.nan], np.float32).tobytes()
    lat.load(bytes(snap))
    with pytest.raises(GGError) as e:
        lat.diagnostics()
    assert e.value.status == GG_ERR_NONFINITE
    d = lat.diagnostics(check_finite=False)
    assert d["n_nonfinite"] == 1
    lat.step(2)
    d = lat.diagnostics(check_finite=False)
    log(f"non-finite nodes after 2 steps: {d['n_nonfinite']}")
    assert 1 < d["n_nonfinite"] <= 25  # within two steps of the poisoned node
