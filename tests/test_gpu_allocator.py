"""Device memory from the caller's allocator (gg_create_ex): a lattice whose
every buffer comes from PyTorch's caching allocator steps, reads back,
runs the compound alone and the adjoint exactly as one on hipMalloc (bit
for bit), the memory shows in PyTorch's accounting while the lattice lives
and goes back when it is destroyed, and an allocator that fails makes the
creation fail cleanly."""
import ctypes

import numpy as np
import pytest

from paper_1307_4703_amd import Lattice
from paper_1307_4703_amd import _abi as A
from paper_1307_4703_amd import workloads as W
from tests.parity_util import log, seeded_init

pytestmark = pytest.mark.gpu


def _pair(storage):
    import torch
    wl = W.gradient_generator(nx=300, ny=150, half_period=9, storage=storage)
    init = seeded_init(wl, 21, amp_u=0.005)
    base = torch.cuda.memory_allocated()
    a = Lattice.from_workload(wl, storage=storage, init=False)
    b = Lattice.from_workload(wl, storage=storage, init=False, device_allocator="torch")
    held = torch.cuda.memory_allocated() - base
    for lat in (a, b):
        lat.init(**init)
    return wl, init, a, b, held


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_steps_and_compound_only_match_hipmalloc(storage):
    import torch
    wl, init, a, b, held = _pair(storage)
    esize = {"f64": 8, "f32": 4, "f16": 2}[storage]
    info = b.info()
    log(f"torch allocator {storage}: {held} bytes held by the lattice")
    # at least the two plane sets of 14 populations
    assert held >= 2 * 14 * (wl.ny + 2) * wl.nx * esize
    for n in (3, 16, 64, 5):
        a.step(n)
        b.step(n)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb, equal_nan=True) and np.array_equal(ga, gb, equal_nan=True)
    for lat in (a, b):
        lat.set_velocity_field(0)
        lat.cde_step(40)
    assert np.array_equal(a.read()[3], b.read()[3], equal_nan=True)
    assert info["n_fluid"] == a.info()["n_fluid"]
    before = torch.cuda.memory_allocated()
    b.close()
    a.close()
    assert torch.cuda.memory_allocated() < before  # handed back on destroy


def test_adjoint_matches_hipmalloc():
    wl, init, a, b, _ = _pair("f32")
    weight, target, r_box = W.chamber_misfit_setup(wl)
    ga = a.adjoint(300, weight, target, r_box=r_box)
    gb = b.adjoint(300, weight, target, r_box=r_box)
    assert ga["loss"] == gb["loss"] and ga["d_D"] == gb["d_D"]
    assert np.array_equal(ga["d_R"], gb["d_R"])
    # (dL/dC_in is summed with FP64 atomics: equal up to the order of the sums)
    np.testing.assert_allclose(ga["d_c_in"], gb["d_c_in"], rtol=1e-12, atol=0)
    a.close()
    b.close()


def test_failing_allocator_fails_the_creation():
    calls = []

    def alloc(nbytes, _ctx):
        calls.append(nbytes)
        return None

    def release(ptr, _ctx):
        raise AssertionError("nothing was allocated")

    al = A.gg_alloc(A.GG_ALLOC_FN(alloc), A.GG_RELEASE_FN(release), None)
    mask = np.zeros((32, 64), np.uint8)
    p = A.gg_params(0.8, 0.02, 1.0 / 3.0, 1.0, 0.0, 0.0, 1, 1)
    h = ctypes.c_void_p()
    with pytest.raises(A.GGError) as e:
        A.call("gg_create_ex", mask.ctypes.data_as(ctypes.c_void_p), 64, 32, ctypes.byref(p),
               A.STORAGE["f32"], None, ctypes.byref(al), ctypes.byref(h))
    assert e.value.status == A.GG_ERR_OOM
    assert len(calls) == 1 and not h.value
