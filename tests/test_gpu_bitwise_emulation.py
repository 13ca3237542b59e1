"""Bit-level check of the storage rounding: the GPU state after some steps
equals, bit for bit, the storage-rounded replay of the kernels' arithmetic
on the CPU (tests/emu: deviation form, the compute type's operations in the
kernels' order with explicit fused multiply-adds, binary16 stores rounded to
nearest even), from the same raw initial state, in FP64, FP32 and
FP16-shifted storage, in single steps and two-step passes. So the FP32 and
FP16 differences from the FP64 oracle are the rounding of this arithmetic
and nothing else (the replay itself follows the oracle, tests/test_emu_pins.py)."""
import numpy as np
import pytest

from paper_1307_4703_amd import Lattice
from tests.emu import emu
from tests.emu_cases import cases
from tests.parity_util import log, seeded_init, snapshot_header, snapshot_planes

pytestmark = pytest.mark.gpu

RAW = {"f64": np.float64, "f32": np.float32, "f16": np.float16}


def _raw_state(lat, storage):
    """Deviation planes (9, ny, nx) and (5, ny, nx) from a snapshot taken at
    an even step (natural order), as values of the compute type."""
    snap = lat.save()
    hd = snapshot_header(snap)
    pitch, t, node0 = hd["pitch"], hd["t"], hd["node0"]
    assert t % 2 == 0
    raw = snapshot_planes(snap, RAW[storage])
    ny, nx = lat.ny, lat.nx
    idx = node0 + np.arange(ny)[:, None] * pitch + np.arange(nx)[None, :]
    vals = raw[:, idx]
    ct = np.float64 if storage == "f64" else np.float32
    return vals[:9].astype(ct), vals[9:].astype(ct), t


@pytest.mark.parametrize("layout", ["paired", "planes"])
@pytest.mark.parametrize("fuse", [1, 3, 4])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("name", ["gradient_generator", "random_source_decay", "straight_channel"])
def test_gpu_state_equals_storage_rounded_replay(name, storage, fuse, layout):
    wl, R = cases()[name]
    cs = wl.c_shift if storage == "f16" else 0.0
    lat = Lattice.from_workload(wl, storage=storage, init=False, layout=layout)
    lat.init(**seeded_init(wl, 21))
    if R is not None:
        lat.set_source(R)
    lat.set_launch(64, 4, 8)
    lat.set_two_step(fuse, 6)
    h, k, t = _raw_state(lat, storage)
    e = emu.Emulator(wl, storage, c_shift=cs, R=R)
    fl = wl.mask == 0
    log(f"bitwise replay {name} {storage} fuse {fuse} layout {layout}")
    for n in (2, 10, 12):
        lat.step(n)
        h, k = e.step(h, k, t, n)
        t += n
        hg, kg, tg = _raw_state(lat, storage)
        assert tg == t
        bad_h = np.argwhere(~(hg == h)[:, fl])
        bad_k = np.argwhere(~(kg == k)[:, fl])
        assert len(bad_h) == 0 and len(bad_k) == 0, (t, len(bad_h), len(bad_k))
    lat.close()
