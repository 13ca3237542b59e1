"""CPU pins of the storage-rounded step emulator (tests/emu), the instrument
the GPU bit-level tests compare against: its binary16 rounding equals
numpy's round-to-nearest-even conversion on every half value, ties and
subnormals included; run in FP64 it follows the FP64 oracle step for step
(the same scheme, paper Eqs. 4-9, and link rules, in another operation
order); run in FP32 and with binary16 storage it stays within the FP32 and
FP16 tolerances of the oracle."""
import ctypes

import numpy as np
import pytest

from tests.emu import emu
from tests.emu_cases import cases
from tests.parity_util import make_oracle, seeded_init
from tests.test_gpu_parity import F16_TOL, F32_TOL

W9 = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def test_half_rounding_matches_numpy():
    L = emu.lib("f32")
    rng = np.random.default_rng(0)
    # every binary16 value back to binary32, and the midpoints between
    # neighbouring halves (exact ties), nudged up and down by one ulp
    bits = np.arange(0, 1 << 16, dtype=np.uint32).astype(np.uint16)
    hv = bits.view(np.float16).astype(np.float32)
    for b, v in zip(bits[::7], hv[::7]):
        got = L.emu_from_half(int(b))
        assert (np.isnan(v) and np.isnan(got)) or np.float32(got).tobytes() == v.tobytes()
    fin = np.isfinite(hv) & (hv >= 0)
    pos = np.sort(np.unique(hv[fin]))
    mid = ((pos[:-1].astype(np.float64) + pos[1:]) / 2).astype(np.float32)
    vals = np.concatenate([mid, np.nextafter(mid, np.float32(np.inf)),
                           np.nextafter(mid, np.float32(0)),
                           rng.standard_normal(20000).astype(np.float32) *
                           np.float32(10.0) ** rng.integers(-9, 5, 20000).astype(np.float32),
                           np.array([65504, 65519.99, 65520, 7e4, 1e-8, 2.0 ** -25, 2.0 ** -24,
                                     3 * 2.0 ** -26, 0.0], np.float32)])
    vals = np.concatenate([vals, -vals])
    sel = vals[:: max(1, len(vals) // 60000)]
    with np.errstate(over="ignore"):
        want = sel.astype(np.float16).view(np.uint16)
    got = np.array([L.emu_to_half(ctypes.c_float(float(v))) for v in sel], np.uint16)
    assert np.array_equal(got, want)


def test_fluid_collision_constants_exact():
    """The fluid's relaxation constants (om w_axis rounded so that 9 om
    w_axis, 1 - 9 om w_axis and every weight product are exact in the
    compute type, the kernels' and the replay's shared rule): for FP32 and
    FP64 and relaxation rates over (0, 2), each constant is representable,
    the products with the weights are exact, the rest and the moving
    weights add up to the rate exactly, and the rate stays within 2^(4-p)
    relative (2^-(p+1) 9/om absolute below om = 9/32)."""
    L = emu.lib("f64")
    rng = np.random.default_rng(7)
    oms = np.concatenate([rng.uniform(0.02, 1.999, 3000), [1 / 0.8, 1.0, 0.5, 1.9, 9 / 32, 0.05]])
    for p, ftype in ((24, np.float32), (53, np.float64)):
        for om in oms:
            ka = L.emu_fluid_ka(float(om), p)
            k = ftype(ka)
            assert float(k) == ka                                  # representable
            rate = ftype(9) * k
            assert float(rate) == 9 * ka                           # 9 ka exact
            omc = ftype(1) - rate
            assert float(omc) == 1 - 9 * ka                        # 1 - 9 ka exact
            assert float(ftype(3) * k) == 3 * ka
            assert float(ftype(4) * k) == 4 * ka
            assert float(k * ftype(0.25)) == ka / 4
            # rest + 4 axis + 4 diagonal products sum to the rate exactly
            assert 4 * ka + 4 * ka + 4 * (ka / 4) == 9 * ka
            tol = 2.0 ** (4 - p) * om if om >= 9 / 32 else 2.0 ** -(p + 1) * 9
            assert abs(9 * ka - om) <= tol * (1 + 1e-12)


def _deviations(o, rho0, c_shift, w0):
    wg = np.array([w0] + [(1 - w0) / 4] * 4)
    h = np.moveaxis(o.f, 2, 0) - W9[:, None, None] * rho0
    k = np.moveaxis(o.g, 2, 0) - wg[:, None, None] * c_shift
    return h, k, wg


def _fields(h, k, rho0, c_shift):
    h = h.astype(np.float64)
    k = k.astype(np.float64)
    rho = rho0 + h.sum(0)
    ux = (CX[:, None, None] * h).sum(0) / rho
    uy = (CY[:, None, None] * h).sum(0) / rho
    return rho, ux, uy, c_shift + k.sum(0)


@pytest.mark.parametrize("name", ["gradient_generator", "random_source_decay", "straight_channel"])
def test_emulator_f64_follows_oracle(name):
    wl, R = cases()[name]
    o = make_oracle(wl)
    if R is not None:
        o = type(o)(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, rho0=wl.rho0,
                    k_decay=wl.k_decay, periodic=wl.periodic, segments=wl.segments,
                    schedule=wl.schedule, R=R)
    o.init(**seeded_init(wl, 11))
    h, k, wg = _deviations(o, wl.rho0, 0.0, wl.w0)
    e = emu.Emulator(wl, "f64", R=R)
    fl = wl.mask == 0
    t = 0
    for n in (1, 6, 13):
        h, k = e.step(h, k, t, n)
        o.step(n)
        t += n
        f = h + W9[:, None, None] * wl.rho0
        g = k
        fo = np.moveaxis(o.f, 2, 0)
        go = np.moveaxis(o.g, 2, 0)
        assert np.abs(f[:, fl] - fo[:, fl]).max() <= 1e-13 * np.abs(fo[:, fl]).max()
        assert np.abs(g[:, fl] - go[:, fl]).max() <= 1e-13 * max(1.0, np.abs(go[:, fl]).max())


@pytest.mark.parametrize("storage,tol", [("f32", F32_TOL), ("f16", F16_TOL)])
@pytest.mark.parametrize("name", ["gradient_generator", "random_source_decay"])
def test_emulator_reduced_precision_near_oracle(name, storage, tol):
    wl, R = cases()[name]
    o = make_oracle(wl)
    if R is not None:
        o = type(o)(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, rho0=wl.rho0,
                    k_decay=wl.k_decay, periodic=wl.periodic, segments=wl.segments,
                    schedule=wl.schedule, R=R)
    o.init(**seeded_init(wl, 12))
    cs = 0.5 if storage == "f16" else 0.0
    h, k, wg = _deviations(o, wl.rho0, cs, wl.w0)
    dt = np.float32
    h = h.astype(dt)
    k = k.astype(dt)
    if storage == "f16":
        h = h.astype(np.float16).astype(dt)
        k = k.astype(np.float16).astype(dt)
    e = emu.Emulator(wl, storage, c_shift=cs, R=R)
    h, k = e.step(h, k, 0, 40)
    o.step(40)
    fl = wl.mask == 0
    rho, ux, uy, C = _fields(h, k, wl.rho0, cs)
    ro, uxo, uyo, Co = o.fields()
    umax = max(np.abs(uxo[fl]).max(), np.abs(uyo[fl]).max())
    assert np.abs(rho - ro)[fl].max() / wl.rho0 <= tol["rho"]
    assert max(np.abs(ux - uxo)[fl].max(), np.abs(uy - uyo)[fl].max()) / umax <= tol["u"]
    assert np.abs(C - Co)[fl].max() / max(1.0, np.abs(Co[fl]).max()) <= tol["C"]
