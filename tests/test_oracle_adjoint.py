"""Pins of the oracle's discrete adjoint of the compound lattice.

The adjoint step is checked against the forward step itself (dot-product
test of the transposed linear map) and the whole adjoint against central
finite differences of the forward oracle. The loss is quadratic in the inlet
concentrations and the source, so central differences are exact there up to
rounding; the diffusion coefficient enters through the relaxation rate and
carries an O(h^2) truncation.
"""
import ctypes

import numpy as np
import pytest

from oracle import Oracle
from oracle import oracle as orc
from paper_1307_4703_amd import workloads as W


def _small_gg(half_period=15, c_source=1.0, c_sink=0.0, **kw):
    wl = W.gradient_generator(nx=160, ny=80, half_period=half_period, storage="f64", **kw)
    wl.schedule = W.alternating_schedule(half_period, c_source, c_sink)
    return wl


def _oracle(wl, R=None, k=0.0, D=None):
    return Oracle(wl.mask, tau_f=wl.tau_f, D=wl.D if D is None else D, w0=wl.w0,
                  k_decay=k, segments=wl.segments, schedule=wl.schedule, R=R)


def _init(wl, seed):
    rng = np.random.default_rng(seed)
    sh = wl.mask.shape
    return {"rho": 1.0 + 0.01 * rng.standard_normal(sh),
            "ux": 0.02 * rng.standard_normal(sh), "uy": 0.02 * rng.standard_normal(sh),
            "C": rng.random(sh)}


@pytest.mark.parametrize("t_phase", [0, 15])
def test_adjoint_step_is_transpose_of_forward_step(t_phase):
    """<M v, w> = <v, M^T w> for the linear part of one compound step, with
    walls, an open inlet, an open outlet, closed valves and decay."""
    wl = _small_gg(c_source=0.0, c_sink=0.0)  # C_in = 0: the step is linear in g
    o = _oracle(wl, k=3e-3)
    o.init(**_init(wl, 1))
    o.step(3)  # a developed, non-equilibrium fluid state
    o.t = t_phase
    rng = np.random.default_rng(2)
    fl = (wl.mask == 0)[:, :, None]
    v = np.where(fl, rng.standard_normal(o.g.shape), 0.0)
    w = np.where(fl, rng.standard_normal(o.g.shape), 0.0)
    f0 = o.f.copy()
    open_, _ = o.phase(o.t)
    assert open_.any()
    # forward: M v
    o.f[...] = f0
    o.g[...] = v
    o.step(1)
    Mv = o.g.copy()
    # adjoint: M^T w
    lam_out = np.zeros_like(w)
    dR = np.zeros(wl.mask.shape)
    dcin = np.zeros(256)
    dom = ctypes.c_double(0.0)
    orc.lib().orc_adjoint_step(ctypes.byref(o._c), orc._ptr(f0), orc._ptr(v),
                               orc._ptr(np.ascontiguousarray(w)), orc._ptr(lam_out),
                               orc._ptr(open_), orc._ptr(dR), orc._ptr(dcin),
                               ctypes.byref(dom))
    lhs = float(np.sum(Mv * w))
    rhs = float(np.sum(v * lam_out))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def _loss(wl, init, steps, weight, target, R=None, D=None, c_source=1.0, c_sink=0.0):
    wl2 = _small_gg(c_source=c_source, c_sink=c_sink)
    o = _oracle(wl2, R=R, D=D)
    o.init(**init)
    o.step(steps)
    C = o.g.sum(axis=2)
    fl = wl.mask == 0
    return 0.5 * float(np.sum(np.where(fl, weight * (C - target) ** 2, 0.0)))


def test_adjoint_gradients_match_central_differences():
    wl = _small_gg()
    init = _init(wl, 3)
    steps = 40
    rng = np.random.default_rng(4)
    weight = np.where(wl.mask == 0, rng.random(wl.mask.shape), 0.0)
    target = rng.random(wl.mask.shape)
    R = np.zeros(wl.mask.shape)
    o = _oracle(wl, R=R)
    o.init(**init)
    loss, dcin, dD, dR = o.adjoint(steps, weight, target)
    assert loss == pytest.approx(_loss(wl, init, steps, weight, target), rel=1e-14)

    h = 1e-2  # exact for a quadratic loss
    for sid, base, kw in ((2, 1.0, "c_source"), (4, 0.0, "c_sink")):
        lp = _loss(wl, init, steps, weight, target, **{kw: base + h})
        lm = _loss(wl, init, steps, weight, target, **{kw: base - h})
        fd = (lp - lm) / (2 * h)
        assert dcin[sid] == pytest.approx(fd, rel=1e-8, abs=1e-12), (sid, dcin[sid], fd)
        assert abs(fd) > 1e-6

    hD = wl.D * 1e-4
    fd = (_loss(wl, init, steps, weight, target, D=wl.D + hD) -
          _loss(wl, init, steps, weight, target, D=wl.D - hD)) / (2 * hD)
    assert dD == pytest.approx(fd, rel=1e-6)

    fl = np.argwhere(wl.mask == 0)
    for k in (0, len(fl) // 3, len(fl) // 2, len(fl) - 1):
        y, x = fl[k]
        Rp = R.copy()
        Rp[y, x] += 1e-3
        Rm = R.copy()
        Rm[y, x] -= 1e-3
        fd = (_loss(wl, init, steps, weight, target, R=Rp) -
              _loss(wl, init, steps, weight, target, R=Rm)) / 2e-3
        assert dR[y, x] == pytest.approx(fd, rel=1e-7, abs=1e-12)
