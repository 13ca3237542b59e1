"""Pins of the oracle's compound-only step on a frozen velocity field (the
paper's decoupled production path, Results section).

The compound-only step is written apart from the coupled step. It is tied
(1) to the coupled step, itself pinned by closed forms: fed at every step
with the velocity the coupled step's fluid has at that step, it must give
exactly the coupled step's compound, through valve switches, inlets,
outlets, walls, a source and decay; (2) to the exact spectral evolution of
the compound lattice under a uniform velocity; (3) to conservation in a
closed box under an arbitrary frozen field.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_1307_4703_amd import workloads as W

EX = np.array([0, 1, 0, -1, 0])
EY = np.array([0, 0, 1, 0, -1])


def _gg_pair(half_period=9, k_decay=1e-3, seed=3):
    wl = W.gradient_generator(nx=256, ny=128, half_period=half_period)
    rng = np.random.default_rng(seed)
    R = np.zeros(wl.mask.shape)
    R[50:70, 90:130] = 1e-3 * rng.random((20, 40))
    mk = lambda: Oracle(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, k_decay=k_decay,
                        segments=wl.segments, schedule=wl.schedule, R=R)
    a, b = mk(), mk()
    sh = wl.mask.shape
    fl = wl.mask == 0
    init = dict(rho=np.where(fl, 1 + 0.01 * rng.standard_normal(sh), 1.0),
                ux=np.where(fl, 0.02 * rng.standard_normal(sh), 0.0),
                uy=np.where(fl, 0.02 * rng.standard_normal(sh), 0.0),
                C=np.where(fl, rng.random(sh), 0.0))
    a.init(**init)
    b.init(**init)
    return wl, a, b


def test_cde_step_equals_the_coupled_compound_update():
    """Coupled run a; compound-only run b fed with a's fluid velocity of the
    same step: identical compound populations and solute fluxes, step after
    step, across several valve switches (phases of 9 steps)."""
    wl, a, b = _gg_pair()
    for _ in range(40):
        _, ux, uy, _ = a.fields()
        ux = np.nan_to_num(ux)
        uy = np.nan_to_num(uy)
        a.step(1)
        b.cde_step(1, [(ux, uy)])
    assert np.array_equal(a.g, b.g)
    assert np.array_equal(a.flux_solute, b.flux_solute)
    assert b.t == a.t == 40
    # the fluid of the compound-only run stayed as it was
    _, a0, _ = _gg_pair()
    assert np.array_equal(b.f, a0.f)


def test_cde_phase_fields():
    """phase_field picks the frozen field per schedule phase: with the
    field of each phase equal to the coupled fluid's velocity at that step,
    the result matches the per-step feed above."""
    wl, a, b = _gg_pair(half_period=5)
    fields, per_step = [], []
    for t in range(20):
        _, ux, uy, _ = a.fields()
        per_step.append((np.nan_to_num(ux), np.nan_to_num(uy)))
        a.step(1)
    # two constant fields, one per phase, applied through the schedule
    f0 = (np.full(wl.mask.shape, 0.01), np.full(wl.mask.shape, -0.02))
    f1 = (np.full(wl.mask.shape, -0.03), np.full(wl.mask.shape, 0.005))
    c1, c2 = _gg_pair(half_period=5)[1:]
    c1.cde_step(20, [f0, f1], phase_field=[0, 1])
    for t in range(20):
        c2.cde_step(1, [f0 if (t // 5) % 2 == 0 else f1])
    assert np.array_equal(c1.g, c2.g)


def test_cde_uniform_velocity_exact_fourier_evolution():
    """Uniform frozen u on a periodic lattice: each Fourier mode evolves by
    diag(exp(-i k.e_j)) [(1 - w) I + w W(u) 1^T]; 30 steps against numpy."""
    nx = ny = 16
    w0, tau_g = 1 / 3, 0.58
    mask = np.zeros((ny, nx), np.uint8)
    o = Oracle(mask, tau_f=0.8, D=1.0, w0=w0, periodic=(True, True), tau_g=tau_g)
    rng = np.random.default_rng(4)
    o.g[...] = 0.2 + 0.05 * rng.random(o.g.shape)
    g0 = o.g.copy()
    u = (0.09, 0.04)
    o.cde_step(30, [(np.full((ny, nx), u[0]), np.full((ny, nx), u[1]))])
    cs2 = (1 - w0) / 2
    wg = np.array([w0] + [(1 - w0) / 4] * 4)
    Wu = wg * (1 + (EX * u[0] + EY * u[1]) / cs2)
    om = 1 / tau_g
    A = (1 - om) * np.eye(5) + om * np.outer(Wu, np.ones(5))
    G = np.fft.fft2(g0, axes=(0, 1))
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    out = np.empty_like(G)
    for a_ in range(ny):
        for b_ in range(nx):
            Sh = np.diag(np.exp(-1j * (kx[b_] * EX + ky[a_] * EY)))
            out[a_, b_] = np.linalg.matrix_power(Sh @ A, 30) @ G[a_, b_]
    np.testing.assert_allclose(o.g, np.real(np.fft.ifft2(out, axes=(0, 1))), atol=1e-12)


def test_cde_closed_box_conserves_solute():
    """Valves closed, any frozen velocity field: bounce-back on every
    boundary link conserves the compound exactly."""
    wl = W.gradient_generator(nx=256, ny=128, half_period=50)
    o = Oracle(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, segments=wl.segments,
               schedule=[W.Phase(100, frozenset())])
    rng = np.random.default_rng(12)
    sh = wl.mask.shape
    fl = wl.mask == 0
    o.init(C=np.where(fl, rng.random(sh), 0.0))
    _, s0 = o.totals()
    o.cde_step(150, [(0.05 * rng.standard_normal(sh), 0.05 * rng.standard_normal(sh))])
    _, s1 = o.totals()
    assert s1 == pytest.approx(s0, rel=1e-13)
    assert np.all(o.flux_solute == 0)
