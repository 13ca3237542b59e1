"""Pins of the oracle's version of the paper's walls (Boundary Conditions
section): a wall or closed-valve cell s = z - e_i next to fluid node z acts
as a node whose populations are the fluid equilibrium at the density
extrapolated linearly from the fluid (2 rho(z) - rho(z + e_i)) and the
momentum that vanishes linearly at the wall halfway between s and z
(j_s = -j(z)), and, for the compound, the no-flux extrapolation of Guo et
al. (z's concentration, the ghost velocity, z's non-equilibrium part after
the collision).

Pinned by: the ghost-node picture itself, exactly, on the first step from
equilibrium states whose continuation across the wall matches the rules (a
linear density at rest; a shear through zero at the wall; a compound even
about the wall), against the same lattice extended by the ghost row; a rest
state as a fixed point; a compound uniform across the channel staying so;
steady pressure-driven flow settling to a parabola whose no-slip points sit
symmetric about the channel, within a fraction of a cell of the walls, and
moving outward as tau_f grows (the slip of equilibrium walls)."""
import numpy as np
import pytest

from oracle import Oracle
from paper_1307_4703_amd import workloads as W

NX = 24


def _pair(ny_wall=10, valve=False):
    """The walled channel (walls on rows 0 and ny-1, periodic in x; with
    valve, the bottom row is the ghost line of a closed valve instead) and
    the channel extended by one fluid row below (the ghost row of the bottom
    wall), walls beyond."""
    walled = np.zeros((ny_wall, NX), np.uint8)
    walled[0, :] = 2 if valve else 1
    walled[-1, :] = 1
    ext = np.zeros((ny_wall + 1, NX), np.uint8)
    ext[0, :] = 1
    ext[-1, :] = 1
    kw = dict(tau_f=0.8, D=0.02, periodic=(True, False))
    extra = {}
    if valve:
        extra = dict(segments=[W.Segment(2, "inlet", (0, -1), u_max=0.05, c_in=1.0)],
                     schedule=[W.Phase(10, frozenset())])
    return (Oracle(walled, wall_scheme="equilibrium", **kw, **extra),
            Oracle(ext, wall_scheme="bounce_back", **kw))


def _first_step_matches(fields, valve=False):
    """fields(y) -> dict of rho, ux, C at lattice row y of the walled
    channel (y = 0 is the bottom wall row, so the ghost row is y = 0 and
    the first fluid row y = 1); the extended lattice has the ghost row as
    fluid row 1 and the walled row y at y + 1."""
    a, b = _pair(valve=valve)
    ny = a.ny
    def grid(oracle, shift):
        out = {k: np.zeros((oracle.ny, NX)) for k in ("rho", "ux", "uy", "C")}
        out["rho"][:] = 1.0
        for y in range(oracle.ny):
            v = fields(y - shift)
            for k in v:
                out[k][y, :] = v[k]
        return out
    ga, gb = grid(a, 0), grid(b, 1)
    a.init(rho=ga["rho"], ux=ga["ux"], uy=ga["uy"], C=ga["C"])
    b.init(rho=gb["rho"], ux=gb["ux"], uy=gb["uy"], C=gb["C"])
    a.step(1)
    b.step(1)
    # the walled lattice's first fluid row against the extended lattice's
    # same row (one up), every population
    np.testing.assert_allclose(a.f[1], b.f[2], rtol=0, atol=1e-15)
    np.testing.assert_allclose(a.g[1], b.g[2], rtol=0, atol=1e-15)
    return ny


@pytest.mark.parametrize("valve", [False, True])
def test_ghost_density_extrapolated_linearly(valve):
    _first_step_matches(lambda y: {"rho": 1.0 + 0.01 * y}, valve)


def test_ghost_momentum_vanishes_at_the_halfway_wall():
    """Both velocity components through zero at the wall (a flow into the
    wall is no steady state, but the first step only asks what the ghost
    emits), with a uniform compound carried by it."""
    _first_step_matches(lambda y: {"ux": 0.02 * (y - 0.5), "uy": 0.01 * (y - 0.5), "C": 0.5})


def test_ghost_compound_even_about_the_wall():
    _first_step_matches(lambda y: {"C": 0.4 + 0.003 * (y - 0.5) ** 2})


def test_rest_state_is_fixed_point():
    mask = np.ones((12, 16), np.uint8)
    mask[1:-1, 1:-1] = 0
    o = Oracle(mask, tau_f=0.8, D=0.02, wall_scheme="equilibrium")
    fl = mask == 0
    o.init(C=np.where(fl, 0.7, 0.0))
    f0, g0 = o.f.copy(), o.g.copy()
    o.step(50)
    np.testing.assert_allclose(o.f[fl], f0[fl], rtol=0, atol=1e-14)
    np.testing.assert_allclose(o.g[fl], g0[fl], rtol=0, atol=1e-14)


def test_compound_uniform_across_the_channel_stays_so():
    mask = np.ones((20, 64), np.uint8)
    mask[1:-1, :] = 0
    o = Oracle(mask, tau_f=0.8, D=0.02, periodic=(True, False), wall_scheme="equilibrium")
    x = np.arange(64)
    o.init(C=np.where(mask == 0, 0.5 + 0.3 * np.sin(2 * np.pi * x / 64)[None, :], 0.0))
    o.step(200)
    C = o.fields()[3]
    assert np.nanmax(np.ptp(C[1:-1, :], axis=0)) < 1e-13


def _poiseuille_roots(tau):
    nx, ny = 66, 18
    mask = np.zeros((ny, nx), np.uint8)
    mask[0, :] = 1
    mask[-1, :] = 1
    mask[1:-1, 0] = 2
    mask[1:-1, -1] = 3
    segs = [W.Segment(2, "pressure", (-1, 0), rho=1.002, c_in=1.0, fix_c=True),
            W.Segment(3, "pressure", (1, 0), rho=0.998)]
    o = Oracle(mask, tau_f=tau, D=0.02, segments=segs, wall_scheme="equilibrium")
    o.init()
    o.step(6000)
    ux = o.fields()[1]
    y = np.arange(1, ny - 1).astype(float)
    u = ux[1:-1, nx // 2]
    c = np.polyfit(y, u, 2)
    assert np.abs(np.polyval(c, y) - u).max() < 1e-4 * u.max()  # a parabola
    return np.sort(np.roots(c).real), ny - 2


def test_pressure_driven_flow_no_slip_points():
    roots = {}
    for tau in (0.6, 1.0, 1.5):
        r, H = _poiseuille_roots(tau)
        assert r[0] + r[1] == pytest.approx(H + 1, abs=1e-6)  # symmetric about the centre
        assert 0.1 < r[0] < 0.9  # within half a cell of the halfway wall at 0.5
        roots[tau] = r[0]
    assert roots[0.6] > roots[1.0] > roots[1.5]  # the wall slips outward as tau grows


def test_compound_only_step_ghost_rule():
    """The compound-only step's wall rule (the ghost moves at minus the
    frozen velocity of z) against the extended lattice whose ghost row
    carries the continued field and compound, first step from equilibrium."""
    a, b = _pair()
    def rows(o, shift):
        ux = np.zeros((o.ny, NX))
        uy = np.zeros((o.ny, NX))
        C = np.zeros((o.ny, NX))
        for y in range(o.ny):
            yy = y - shift
            ux[y, :] = 0.03 * (yy - 0.5)
            uy[y, :] = 0.01 * (yy - 0.5)
            C[y, :] = 0.4 + 0.003 * (yy - 0.5) ** 2
        return ux, uy, C
    uxa, uya, Ca = rows(a, 0)
    uxb, uyb, Cb = rows(b, 1)
    a.init(ux=uxa, uy=uya, C=Ca)
    b.init(ux=uxb, uy=uyb, C=Cb)
    a.cde_step(1, [(uxa, uya)])
    b.cde_step(1, [(uxb, uyb)])
    np.testing.assert_allclose(a.g[1], b.g[2], rtol=0, atol=1e-15)
