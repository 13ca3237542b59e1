"""Seeded synthetic inputs: masks, boundary segments, valve schedules.

This module describes WHAT is simulated and holds none of the lattice
Boltzmann arithmetic. The same objects are handed both to the HIP library and,
in the tests, to the FP64 oracle.

Mask convention: ``mask[y, x]`` (x fastest in memory), 0 = fluid, 1 = wall,
2..17 = ghost cells of boundary segment ``id``. A segment is a straight line of
ghost cells next to the fluid; its ``normal`` points from the fluid into the
ghost line.

The gradient-generator layout follows the paper's description of the chip
(Experimental Layout and Conditions section): two parallel channels, each
opened by a valve at its inlet and outlet, joined by a pre-chamber and a
cell chamber. The paper's figure with the exact dimensions is not available,
so the dimensions below are synthetic: 100-cell channels of length 1000, a
200 x 100 pre-chamber on each side and a 600 x 400 chamber at 1 um per cell,
with x across the channels and y along them. The fence and dead-end channels
are left out.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, FrozenSet, List, Optional, Tuple

import numpy as np

FLUID = 0
WALL = 1
FIRST_SEGMENT = 2
MAX_SEGMENTS = 16


@dataclass(frozen=True)
class Segment:
    """A boundary segment: a line of ghost cells with a mask value ``id``.

    kind   : "inlet" (velocity inlet carrying a parabolic profile of centre
             speed ``u_max`` and compound concentration ``c_in``),
             "outlet" (zero-gradient outflow) or "pressure" (the paper's
             pressure boundary holding density ``rho``, and, with
             ``fix_c``, the compound at ``c_in``).
    normal : outward unit normal (from the fluid into the ghost line).
    """
    id: int
    kind: str
    normal: Tuple[int, int]
    u_max: float = 0.0
    c_in: float = 0.0
    rho: float = 1.0
    fix_c: bool = False


@dataclass(frozen=True)
class Phase:
    """One entry of a periodic valve schedule.

    duration : number of time steps the phase lasts.
    open     : ids of the segments that are open; every other segment acts
               as a closed valve (a wall).
    c_in     : per-segment inlet concentrations overriding ``Segment.c_in``
               during this phase.
    """
    duration: int
    open: FrozenSet[int]
    c_in: Tuple[Tuple[int, float], ...] = ()


@dataclass
class Workload:
    """A complete, seeded description of one lattice run."""
    name: str
    mask: np.ndarray
    tau_f: float
    D: float
    w0: float = 1.0 / 3.0
    rho0: float = 1.0
    k_decay: float = 0.0
    c_shift: float = 0.0
    periodic: Tuple[bool, bool] = (False, False)
    segments: List[Segment] = field(default_factory=list)
    schedule: Optional[List[Phase]] = None
    t_origin: int = 0
    steps: int = 1000
    storage: str = "f64"
    init: Optional[Dict[str, np.ndarray]] = None
    region: Optional[np.ndarray] = None

    @property
    def nx(self) -> int:
        return int(self.mask.shape[1])

    @property
    def ny(self) -> int:
        return int(self.mask.shape[0])

    @property
    def n_fluid(self) -> int:
        return int(np.count_nonzero(self.mask == FLUID))


# ---------------------------------------------------------------------------
# Straight channel
# ---------------------------------------------------------------------------

def straight_channel(nx: int = 128, ny: int = 64, *, u_max: float = 0.05,
                     tau_f: float = 0.8, D: float = 0.01, c_in: float = 1.0,
                     w0: float = 1.0 / 3.0, steps: int = 1000,
                     storage: str = "f64", poiseuille_init: bool = True) -> Workload:
    """Channel between walls at rows 0 and ny-1, inlet ghost column 0 (id 2),
    outlet ghost column nx-1 (id 3); always open.

    With ``poiseuille_init`` the run starts from the fully developed state
    instead of rest: u = 4 u_max s (H - s) / H^2 across the H = ny - 2 fluid
    rows (s measured from the halfway wall) and a density falling linearly
    along the channel with the Poiseuille pressure gradient
    dp/dx = -8 rho nu u_max / H^2, p = rho / 3, nu = (tau_f - 1/2) / 3
    (the viscosity relation stated after Eq. 6), so that the profile can be
    checked after a short run.
    """
    mask = np.full((ny, nx), FLUID, np.uint8)
    mask[0, :] = WALL
    mask[-1, :] = WALL
    mask[1:-1, 0] = 2
    mask[1:-1, -1] = 3
    segs = [Segment(2, "inlet", (-1, 0), u_max=u_max, c_in=c_in),
            Segment(3, "outlet", (1, 0))]
    init = None
    if poiseuille_init:
        H = ny - 2
        s = np.arange(ny) - 0.5
        prof = np.where((s > 0) & (s < H), 4.0 * u_max * s * (H - s) / H ** 2, 0.0)
        nu = (tau_f - 0.5) / 3.0
        dpdx = -8.0 * nu * u_max / H ** 2
        x = np.arange(nx, dtype=np.float64)
        rho_x = 1.0 + 3.0 * dpdx * (x - (nx - 1))
        init = {
            "rho": np.broadcast_to(rho_x[None, :], (ny, nx)).copy(),
            "ux": np.broadcast_to(prof[:, None], (ny, nx)).copy(),
            "uy": np.zeros((ny, nx)),
            "C": np.zeros((ny, nx)),
        }
    return Workload(name=f"straight_channel_{nx}x{ny}", mask=mask, tau_f=tau_f,
                    D=D, w0=w0, segments=segs, schedule=None, steps=steps,
                    storage=storage, init=init)


# Step-profile advection test (paper Table 3): the first opening of the
# source channel. A straight channel 20 nodes wide, at rest with C = 0; its
# inlet holds C = 1 from t = 0 and the stationary channel flow (a Poiseuille
# profile peaking at U) carries the step into the channel. Cases (a)-(d):
# U and D in lattice units and the step count T / dt of Table 3; each front
# travels 200 nodes.
STEP_PROFILE_CASES: Dict[str, Tuple[float, float, int]] = {
    "a": (0.5, 0.00244, 400),
    "b": (0.05, 0.000244, 4000),
    "c": (0.1, 0.00244, 2000),
    "d": (0.01, 0.000244, 20000),
}


def step_profile(case: str, nx: int = 402, width: int = 20,
                 storage: str = "f64") -> Tuple[Workload, Tuple[np.ndarray, np.ndarray]]:
    """The channel of the step-profile test and its frozen velocity field.

    Walls at rows 0 and width + 1, inlet ghost column 0 (id 2, C_in = 1),
    outlet ghost column nx - 1 (id 3). D2Q4 compound lattice (w0 = 0): with
    U = 0.5 (case a) the equilibrium stays non-negative only there. The
    field is u_x = 4 U s (H - s) / H^2, s the distance from the halfway wall,
    H = width; u_y = 0. The fluid parameters (tau_f, the inlet's u_max) do
    not enter a compound-only run.
    """
    U, D, steps = STEP_PROFILE_CASES[case]
    ny = width + 2
    mask = np.full((ny, nx), FLUID, np.uint8)
    mask[0, :] = WALL
    mask[-1, :] = WALL
    mask[1:-1, 0] = 2
    mask[1:-1, -1] = 3
    segs = [Segment(2, "inlet", (-1, 0), u_max=0.0, c_in=1.0), Segment(3, "outlet", (1, 0))]
    s = np.arange(ny) - 0.5
    prof = np.where((s > 0) & (s < width), 4.0 * U * s * (width - s) / width ** 2, 0.0)
    ux = np.broadcast_to(prof[:, None], (ny, nx)).copy()
    uy = np.zeros((ny, nx))
    wl = Workload(name=f"step_profile_{case}", mask=mask, tau_f=0.8, D=D, w0=0.0,
                  segments=segs, schedule=None, steps=steps, storage=storage)
    return wl, (ux, uy)


# ---------------------------------------------------------------------------
# Gradient generator
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class GGLayout:
    """Rectangles of a gradient generator, as half-open [x0, x1) x [y0, y1)."""
    left_channel: Tuple[int, int, int, int]
    right_channel: Tuple[int, int, int, int]
    left_prechamber: Tuple[int, int, int, int]
    right_prechamber: Tuple[int, int, int, int]
    chamber: Tuple[int, int, int, int]
    inlet_row: int
    outlet_row: int


def gradient_generator_layout(nx: int, ny: int, *, channel_width: int,
                              channel_length: int, pre_length: int,
                              pre_height: int, chamber_width: int,
                              chamber_height: int) -> GGLayout:
    """Centre the structure in the lattice; channels run along +y."""
    total_w = 2 * channel_width + 2 * pre_length + chamber_width
    if total_w + 2 > nx or channel_length + 2 > ny:
        raise ValueError("gradient generator does not fit the lattice")
    if chamber_height < pre_height or channel_length < chamber_height:
        raise ValueError("inconsistent gradient generator proportions")
    x0 = (nx - total_w) // 2
    y0 = (ny - channel_length) // 2
    yc = y0 + channel_length // 2
    lc = (x0, x0 + channel_width, y0, y0 + channel_length)
    xp = lc[1]
    lp = (xp, xp + pre_length, yc - pre_height // 2, yc - pre_height // 2 + pre_height)
    xch = lp[1]
    ch = (xch, xch + chamber_width, yc - chamber_height // 2,
          yc - chamber_height // 2 + chamber_height)
    rp = (ch[1], ch[1] + pre_length, lp[2], lp[3])
    rc = (rp[1], rp[1] + channel_width, y0, y0 + channel_length)
    return GGLayout(lc, rc, lp, rp, ch, inlet_row=y0 - 1, outlet_row=y0 + channel_length)


def gradient_generator_mask(layout: GGLayout, nx: int, ny: int) -> np.ndarray:
    """Mask with segment ids 2 = left inlet, 3 = left outlet, 4 = right inlet,
    5 = right outlet; everything outside the rectangles is wall."""
    mask = np.full((ny, nx), WALL, np.uint8)
    for (a, b, c, d) in (layout.left_channel, layout.right_channel,
                         layout.left_prechamber, layout.right_prechamber,
                         layout.chamber):
        mask[c:d, a:b] = FLUID
    for ch, sin, sout in ((layout.left_channel, 2, 3), (layout.right_channel, 4, 5)):
        mask[layout.inlet_row, ch[0]:ch[1]] = sin
        mask[layout.outlet_row, ch[0]:ch[1]] = sout
    return mask


def alternating_schedule(half_period: int, c_source: float = 1.0,
                         c_sink: float = 0.0) -> List[Phase]:
    """Left channel (source) open for ``half_period`` steps, then the right
    channel (sink); no all-closed phase. Valve alternation after the
    Experimental Layout section, compressed to back-to-back flushes."""
    return [Phase(half_period, frozenset({2, 3}), ((2, c_source),)),
            Phase(half_period, frozenset({4, 5}), ((4, c_sink),))]


def paper_schedule(open_steps: int = 2000, closed_steps: int = 118000,
                   c_source: float = 1.0, c_sink: float = 0.0) -> List[Phase]:
    """The paper's flushing pattern: left open, all closed, right open, all
    closed (1 s open per channel every 2 min, offset by 1 min; at the CDE
    time step of Table 2, 1 s = 2000 steps)."""
    return [Phase(open_steps, frozenset({2, 3}), ((2, c_source),)),
            Phase(closed_steps, frozenset()),
            Phase(open_steps, frozenset({4, 5}), ((4, c_sink),)),
            Phase(closed_steps, frozenset())]


def gradient_generator(scale: float = 1.0, *, nx: Optional[int] = None,
                       ny: Optional[int] = None, u_max: float = 0.04,
                       peclet: float = 500.0, tau_f: float = 0.8,
                       w0: float = 1.0 / 3.0, half_period: int = 2000,
                       chamber_width: Optional[int] = None,
                       storage: str = "f32", steps: int = 50000,
                       c_shift: float = 0.5) -> Workload:
    """Gradient generator at ``scale`` x (2048 x 1024); scale 4 is 8192 x 4096.

    D is chosen so that the channel Peclet number u_max * W / D equals
    ``peclet`` (Eq. 12 with the channel width as length scale and the maximal
    speed, as in the Experimental Layout section).
    """
    nx = int(round(2048 * scale)) if nx is None else int(nx)
    ny = int(round(1024 * scale)) if ny is None else int(ny)
    s = nx / 2048.0
    cw = max(4, int(round(100 * s)))
    lay = gradient_generator_layout(
        nx, ny, channel_width=cw, channel_length=int(round(1000 * s)),
        pre_length=int(round(200 * s)), pre_height=max(2, int(round(100 * s))),
        chamber_width=int(round((600 if chamber_width is None else chamber_width) * s)),
        chamber_height=int(round(400 * s)))
    mask = gradient_generator_mask(lay, nx, ny)
    D = u_max * cw / peclet
    segs = [Segment(2, "inlet", (0, -1), u_max=u_max, c_in=1.0),
            Segment(3, "outlet", (0, 1)),
            Segment(4, "inlet", (0, -1), u_max=u_max, c_in=0.0),
            Segment(5, "outlet", (0, 1))]
    region = np.zeros((ny, nx), np.uint8)
    a, b, c, d = lay.chamber
    region[c:d, a:b] = 1
    wl = Workload(name=f"gradient_generator_{nx}x{ny}", mask=mask, tau_f=tau_f,
                  D=D, w0=w0, c_shift=c_shift, segments=segs,
                  schedule=alternating_schedule(half_period), steps=steps,
                  storage=storage, region=region)
    wl.layout = lay  # type: ignore[attr-defined]
    wl.peclet = peclet  # type: ignore[attr-defined]
    return wl


def batch_instances(n: int = 64, seed: int = 4703, *, u_max: float = 0.04,
                    steps: int = 10000) -> List[Workload]:
    """Seeded set of uneven gradient generators.

    Lattice widths uniform over {512, 768, ..., 2048} with ny = nx / 2;
    chamber width uniform in [200, 600] cells at full scale (scaled with the
    lattice); valve half-period uniform over {500, ..., 4000} steps; channel
    Peclet number log-uniform in [100, 2000].
    """
    rng = np.random.default_rng(seed)
    out = []
    widths = np.arange(512, 2049, 256)
    for k in range(n):
        nx = int(rng.choice(widths))
        cw = float(rng.uniform(200.0, 600.0))
        hp = int(rng.integers(500, 4001))
        pe = float(np.exp(rng.uniform(np.log(100.0), np.log(2000.0))))
        wl = gradient_generator(nx=nx, ny=nx // 2, u_max=u_max, peclet=pe,
                                half_period=hp, chamber_width=int(round(cw)),
                                storage="f32", steps=steps)
        wl.name = f"batch{k:02d}_{nx}x{nx // 2}"
        out.append(wl)
    return out


# ---------------------------------------------------------------------------
# Roofline lattice and small periodic boxes
# ---------------------------------------------------------------------------

def all_fluid_channel(nx: int = 8192, ny: int = 4096, *, u0: float = 0.04,
                      tau_f: float = 0.8, D: float = 0.008,
                      storage: str = "f32") -> Workload:
    """All-fluid lattice, periodic along x, lattice edges in y act as walls;
    uniform initial speed u0 along x and a compound stripe in the middle
    third. Every node is fluid, so every node update is a full update."""
    mask = np.zeros((ny, nx), np.uint8)
    C = np.zeros((ny, nx))
    C[ny // 3: 2 * ny // 3, :] = 1.0
    init = {"rho": np.ones((ny, nx)), "ux": np.full((ny, nx), u0),
            "uy": np.zeros((ny, nx)), "C": C}
    return Workload(name=f"all_fluid_{nx}x{ny}", mask=mask, tau_f=tau_f, D=D,
                    periodic=(True, False), storage=storage, init=init,
                    c_shift=0.5)


def random_mask(nx: int, ny: int, seed: int, *, wall_frac: float = 0.15,
                periodic: Tuple[bool, bool] = (False, False)) -> np.ndarray:
    """Seeded random obstacle field with a wall frame on non-periodic edges.
    Fluid cells whose eight neighbours are all non-fluid are turned into
    wall, since such a cell is disconnected from the flow."""
    rng = np.random.default_rng(seed)
    mask = np.where(rng.random((ny, nx)) < wall_frac, WALL, FLUID).astype(np.uint8)
    if not periodic[1]:
        mask[0, :] = WALL
        mask[-1, :] = WALL
    if not periodic[0]:
        mask[:, 0] = WALL
        mask[:, -1] = WALL
    fl = mask == FLUID
    pad = np.pad(fl, 1, mode="wrap")
    if not periodic[1]:
        pad[0, :] = False
        pad[-1, :] = False
    if not periodic[0]:
        pad[:, 0] = False
        pad[:, -1] = False
    nb = np.zeros(fl.shape, dtype=np.int32)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            nb += pad[1 + dy: 1 + dy + ny, 1 + dx: 1 + dx + nx]
    mask[fl & (nb == 0)] = WALL
    return mask


# ---------------------------------------------------------------------------
# Chamber misfit (inverse problem on the gradient generator)
# ---------------------------------------------------------------------------

def chamber_misfit_setup(wl: Workload):
    """Loss window, linear target ramp and source patch for a gradient
    generator: the window is the two pre-chambers and the chamber; the target
    falls linearly from 1 at the source-channel wall to 0 at the sink-channel
    wall; the source patch is a 64 x 64 box (scaled with the lattice) at the
    mouth of the left pre-chamber. Returns (weight, target, r_box)."""
    lay = wl.layout  # type: ignore[attr-defined]
    weight = np.zeros(wl.mask.shape)
    for (a, b, c, d) in (lay.left_prechamber, lay.chamber, lay.right_prechamber):
        weight[c:d, a:b] = 1.0
    weight[wl.mask != FLUID] = 0.0
    x = np.arange(wl.nx, dtype=np.float64)
    x_src = lay.left_channel[1]
    x_snk = lay.right_channel[0]
    ramp = np.clip(1.0 - (x - x_src) / float(x_snk - x_src), 0.0, 1.0)
    target = np.broadcast_to(ramp[None, :], wl.mask.shape).copy()
    s = wl.nx / 2048.0
    side = max(2, int(round(64 * s)))
    a, b, c, d = lay.left_prechamber
    yc = (c + d) // 2
    r_box = (a, max(c, yc - side // 2), min(side, b - a), min(side, d - c))
    return weight, target, r_box
