"""Drivers of the paper's experiments that run on the compound-only step.

step_profile: the step-profile advection test of Table 3 (the first opening
of the source channel): a 20-node channel at rest with C = 0, its inlet held
at C = 1, the stationary channel flow frozen in a field slot. The paper
reports that at Pe ~ 4100 (cases a, b) oscillations appear at the front and
do not decay, that at Pe ~ 800 (cases c, d) they are smoothed out, and that
a tenfold smaller time step (b against a, d against c) changes neither.
The overshoot max C - 1 and undershoot min C over the channel measure them.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional

import numpy as np

from . import workloads as W
from .lattice import Lattice


def step_profile(case: str, storage: str = "f64", n_records: int = 20,
                 nx: int = 402) -> Dict:
    """Run case a, b, c or d of Table 3 on the GPU. Returns the overshoot
    (max C - 1) and undershoot (min C) over the fluid after each of
    n_records equal stretches of the run, the final concentration field C
    (NaN off the fluid) and its centre row, and the run time of the
    compound-only steps."""
    wl, (ux, uy) = W.step_profile(case, nx=nx, storage=storage)
    U, D, steps = W.STEP_PROFILE_CASES[case]
    if steps % (2 * n_records):
        raise ValueError("the record stretches must be an even number of steps")
    lat = Lattice.from_workload(wl, storage=storage, layout="planes")
    lat.set_velocity_field(0, ux, uy)
    fluid = wl.mask == 0
    over: List[float] = []
    under: List[float] = []
    t_run = 0.0
    try:
        for _ in range(n_records):
            t0 = time.perf_counter()
            lat.cde_step(steps // n_records)
            lat.sync()
            t_run += time.perf_counter() - t0
            C = lat.read()[3]
            over.append(float(C[fluid].max() - 1.0))
            under.append(float(C[fluid].min()))
        C = lat.read()[3]
    finally:
        lat.close()
    nf = int(np.count_nonzero(fluid))
    return {"case": case, "U": U, "D": D, "steps": steps, "peclet": U * (wl.ny - 2) / D,
            "storage": storage, "overshoot": over, "undershoot": under,
            "centre_row": C[wl.ny // 2, 1:-1].tolist(), "C": C, "seconds": t_run,
            "mlups": nf * steps / t_run / 1e6 if t_run > 0 else None}


def step_profile_summary(runs: Optional[Dict[str, Dict]] = None, storage: str = "f64") -> Dict:
    """All four cases with the figures the paper's comparison rests on."""
    runs = runs or {c: step_profile(c, storage) for c in W.STEP_PROFILE_CASES}
    out = {}
    for c, r in runs.items():
        out[c] = {"peclet": round(r["peclet"], 1), "steps": r["steps"],
                  "max_overshoot": round(max(r["overshoot"]), 5),
                  "final_overshoot": round(r["overshoot"][-1], 5),
                  "min_undershoot": round(min(r["undershoot"]), 5),
                  "final_undershoot": round(r["undershoot"][-1], 6),
                  "seconds": round(r["seconds"], 4),
                  "mlups": None if r["mlups"] is None else round(r["mlups"], 1)}
    return out


# ---------------------------------------------------------------------------
# Long-time gradient formation and inversion (Results; Tables 1-2)
# ---------------------------------------------------------------------------

# Table 2: compound time step 5e-4 s, so 4 h = 28 800 000 steps; D and the
# decay rate in lattice units; peak velocity U = 0.5 after rescaling.
GF_STEPS_PER_HOUR = 7_200_000
GF_D = 0.00244
GF_K = 3.34255e-7
GF_U = 0.5


def gradient_generator_paper_scale(storage: str = "f32", k_decay: float = 0.0) -> W.Workload:
    """The synthetic gradient generator at the paper's resolution (channels
    20 nodes = 100 um wide, dx = 5 um: 0.2 x the 2048 x 1024 layout), with
    the compound lattice of Table 2 (D2Q4, D = 0.00244, decay k) and the
    paper's valve pattern."""
    wl = W.gradient_generator(scale=0.2, w0=0.0, storage=storage)
    wl.D = GF_D
    wl.k_decay = k_decay
    wl.schedule = W.paper_schedule()
    return wl


def flow_fields(wl, storage: str = "f64", flow_steps: int = 40000) -> Dict[str, tuple]:
    """Velocity of each valve state after flow_steps coupled steps from rest
    with only that channel's valves open (the paper precomputes these three
    fields; with every valve closed the fluid is at rest)."""
    out = {}
    for name, open_ids in (("left", frozenset({2, 3})), ("right", frozenset({4, 5}))):
        lat = Lattice.from_workload(wl, storage=storage)
        try:
            lat.set_schedule([W.Phase(flow_steps + 1, open_ids)])
            lat.step(flow_steps)
            _, ux, uy, _ = lat.read()
        finally:
            lat.close()
        out[name] = (np.nan_to_num(ux), np.nan_to_num(uy))
    z = np.zeros(wl.mask.shape)
    out["closed"] = (z, z.copy())
    return out


def monitor_points(wl) -> Dict[str, tuple]:
    """(y, x) of three points at the chamber's mid-height: near its left
    edge, at its centre and near its right edge (stand-ins for the paper's
    monitoring points, whose positions its figure gives)."""
    a, b, c, d = wl.layout.chamber
    yc = (c + d) // 2
    return {"left": (yc, a + 2), "centre": (yc, (a + b) // 2), "right": (yc, b - 3)}


def gradient_formation(hours: float = 4.0, storage: str = "f32", samples_per_hour: int = 30,
                       flow_steps: int = 40000, swap_hours: Optional[float] = None,
                       progress=None) -> Dict:
    """The paper's last experiment on the compound-only step: 4 h of valve
    flushing (left channel source, right sink), the media swapped at 2 h,
    once with and once without decay; the two runs advance side by side on
    two HIP streams. Returns the time series of C at the monitoring points,
    the mid-height profile across pre-chambers and chamber at the swap and
    at the end, and the run's update rate. progress(msg), if given, hears
    of every simulated quarter hour."""
    import torch
    swap_hours = hours / 2 if swap_hours is None else swap_hours
    steps_total = int(round(hours * GF_STEPS_PER_HOUR))
    chunk = GF_STEPS_PER_HOUR // samples_per_hour
    swap = int(round(swap_hours * GF_STEPS_PER_HOUR))
    period = sum(p.duration for p in W.paper_schedule())
    if chunk % 4 or swap % chunk or swap % period:
        raise ValueError("samples and the swap must fall on whole passes and periods")
    base = gradient_generator_paper_scale(storage)
    fields = flow_fields(base, "f64", flow_steps)
    umax = max(float(np.hypot(*fields[k]).max()) for k in ("left", "right"))
    scale = GF_U / umax
    pts = monitor_points(base)
    a, b, c, d = base.layout.chamber
    yc = (c + d) // 2
    xs = slice(base.layout.left_prechamber[0], base.layout.right_prechamber[1])
    runs = {}
    streams = {}
    for label, k in (("decay", GF_K), ("no_decay", 0.0)):
        wl = gradient_generator_paper_scale(storage, k)
        streams[label] = torch.cuda.Stream()
        lat = Lattice.from_workload(wl, storage=storage, stream=int(streams[label].cuda_stream),
                                    layout="planes")
        for slot, name in enumerate(("left", "right", "closed")):
            lat.set_velocity_field(slot, *fields[name], scale=scale)
        lat.set_phase_fields([0, 2, 1, 2])  # left open, closed, right open, closed
        runs[label] = {"lat": lat, "t": [], **{p: [] for p in pts}}
    t0 = time.perf_counter()
    t_steps = 0.0
    profiles = {}
    try:
        for t in range(0, steps_total, chunk):
            if t == swap:
                for label, r in runs.items():
                    r["lat"].set_schedule(W.paper_schedule(c_source=0.0, c_sink=1.0))
            s0 = time.perf_counter()
            for r in runs.values():
                r["lat"].cde_step(chunk)
            for r in runs.values():
                r["lat"].sync()
            t_steps += time.perf_counter() - s0
            for label, r in runs.items():
                C = r["lat"].read()[3]
                r["t"].append((t + chunk) / GF_STEPS_PER_HOUR)
                for p, (y, x) in pts.items():
                    r[p].append(float(C[y, x]))
                if progress and (t + chunk) % (GF_STEPS_PER_HOUR // 4) == 0 and label == "decay":
                    progress(f"{(t + chunk) / GF_STEPS_PER_HOUR:.2f} h: centre C "
                             f"{r['centre'][-1]:.4f} (decay), {time.perf_counter() - t0:.0f} s")
                if t + chunk in (swap, steps_total):
                    profiles.setdefault(label, {})[f"{(t + chunk) / GF_STEPS_PER_HOUR:g}h"] = \
                        np.nan_to_num(C[yc, xs]).tolist()
        diag = {label: r["lat"].diagnostics(check_finite=False) for label, r in runs.items()}
    finally:
        for r in runs.values():
            r["lat"].close()
    nf = int(np.count_nonzero(base.mask == 0))
    a_, b_, c_, d_ = base.layout.chamber
    u_ch = max(float(np.hypot(*fields[k])[c_:d_, a_:b_].max()) for k in ("left", "right"))
    out = {"hours": hours, "swap_hours": swap_hours, "steps": steps_total, "storage": storage,
           "scale": scale, "u_max_flow": umax, "chamber_max_u_scaled": u_ch * scale,
           "n_fluid": nf, "seconds": time.perf_counter() - t0,
           "seconds_stepping": t_steps,
           "mlups_two_lattices": 2 * nf * steps_total / t_steps / 1e6,
           "monitor_points": {p: list(v) for p, v in pts.items()},
           "profile_x0": xs.start, "profiles": profiles}
    for label, r in runs.items():
        out[label] = {"t_hours": r["t"], **{p: r[p] for p in pts},
                      "n_nonfinite": diag[label]["n_nonfinite"],
                      "solute": diag[label]["solute"]}
    return out


def time_to_settle(t: List[float], c: List[float], t_from: float, t_to: float,
                   frac: float = 0.9) -> Optional[float]:
    """Hours after t_from until c first covers frac of its change between
    t_from and t_to (the value at the last sample before t_to)."""
    ts = np.asarray(t)
    cs = np.asarray(c)
    i0 = int(np.searchsorted(ts, t_from, side="right")) - 1
    i1 = int(np.searchsorted(ts, t_to, side="right")) - 1
    c0 = cs[i0] if i0 >= 0 else 0.0
    c1 = cs[i1]
    if c1 == c0:
        return None
    goal = c0 + frac * (c1 - c0)
    for i in range(max(i0, 0), i1 + 1):
        if (c1 - c0) * (cs[i] - goal) >= 0:
            return float(ts[i] - t_from)
    return None


def curvature(profile: List[float]) -> float:
    """Deviation of a profile's middle from the straight line through its
    ends, relative to the end-to-end difference: 0 for a linear profile,
    negative where the middle sags below the line."""
    p = np.asarray(profile)
    mid = p[len(p) // 2]
    return float((mid - 0.5 * (p[0] + p[-1])) / abs(p[0] - p[-1]))


def gradient_formation_summary(r: Dict) -> Dict:
    out = {}
    for label in ("decay", "no_decay"):
        s = r[label]
        t = s["t_hours"]
        prof = r["profiles"][label]
        out[label] = {
            "centre_C_at_swap": s["centre"][int(np.argmin(np.abs(np.asarray(t) - r["swap_hours"])))],
            "centre_C_end": s["centre"][-1],
            "max_C_chamber_points": max(max(s[p]) for p in r["monitor_points"]),
            "hours_to_90pct_formation_left_point":
                time_to_settle(t, s["left"], 0.0, r["swap_hours"]),
            "hours_to_90pct_after_swap_left_point":
                time_to_settle(t, s["left"], r["swap_hours"], r["hours"]),
            "profile_curvature": {k: round(curvature(v), 4) for k, v in prof.items()},
            "n_nonfinite": s["n_nonfinite"]}
    out["chamber_max_u_scaled"] = r["chamber_max_u_scaled"]
    out["mlups_two_lattices"] = round(r["mlups_two_lattices"], 1)
    out["seconds_stepping"] = round(r["seconds_stepping"], 2)
    return out


# ---------------------------------------------------------------------------
# The paper's pressure boundary against the bounce-back family
# ---------------------------------------------------------------------------

def _poiseuille_error(rho, ux, H, nu, xm):
    """Deviation of the profile at column xm from the parabola of the local
    pressure gradient (p = rho / 3), relative to its peak."""
    G = -(rho[1:-1, xm + 20] - rho[1:-1, xm - 20]).mean() / 40 / 3
    umax = G * H * H / (8 * nu * rho[1:-1, xm].mean())
    s = np.arange(1, H + 1) - 0.5
    prof = 4 * umax * s * (H - s) / H ** 2
    return float(np.abs(ux[1:-1, xm] - prof).max() / umax), float(umax)


def boundary_comparison(storage: str = "f64", steps: int = 30000,
                        rate_steps: int = 2000) -> Dict:
    """The straight channel (128 x 64, H = 62) driven two ways to steady
    state: by the velocity inlet and outflow links of the bounce-back family
    (u_max = 0.05) and by the paper's pressure boundaries holding the
    densities that drive the same flow; for each, the profile's deviation
    from the parabola of its own pressure gradient and the spread of the
    mass flux along the channel, and where the fitted parabola vanishes
    (the no-slip points, relative to the halfway wall at 0.5 from the wall
    row); then the pressure-driven channel once more with the paper's walls
    in place of bounce-back. Then the rate of the 2048 x 1024 gradient
    generator (FP32) with each kind on its four segments, and with the
    pressure boundaries and the paper's walls; and that lattice driven each
    way for 20000 steps (boundary_gradient_generator)."""
    out: Dict = {}
    nu = (0.8 - 0.5) / 3
    base = W.straight_channel(storage=storage, steps=steps)
    H = base.ny - 2
    # the density drop that drives u_max = 0.05 over the channel's length
    drho = 3 * 0.05 * 8 * nu / (H * H) * (base.nx - 3)
    pres = W.Workload(base.name + "_pressure", base.mask, tau_f=0.8, D=base.D, w0=base.w0,
                      segments=[W.Segment(2, "pressure", (-1, 0), rho=1 + drho / 2, c_in=1.0,
                                          fix_c=True),
                                W.Segment(3, "pressure", (1, 0), rho=1 - drho / 2)],
                      storage=storage)
    for label, wl in (("velocity_inlet", base), ("pressure", pres), ("pressure_paper_walls", pres)):
        lat = Lattice.from_workload(wl, storage=storage)
        try:
            if label.endswith("paper_walls"):
                lat.set_wall_scheme("equilibrium")
            lat.step(steps)
            rho, ux, _, C = lat.read()
        finally:
            lat.close()
        err, umax = _poiseuille_error(rho, ux, H, nu, base.nx // 2)
        flux = [(rho[1:-1, x] * ux[1:-1, x]).sum() for x in range(1, base.nx - 1)]
        y = np.arange(1, H + 1, dtype=float)
        roots = np.sort(np.roots(np.polyfit(y, ux[1:-1, base.nx // 2], 2)).real)
        out[label] = {"profile_error_vs_local_gradient": round(err, 6),
                      "no_slip_points": [round(float(roots[0]), 4), round(float(roots[1]), 4)],
                      "u_max_local_gradient": round(umax, 6),
                      "u_centre": round(float(ux[1 + H // 2, base.nx // 2]), 6),
                      "mass_flux_spread": float(np.ptp(flux) / np.mean(flux)),
                      "C_outlet_column_mean": round(float(np.nanmean(C[1:-1, -2])), 4)}
    for label, r in boundary_rates(rate_steps).items():
        out[label].update(r)
    out["gradient_generator_2048"] = boundary_gradient_generator()
    return out


def boundary_gradient_generator(steps: int = 18000, storage: str = "f32") -> Dict:
    """The 2048 x 1024 gradient generator from rest with its valves
    alternating every 2000 steps (source channel open first), driven three
    ways: velocity inlets and outlets (u_max = 0.04) with bounce-back walls;
    pressure boundaries whose density drop would drive the same centre
    speed through a developed straight channel of the channels' width and
    length, with bounce-back walls; the same with the paper's walls. After
    `steps` steps (18000: the source channel has just been open for 2000
    steps): the largest speed in the chamber (the design asks it to be
    negligible), the centre speed of the source channel at mid-length, the
    compound there and where its front has reached along the channel's
    centre line (C = 1/2), and the total mass against its start plus the
    boundary fluxes (what the boundaries themselves create)."""
    wl = W.gradient_generator(storage=storage)
    lay = wl.layout  # type: ignore[attr-defined]
    la, lb, lc_, ld = lay.left_channel
    H = lb - la
    nu = (wl.tau_f - 0.5) / 3
    drho = 3 * 0.04 * 8 * nu / (H * H) * (ld - lc_)
    press = [W.Segment(2, "pressure", (0, -1), rho=1 + drho / 2, c_in=1.0, fix_c=True),
             W.Segment(3, "pressure", (0, 1), rho=1 - drho / 2),
             W.Segment(4, "pressure", (0, -1), rho=1 + drho / 2, c_in=0.0, fix_c=True),
             W.Segment(5, "pressure", (0, 1), rho=1 - drho / 2)]
    xc, ymid = (la + lb) // 2, (lc_ + ld) // 2
    out: Dict = {"steps": steps, "pressure_drop": round(drho, 6),
                 "viscous_time_H2_over_nu": round(H * H / nu)}
    for label in ("velocity_inlet", "pressure", "pressure_paper_walls"):
        if label != "velocity_inlet":
            wl.segments = press
        lat = Lattice.from_workload(wl)
        try:
            if label.endswith("paper_walls"):
                lat.set_wall_scheme("equilibrium")
            d0 = lat.diagnostics()
            lat.step(steps)
            d1 = lat.diagnostics()
            rho, ux, uy, C = lat.read()
        finally:
            lat.close()
        line = np.nan_to_num(C[lc_:ld, xc])
        reached = np.nonzero(line >= 0.5)[0]
        net_in = sum(d1["seg_mass"]) - sum(d0["seg_mass"])
        out[label] = {
            "max_u_chamber": float(d1["max_u_region"]),
            "u_centre_source_channel": float(np.hypot(ux[ymid, xc], uy[ymid, xc])),
            "C_source_channel_mid": round(float(C[ymid, xc]), 4),
            "front_C_half_cells_from_inlet": int(reached.max() + 1) if reached.size else 0,
            "mass_change_minus_net_inflow": float(d1["mass"] - d0["mass"] - net_in)}
    return out


def boundary_rates(rate_steps: int = 2000) -> Dict:
    """Rate of the 2048 x 1024 gradient generator (FP32) with velocity
    inlets and outlets, with pressure boundaries on its four segments, and
    with the pressure boundaries and the paper's walls; each with the fastest
    of the row-parallel pass forms (two-step passes with the boundary tiles
    in a kernel of their own beside the others, or every tile in one
    kernel; 6-row tiles; four-step passes where the lattice takes them). For
    the first two, also the compound alone on the flow's frozen velocity."""
    import torch
    out: Dict = {}
    gg = W.gradient_generator(storage="f32")
    stream = torch.cuda.current_stream()
    for label in ("velocity_inlet", "pressure", "pressure_paper_walls"):
        if label != "velocity_inlet":
            gg.segments = [W.Segment(2, "pressure", (0, -1), rho=1.002, c_in=1.0, fix_c=True),
                           W.Segment(3, "pressure", (0, 1), rho=0.998),
                           W.Segment(4, "pressure", (0, -1), rho=1.002, c_in=0.0, fix_c=True),
                           W.Segment(5, "pressure", (0, 1), rho=0.998)]
        best = None
        # (the paper's walls step in single steps whatever the form)
        for fuse in ((1,) if label.endswith("paper_walls") else (3, 4, 5)):
            lat = Lattice.from_workload(gg)
            try:
                if fuse > 1:
                    lat.set_two_step(fuse, 6)
                if label.endswith("paper_walls"):
                    lat.set_wall_scheme("equilibrium")
                lat.step(256)
                lat.sync()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                lat.step(rate_steps)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / rate_steps
                nf = lat.info()["n_fluid"]
            finally:
                lat.close()
            if best is None or ms < best[0]:
                best = (ms, fuse)
        ms, fuse = best
        out[label] = {"gg2048_f32_mlups": round(nf / (ms * 1e-3) / 1e6, 1),
                      "gg2048_f32_us_per_step": round(ms * 1e3, 3),
                      "pass_form": {"fuse": fuse, "rows": 6 if fuse > 1 else 0}}
        if label == "pressure_paper_walls":
            continue
        # the compound alone on the flow's frozen velocity (two-step passes
        # of 14-row tiles)
        lat = Lattice.from_workload(gg)
        try:
            lat.step(256)
            lat.set_velocity_field(0)
            lat.set_layout("planes")  # (the compound alone reads g only)
            lat.set_cde_launch(14)
            lat.cde_step(256)
            lat.sync()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lat.cde_step(rate_steps)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / rate_steps
        finally:
            lat.close()
        out[label]["gg2048_f32_compound_only_mlups"] = round(nf / (ms * 1e-3) / 1e6, 1)
        out[label]["gg2048_f32_compound_only_us_per_step"] = round(ms * 1e3, 3)
    return out


# ---------------------------------------------------------------------------
# Reduced-precision storage against FP64 at full size
# ---------------------------------------------------------------------------

def block_means(a: np.ndarray, fluid: np.ndarray, b: int = 8) -> np.ndarray:
    """Means over b x b blocks of the fluid nodes (NaN for blocks without
    fluid): the 1024 x 512 view of an 8192 x 4096 field."""
    ny, nx = a.shape
    v = np.where(fluid, a, 0.0).reshape(ny // b, b, nx // b, b).sum(axis=(1, 3))
    n = fluid.reshape(ny // b, b, nx // b, b).sum(axis=(1, 3))
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(n > 0, v / np.maximum(n, 1), np.nan)


def precision_report(wl, storages=("f16",), steps: int = 20000, block: int = 8) -> Dict:
    """Run the workload from the same initial state in FP64 and in each
    reduced storage type for `steps` steps (each in its fastest launch form)
    and report, per field (rho, u = (ux, uy), C), the max and L2 error of the
    reduced run against the FP64 run, relative to rho0, max |u| and
    max(1, max C) of the FP64 run: on the block means of `block` x `block`
    fluid nodes and on the full-resolution fields."""
    fluid = wl.mask == 0
    runs = {}
    for st in ("f64",) + tuple(storages):
        lat = Lattice.from_workload(wl, storage=st)
        try:
            lat.set_two_step(3, 14 if st == "f64" else 6)
            t0 = time.perf_counter()
            lat.step(steps)
            lat.sync()
            secs = time.perf_counter() - t0
            runs[st] = (lat.read(), secs)
        finally:
            lat.close()
    (rho0, ux0, uy0, C0), _ = runs["f64"]
    umax = float(max(np.abs(ux0[fluid]).max(), np.abs(uy0[fluid]).max()))
    cmax = float(max(1.0, np.abs(C0[fluid]).max()))
    ref_b = {k: block_means(v, fluid, block) for k, v in
             (("rho", rho0), ("ux", ux0), ("uy", uy0), ("C", C0))}
    out = {"workload": wl.name, "steps": steps, "block": block,
           "fp64_seconds": round(runs["f64"][1], 3), "max_u_fp64": umax, "max_C_fp64": cmax}
    for st in storages:
        (rho, ux, uy, C), secs = runs[st]
        b = {k: block_means(v, fluid, block) for k, v in
             (("rho", rho), ("ux", ux), ("uy", uy), ("C", C))}
        rep = {"seconds": round(secs, 3)}
        for field, scale in (("rho", wl.rho0), ("u", umax), ("C", cmax)):
            if field == "u":
                d_full = np.hypot(ux - ux0, uy - uy0)[fluid]
                db = np.hypot(b["ux"] - ref_b["ux"], b["uy"] - ref_b["uy"])
            else:
                d_full = np.abs((rho - rho0) if field == "rho" else (C - C0))[fluid]
                db = np.abs(b[field] - ref_b[field])
            db = db[np.isfinite(db)]
            rep[field] = {"max_block": float(db.max() / scale),
                          "l2_block": float(np.sqrt(np.mean(db ** 2)) / scale),
                          "max_full": float(d_full.max() / scale),
                          "l2_full": float(np.sqrt(np.mean(d_full ** 2)) / scale)}
        out[st] = rep
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="run the paper's experiments on the GPU")
    ap.add_argument("experiment", choices=["step-profile", "gradient-formation", "boundaries",
                                           "boundary-rates", "precision"])
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--hours", type=float, default=4.0)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--out", default=None, help="write the full result as JSON")
    args = ap.parse_args()
    if args.experiment == "step-profile":
        res = step_profile_summary(storage=args.storage)
        summ = res
    elif args.experiment == "boundaries":
        res = boundary_comparison()
        summ = res
    elif args.experiment == "boundary-rates":
        res = boundary_rates(args.steps)
        summ = res
    elif args.experiment == "precision":
        res = {f"pe{int(pe)}": precision_report(W.gradient_generator(scale=4.0, storage="f16",
                                                                       peclet=pe),
                                                ("f16", "f32"), steps=args.steps)
               for pe in (500.0, 2000.0)}
        summ = res
    else:
        res = gradient_formation(hours=args.hours, storage=args.storage,
                                 progress=lambda m: print(m, flush=True))
        summ = gradient_formation_summary(res)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh)
    print(json.dumps(summ), flush=True)
