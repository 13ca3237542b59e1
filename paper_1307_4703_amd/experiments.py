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
    lat = Lattice.from_workload(wl, storage=storage)
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
