"""Shared helpers of the GPU parity tests: run the HIP path and the FP64
oracle on the same seeded inputs and measure per-field errors."""
from __future__ import annotations

import sys
from typing import Dict, Optional

import numpy as np

from oracle import Oracle


def log(msg: str) -> None:
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def seeded_init(wl, seed: int, amp_u: float = 0.02) -> Dict[str, np.ndarray]:
    """Random initial fields (fluid at rest plus noise) unless the workload
    carries its own initial state."""
    if wl.init is not None:
        return wl.init
    rng = np.random.default_rng(seed)
    sh = wl.mask.shape
    return {"rho": 1.0 + 0.01 * rng.standard_normal(sh),
            "ux": amp_u * rng.standard_normal(sh),
            "uy": amp_u * rng.standard_normal(sh),
            "C": rng.random(sh)}


def make_oracle(wl) -> Oracle:
    return Oracle(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, rho0=wl.rho0,
                  k_decay=wl.k_decay, periodic=wl.periodic, segments=wl.segments,
                  schedule=wl.schedule, t_origin=wl.t_origin)


def make_lattice(wl, storage: str, init: Dict[str, np.ndarray],
                 tile=None, chunk: Optional[int] = None):
    from paper_1307_4703_amd import Lattice
    lat = Lattice.from_workload(wl, storage=storage, init=False)
    if tile is not None or chunk is not None:
        tx, ty = tile if tile is not None else (64, 4)
        lat.set_launch(tx, ty, 64 if chunk is None else chunk)
    lat.init(**init)
    return lat


def field_errors(lat, o: Oracle, fluid: np.ndarray) -> Dict[str, float]:
    """Relative errors per field: rho against rho0, u against max|u| of the
    oracle, C against max(1, max C); populations against max|f|, max|g|."""
    rho, ux, uy, C = lat.read()
    ro, uxo, uyo, Co = o.fields()
    f, g = lat.populations()
    fo = np.moveaxis(o.f, 2, 0)
    go = np.moveaxis(o.g, 2, 0)
    umax = max(np.abs(uxo[fluid]).max(), np.abs(uyo[fluid]).max(), 1e-300)
    out = {
        "rho": float(np.abs(rho[fluid] - ro[fluid]).max() / o.rho0),
        "u": float(max(np.abs(ux[fluid] - uxo[fluid]).max(), np.abs(uy[fluid] - uyo[fluid]).max()) / umax),
        "C": float(np.abs(C[fluid] - Co[fluid]).max() / max(1.0, np.abs(Co[fluid]).max())),
        "f": float(np.abs(f[:, fluid] - fo[:, fluid]).max() / np.abs(fo[:, fluid]).max()),
        "g": float(np.abs(g[:, fluid] - go[:, fluid]).max() / max(1e-300, np.abs(go[:, fluid]).max())),
    }
    out["rho_l2"] = float(np.sqrt(np.mean((rho[fluid] - ro[fluid]) ** 2)) / o.rho0)
    out["u_l2"] = float(np.sqrt(np.mean((ux[fluid] - uxo[fluid]) ** 2 + (uy[fluid] - uyo[fluid]) ** 2)) / umax)
    out["C_l2"] = float(np.sqrt(np.mean((C[fluid] - Co[fluid]) ** 2)) / max(1.0, np.abs(Co[fluid]).max()))
    return out
