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


# Snapshots (gg_save): magic[8], six int32 (version, nx, ny, storage, pairs,
# pad), three int64 (pitch, plane, t), then the 14 population planes in the
# lattice's layout (include/gg.h, gg_set_layout), then the fluxes.
SNAP_DATA = 56


def snapshot_header(snap: bytes) -> Dict[str, int]:
    version, nx, ny, storage, pairs, _ = (int(v) for v in np.frombuffer(snap, np.int32, 6, 8))
    pitch, plane, t = (int(v) for v in np.frombuffer(snap, np.int64, 3, 32))
    assert version == 2
    return {"nx": nx, "ny": ny, "storage": storage, "pairs": pairs, "pitch": pitch,
            "plane": plane, "t": t, "node0": pitch + 64}


def snapshot_slot(h: Dict[str, int], i: int, node: int) -> int:
    """Element index (from the start of the planes) of population i (f0..f8,
    then g0..g4) of node `node`."""
    plane = h["plane"]
    if not h["pairs"]:
        return i * plane + node
    if i < 5:
        return 2 * i * plane + 2 * node
    if i >= 9:
        return 2 * (i - 9) * plane + 2 * node + 1
    return (i + 5) * plane + node


def snapshot_planes(snap: bytes, dtype) -> np.ndarray:
    """The 14 planes as (14, plane) in population order, whatever the layout."""
    h = snapshot_header(snap)
    plane = h["plane"]
    raw = np.frombuffer(snap, dtype, 14 * plane, SNAP_DATA).reshape(14, plane)
    if not h["pairs"]:
        return raw
    pp = raw[:10].reshape(5, 2 * plane)
    return np.concatenate([pp[:, 0::2], raw[10:14], pp[:, 1::2]])
