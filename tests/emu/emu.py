"""ctypes face of step_emu.c, the storage-rounded replay of the kernels'
step arithmetic (test instrument only: the package never imports it).

``Emulator(wl, storage)`` takes the same seeded workload records as the
library and the oracle; ``step(h, k, t)`` advances deviation planes
(9 and 5 planes of ny*nx values in the compute type) by one step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "step_emu.c")
NSEG, NPH = 16, 64
_LIBS = {}


def build(verbose: bool = False):
    """Compile the float and double builds (gcc, no contraction)."""
    outs = []
    for tname, tag in (("float", "f32"), ("double", "f64")):
        out = os.path.join(HERE, f"libstepemu_{tag}.so")
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-Wall", "-Wextra", f"-DEMU_T={tname}", "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
        outs.append(out)
    return outs


class _Lat(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
                ("mask", ctypes.c_void_p),
                ("tau_f", ctypes.c_double), ("D", ctypes.c_double), ("w0", ctypes.c_double),
                ("rho0", ctypes.c_double), ("k_decay", ctypes.c_double),
                ("c_shift", ctypes.c_double),
                ("storage", ctypes.c_int32),
                ("seg_kind", ctypes.c_int32 * NSEG), ("seg_nx", ctypes.c_int32 * NSEG),
                ("seg_ny", ctypes.c_int32 * NSEG),
                ("seg_umax", ctypes.c_double * NSEG), ("seg_s0", ctypes.c_double * NSEG),
                ("seg_s1", ctypes.c_double * NSEG), ("seg_cin", ctypes.c_double * NSEG),
                ("n_phases", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("period", ctypes.c_int64), ("t_origin", ctypes.c_int64),
                ("phase_start", ctypes.c_int64 * NPH), ("phase_open", ctypes.c_uint32 * NPH),
                ("phase_cin", (ctypes.c_double * NSEG) * NPH),
                ("r_x0", ctypes.c_int32), ("r_y0", ctypes.c_int32),
                ("r_w", ctypes.c_int32), ("r_h", ctypes.c_int32),
                ("R", ctypes.c_void_p)]


def lib(tag: str) -> ctypes.CDLL:
    if tag not in _LIBS:
        path = os.path.join(HERE, f"libstepemu_{tag}.so")
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        L.emu_step.argtypes = [ctypes.POINTER(_Lat), ctypes.c_int64] + [ctypes.c_void_p] * 4
        L.emu_step.restype = None
        L.emu_to_half.argtypes = [ctypes.c_float]
        L.emu_to_half.restype = ctypes.c_uint16
        L.emu_fluid_ka.argtypes = [ctypes.c_double, ctypes.c_int]
        L.emu_fluid_ka.restype = ctypes.c_double
        L.emu_from_half.argtypes = [ctypes.c_uint16]
        L.emu_from_half.restype = ctypes.c_float
        _LIBS[tag] = L
    return _LIBS[tag]


def segment_span(mask: np.ndarray, sid: int, normal):
    """Tangential extent of segment sid's ghost line, extended by half a cell
    on each side (the halfway walls next to its outermost cells)."""
    ys, xs = np.nonzero(mask == sid)
    s = ys if normal[0] != 0 else xs
    return float(s.min()) - 0.5, float(s.max()) + 0.5


class Emulator:
    def __init__(self, wl, storage: str, c_shift: float = 0.0, R=None):
        self.tag = "f64" if storage == "f64" else "f32"
        self.dtype = np.float64 if storage == "f64" else np.float32
        self.L = lib(self.tag)
        self.mask = np.ascontiguousarray(wl.mask, np.uint8)
        ny, nx = self.mask.shape
        s = _Lat()
        s.nx, s.ny = nx, ny
        s.periodic_x, s.periodic_y = int(bool(wl.periodic[0])), int(bool(wl.periodic[1]))
        s.mask = self.mask.ctypes.data
        s.tau_f, s.D, s.w0, s.rho0 = wl.tau_f, wl.D, wl.w0, wl.rho0
        s.k_decay, s.c_shift = wl.k_decay, c_shift
        s.storage = 1 if storage == "f16" else 0
        kinds = {"inlet": 1, "outlet": 2}
        for seg in wl.segments:
            j = seg.id - 2
            s.seg_kind[j] = kinds[seg.kind]
            s.seg_nx[j], s.seg_ny[j] = seg.normal
            s.seg_umax[j] = seg.u_max
            s.seg_cin[j] = seg.c_in
            s.seg_s0[j], s.seg_s1[j] = segment_span(self.mask, seg.id, seg.normal)
        if wl.schedule:
            start = 0
            s.n_phases = len(wl.schedule)
            for k, ph in enumerate(wl.schedule):
                s.phase_start[k] = start
                start += int(ph.duration)
                m = 0
                for sid in ph.open:
                    m |= 1 << (int(sid) - 2)
                s.phase_open[k] = m
                over = dict(ph.c_in)
                for seg in wl.segments:
                    s.phase_cin[k][seg.id - 2] = float(over.get(seg.id, seg.c_in))
            s.period = start
            s.t_origin = wl.t_origin
        self._R = None
        if R is not None:
            # the bounding box of the nonzero source on the fluid
            nz = (R != 0) & (self.mask == 0)
            ys, xs = np.nonzero(nz)
            if len(xs):
                x0, x1, y0, y1 = xs.min(), xs.max() + 1, ys.min(), ys.max() + 1
                self._R = np.ascontiguousarray(R[y0:y1, x0:x1], np.float64)
                s.r_x0, s.r_y0, s.r_w, s.r_h = int(x0), int(y0), int(x1 - x0), int(y1 - y0)
                s.R = self._R.ctypes.data
        self.s = s

    def step(self, h: np.ndarray, k: np.ndarray, t: int, n: int = 1):
        """n steps from time t; h (9, ny, nx), k (5, ny, nx) in the compute
        type, values already rounded to the storage type."""
        h = np.ascontiguousarray(h, self.dtype).copy()
        k = np.ascontiguousarray(k, self.dtype).copy()
        for q in range(n):
            ho, ko = h.copy(), k.copy()
            self.L.emu_step(ctypes.byref(self.s), int(t + q), h.ctypes.data, k.ctypes.data,
                            ho.ctypes.data, ko.ctypes.data)
            h, k = ho, ko
        return h, k
