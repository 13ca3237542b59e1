"""Python driver of the FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module. It does not import the library under
test, and the library never imports it. It takes plain arrays and duck-typed
segment / phase records (attributes ``id, kind, normal, u_max, c_in``, for
pressure segments also ``rho, fix_c``, and ``duration, open, c_in``), so the
same seeded inputs can be handed to both.

The time loop, the valve schedule lookup and the boundary-segment geometry
(halfway-wall positions of each inlet profile) are computed here, on the oracle
side, independently of the HIP library.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

SEG_KIND = {"inlet": 1, "outlet": 2, "pressure": 3}


class _OrcLattice(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
        ("mask", ctypes.c_void_p),
        ("tau_f", ctypes.c_double), ("tau_g", ctypes.c_double),
        ("w0", ctypes.c_double), ("rho_w", ctypes.c_double),
        ("k_decay", ctypes.c_double),
        ("R", ctypes.c_void_p),
        ("seg_kind", ctypes.c_void_p), ("seg_nrm", ctypes.c_void_p),
        ("seg_umax", ctypes.c_void_p), ("seg_s0", ctypes.c_void_p),
        ("seg_s1", ctypes.c_void_p),
        ("seg_rho", ctypes.c_void_p), ("seg_fixc", ctypes.c_void_p),
        ("wall_scheme", ctypes.c_int32),
    ]


def use_library(path: Optional[str]) -> None:
    """Point the oracle at another build of lbm_oracle.c (``None``: the
    default oracle/liboracle.so). Used by the test that plants mistakes in
    the oracle source to show that the pins catch them."""
    global _LIB, _LIB_PATH
    _LIB = None
    _LIB_PATH = path


_LIB_PATH: Optional[str] = None


def lib() -> ctypes.CDLL:
    """Load oracle/liboracle.so, building it with gcc if it is absent."""
    global _LIB
    if _LIB is None:
        path = _LIB_PATH or os.path.join(HERE, "liboracle.so")
        if _LIB_PATH is None and not os.path.exists(path):
            from . import build_oracle
            build_oracle.build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        D = ctypes.c_double
        L.orc_feq.argtypes = [D, D, D, P]
        L.orc_geq.argtypes = [D, D, D, D, P]
        L.orc_step.argtypes = [P, P, P, P, P, P, P, P, P]
        L.orc_init_eq.argtypes = [P, P, P, P, P, P, P]
        L.orc_moments.argtypes = [P, P, P, P, P, P, P]
        L.orc_totals.argtypes = [P, P, P, P, P]
        for fn in ("orc_feq", "orc_geq", "orc_step", "orc_init_eq",
                   "orc_moments", "orc_totals"):
            getattr(L, fn).restype = None
        L.orc_cde_step.argtypes = [P] * 8
        L.orc_cde_step.restype = None
        L.orc_adjoint_step.argtypes = [P] * 9
        L.orc_adjoint_step.restype = None
        L.orc_threads.argtypes = []
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        _LIB = L
    return _LIB


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    """D2Q9 equilibrium of Eq. (5) with the weights of Eq. (6)."""
    out = np.zeros(9)
    lib().orc_feq(rho, ux, uy, _ptr(out))
    return out


def geq(C: float, ux: float, uy: float, w0: float) -> np.ndarray:
    """Linear compound equilibrium, Eq. (9) generalised to a rest weight w0."""
    out = np.zeros(5)
    lib().orc_geq(C, ux, uy, w0, _ptr(out))
    return out


def threads() -> int:
    """OpenMP threads used by one oracle step."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """OpenMP threads for the following oracle steps."""
    lib().orc_set_threads(int(n))


def tau_g_from_D(D: float, w0: float) -> float:
    """Compound relaxation time for diffusion coefficient D.

    The paper states D = (2 tau_g - 1)/4 for its D2Q4 lattice (after Eq. 9),
    i.e. D = cs2 (tau_g - 1/2) with cs2 = 1/2. With a rest weight w0 the
    lattice sound speed squared is cs2 = (1 - w0)/2.
    """
    cs2 = (1.0 - w0) / 2.0
    return 0.5 + D / cs2


def segment_extent(mask: np.ndarray, seg_id: int, normal) -> tuple:
    """Halfway-wall positions (s0, s1) of a segment's ghost line.

    The tangential coordinate is y for a segment whose normal is along x and
    x otherwise; the profile vanishes half a cell beyond the outermost ghost
    cells, where the neighbouring walls sit under halfway bounce-back.
    """
    ys, xs = np.nonzero(mask == seg_id)
    if ys.size == 0:
        raise ValueError(f"segment {seg_id} has no cells in the mask")
    s = ys if normal[0] != 0 else xs
    return float(s.min()) - 0.5, float(s.max()) + 0.5


class Oracle:
    """Two-array FP64 reference run of the coupled D2Q9 + D2Q5 lattice."""

    def __init__(self, mask: np.ndarray, *, tau_f: float, D: float,
                 w0: float = 1.0 / 3.0, rho0: float = 1.0, k_decay: float = 0.0,
                 periodic: Sequence[bool] = (False, False),
                 segments: Iterable = (), schedule: Optional[Sequence] = None,
                 t_origin: int = 0, R: Optional[np.ndarray] = None,
                 tau_g: Optional[float] = None, wall_scheme: str = "bounce_back"):
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.ny, self.nx = self.mask.shape
        self.w0 = float(w0)
        self.tau_f = float(tau_f)
        self.tau_g = float(tau_g) if tau_g is not None else tau_g_from_D(D, w0)
        self.rho0 = float(rho0)
        self.segments = {s.id: s for s in segments}
        self.schedule = list(schedule) if schedule else None
        self.t_origin = int(t_origin)
        self.t = 0

        self._kind = np.zeros(256, np.int32)
        self._nrm = np.zeros((256, 2), np.int32)
        self._umax = np.zeros(256)
        self._s0 = np.zeros(256)
        self._s1 = np.ones(256)
        self._cin_default = np.zeros(256)
        self._rho = np.ones(256)
        self._fixc = np.zeros(256, np.int32)
        for s in self.segments.values():
            self._kind[s.id] = SEG_KIND[s.kind]
            self._nrm[s.id] = s.normal
            self._umax[s.id] = s.u_max
            self._cin_default[s.id] = s.c_in
            self._s0[s.id], self._s1[s.id] = segment_extent(self.mask, s.id, s.normal)
            if s.kind == "pressure":
                self._rho[s.id] = float(s.rho)
                self._fixc[s.id] = int(bool(s.fix_c))
        self.R = None if R is None else np.ascontiguousarray(R, dtype=np.float64)

        self._c = _OrcLattice(
            self.nx, self.ny, int(bool(periodic[0])), int(bool(periodic[1])),
            _ptr(self.mask), self.tau_f, self.tau_g, self.w0, self.rho0,
            float(k_decay), _ptr(self.R), _ptr(self._kind), _ptr(self._nrm),
            _ptr(self._umax), _ptr(self._s0), _ptr(self._s1), _ptr(self._rho),
            _ptr(self._fixc), {"bounce_back": 0, "equilibrium": 1}[wall_scheme])
        self.wall_scheme = wall_scheme
        n = self.nx * self.ny
        self.f = np.zeros((self.ny, self.nx, 9))
        self.g = np.zeros((self.ny, self.nx, 5))
        self._fn = np.zeros_like(self.f)
        self._gn = np.zeros_like(self.g)
        self.flux_mass = np.zeros(256)
        self.flux_solute = np.zeros(256)
        self.init()

    def set_wall_scheme(self, wall_scheme: str) -> None:
        """Switch the wall conditions for the following steps."""
        self._c.wall_scheme = {"bounce_back": 0, "equilibrium": 1}[wall_scheme]
        self.wall_scheme = wall_scheme

    # -- schedule -------------------------------------------------------
    def phase(self, t: int):
        """(open[256], c_in[256]) in force during step t -> t+1.

        The schedule is a periodic list of phases; phase k covers the steps
        [t_origin + start_k, t_origin + start_k + duration_k) modulo the
        period. With no schedule every segment is open.
        """
        open_ = np.zeros(256, np.uint8)
        c_in = self._cin_default.copy()
        if self.schedule is None:
            for sid in self.segments:
                open_[sid] = 1
            return open_, c_in
        period = sum(int(p.duration) for p in self.schedule)
        tau = (t - self.t_origin) % period
        for p in self.schedule:
            if tau < p.duration:
                for sid in p.open:
                    open_[sid] = 1
                for sid, v in dict(p.c_in).items():
                    c_in[sid] = v
                return open_, c_in
            tau -= p.duration
        raise AssertionError("unreachable")

    # -- state ------------------------------------------------------------
    def init(self, rho=None, ux=None, uy=None, C=None):
        shape = (self.ny, self.nx)
        def full(a, v):
            return np.full(shape, v) if a is None else np.ascontiguousarray(a, np.float64).reshape(shape)
        rho, ux, uy, C = full(rho, self.rho0), full(ux, 0.0), full(uy, 0.0), full(C, 0.0)
        lib().orc_init_eq(ctypes.byref(self._c), _ptr(rho), _ptr(ux), _ptr(uy),
                          _ptr(C), _ptr(self.f), _ptr(self.g))
        self.t = 0
        self.flux_mass[:] = 0.0
        self.flux_solute[:] = 0.0

    def set_populations(self, f: np.ndarray, g: np.ndarray, t: int = 0):
        self.f[...] = np.asarray(f, np.float64).reshape(self.f.shape)
        self.g[...] = np.asarray(g, np.float64).reshape(self.g.shape)
        self.t = int(t)

    def step(self, n: int = 1):
        L = lib()
        for _ in range(int(n)):
            open_, c_in = self.phase(self.t)
            L.orc_step(ctypes.byref(self._c), _ptr(self.f), _ptr(self.g),
                       _ptr(self._fn), _ptr(self._gn), _ptr(open_), _ptr(c_in),
                       _ptr(self.flux_mass), _ptr(self.flux_solute))
            self.f, self._fn = self._fn, self.f
            self.g, self._gn = self._gn, self.g
            self.t += 1

    def cde_step(self, n: int, fields: Sequence, phase_field: Optional[Sequence[int]] = None):
        """Advance only the compound n steps on frozen velocity fields (the
        paper's decoupled production path); f is left as it is.

        fields: list of (ux, uy) arrays of shape (ny, nx); phase_field[k]:
        the field used while schedule phase k is in force (default: field 0
        throughout). Boundary fluxes of the compound go to flux_solute.
        """
        fl = [(np.ascontiguousarray(ux, np.float64).reshape(self.ny, self.nx),
               np.ascontiguousarray(uy, np.float64).reshape(self.ny, self.nx))
              for ux, uy in fields]
        L = lib()
        for _ in range(int(n)):
            open_, c_in = self.phase(self.t)
            k = self.phase_index(self.t)
            ux, uy = fl[phase_field[k] if phase_field is not None else 0]
            L.orc_cde_step(ctypes.byref(self._c), _ptr(self.g), _ptr(self._gn), _ptr(ux),
                           _ptr(uy), _ptr(open_), _ptr(c_in), _ptr(self.flux_solute))
            self.g, self._gn = self._gn, self.g
            self.t += 1

    def phase_index(self, t: int) -> int:
        """Index of the schedule phase in force during step t (0 without a
        schedule)."""
        if self.schedule is None:
            return 0
        period = sum(int(p.duration) for p in self.schedule)
        tau = (t - self.t_origin) % period
        for k, p in enumerate(self.schedule):
            if tau < p.duration:
                return k
            tau -= p.duration
        raise AssertionError("unreachable")

    def fields(self):
        """rho, ux, uy, C arrays of shape (ny, nx); NaN off the fluid."""
        shape = (self.ny, self.nx)
        rho, ux, uy, C = (np.empty(shape) for _ in range(4))
        lib().orc_moments(ctypes.byref(self._c), _ptr(self.f), _ptr(self.g),
                          _ptr(rho), _ptr(ux), _ptr(uy), _ptr(C))
        return rho, ux, uy, C

    def totals(self):
        """(fluid mass, compound amount) summed over fluid nodes."""
        m = ctypes.c_double()
        s = ctypes.c_double()
        lib().orc_totals(ctypes.byref(self._c), _ptr(self.f), _ptr(self.g),
                         ctypes.byref(m), ctypes.byref(s))
        return m.value, s.value

    # -- discrete adjoint -------------------------------------------------
    def adjoint(self, n_steps: int, weight: np.ndarray, target: np.ndarray):
        """Run n_steps forward from the current state, then the discrete
        adjoint back to the start, for L = 1/2 sum_x weight (C_T - target)^2.

        Returns (loss, dL/dC_in per mask value [256], dL/dD, dL/dR [ny, nx]).
        Every intermediate state is kept in memory (small lattices only).
        """
        if any(s.kind == "pressure" for s in self.segments.values()):
            raise NotImplementedError("the pressure boundary's rescaling is not linear in g")
        if self.wall_scheme != "bounce_back":
            raise NotImplementedError("the adjoint is written for bounce-back walls")
        weight = np.asarray(weight, np.float64).reshape(self.ny, self.nx)
        target = np.asarray(target, np.float64).reshape(self.ny, self.nx)
        fl = self.mask == 0
        states = []
        for _ in range(int(n_steps)):
            states.append((self.f.copy(), self.g.copy(), self.phase(self.t)[0], self.t))
            self.step(1)
        C = self.g.sum(axis=2)
        resid = np.where(fl, weight * (C - target), 0.0)
        loss = 0.5 * float(np.sum(np.where(fl, weight * (C - target) ** 2, 0.0)))
        lam = np.ascontiguousarray(np.repeat(resid[:, :, None], 5, axis=2))
        lam_out = np.zeros_like(lam)
        dR = np.zeros((self.ny, self.nx))
        dcin = np.zeros(256)
        domega = ctypes.c_double(0.0)
        L = lib()
        for f, g, open_, _t in reversed(states):
            L.orc_adjoint_step(ctypes.byref(self._c), _ptr(f), _ptr(g), _ptr(lam),
                               _ptr(lam_out), _ptr(open_), _ptr(dR), _ptr(dcin),
                               ctypes.byref(domega))
            lam, lam_out = lam_out, lam
        self.lam0 = lam
        cs2 = (1.0 - self.w0) / 2.0
        domega_dD = -1.0 / (self.tau_g ** 2 * cs2)
        return loss, dcin, domega.value * domega_dD, dR
