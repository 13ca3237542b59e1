"""Python face of the lattice library: a thin object over the C ABI.

Every time step runs in the HIP kernels of libgg.so; this module only
marshals arguments. PyTorch, when present, supplies the HIP stream and device
buffers for device-side read-back.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Iterable, Optional, Sequence, Tuple

import numpy as np

from . import _abi as A


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _current_stream() -> Optional[int]:
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def make_phases(schedule: Sequence) -> "ctypes.Array":
    """Phase records (attributes duration, open, c_in) -> gg_phase array."""
    arr = (A.gg_phase * max(1, len(schedule)))()
    for k, p in enumerate(schedule):
        arr[k].duration = int(p.duration)
        m = 0
        for sid in p.open:
            m |= 1 << (int(sid) - A.GG_FIRST_SEGMENT)
        arr[k].open_mask = m
        cs = 0
        for sid, v in dict(p.c_in).items():
            j = int(sid) - A.GG_FIRST_SEGMENT
            cs |= 1 << j
            arr[k].c_in[j] = float(v)
        arr[k].c_in_set = cs
    return arr


def _torch_allocator(stream: Optional[int]) -> "A.gg_alloc":
    """A gg_alloc whose functions take device memory from PyTorch's caching
    allocator on the given stream (the structure keeps the callbacks alive
    and must live as long as the lattice)."""
    import torch
    dev = torch.cuda.current_device()
    st = torch.cuda.ExternalStream(stream) if stream else torch.cuda.default_stream(dev)

    def alloc(nbytes, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, st)
        except RuntimeError:  # out of memory: the library reports GG_ERR_OOM
            return None

    def release(ptr, _ctx):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:  # the interpreter (and torch) may be shutting down
            pass

    return A.gg_alloc(A.GG_ALLOC_FN(alloc), A.GG_RELEASE_FN(release), None)


class Lattice:
    """A coupled D2Q9 + D2Q5 lattice on the GPU (see include/gg.h)."""

    def __init__(self, mask: np.ndarray, *, tau_f: float, D: float,
                 w0: float = 1.0 / 3.0, rho0: float = 1.0, k_decay: float = 0.0,
                 c_shift: float = 0.0, periodic: Tuple[bool, bool] = (False, False),
                 storage: str = "f32", stream: Optional[int] = None,
                 device_allocator: Optional[str] = None, layout: str = "paired"):
        """device_allocator: None (the library's hipMalloc) or "torch" (every
        device buffer of the lattice from PyTorch's caching allocator on the
        lattice's stream, gg_create_ex). layout: "paired" or "planes" (see
        set_layout)."""
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.ny, self.nx = self.mask.shape
        self.storage = storage
        self.D = float(D)
        p = A.gg_params(float(tau_f), float(D), float(w0), float(rho0),
                        float(k_decay), float(c_shift), int(bool(periodic[0])),
                        int(bool(periodic[1])))
        self.stream = _current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        self._alloc = None
        if device_allocator is None:
            A.call("gg_create", _dptr(self.mask), self.nx, self.ny, ctypes.byref(p),
                   A.STORAGE[storage], ctypes.c_void_p(self.stream or 0), ctypes.byref(h))
        elif device_allocator == "torch":
            self._alloc = _torch_allocator(self.stream)
            A.call("gg_create_ex", _dptr(self.mask), self.nx, self.ny, ctypes.byref(p),
                   A.STORAGE[storage], ctypes.c_void_p(self.stream or 0),
                   ctypes.byref(self._alloc), ctypes.byref(h))
        else:
            raise ValueError(f"unknown device allocator {device_allocator!r}")
        self._h = h
        self.segments: Dict[int, object] = {}
        if layout != "paired":
            self.set_layout(layout)

    # ------------------------------------------------------------------
    @classmethod
    def from_workload(cls, wl, *, storage: Optional[str] = None,
                      stream: Optional[int] = None, init: bool = True,
                      device_allocator: Optional[str] = None,
                      layout: str = "paired") -> "Lattice":
        """The workload's compound shift C_s applies to FP16 storage only; the
        wider types keep C_s = 0, where a compound at rest at 0 or at an
        inlet value is held without rounding."""
        storage = storage or wl.storage
        lat = cls(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, rho0=wl.rho0,
                  k_decay=wl.k_decay, c_shift=wl.c_shift if storage == "f16" else 0.0,
                  periodic=wl.periodic, storage=storage, stream=stream,
                  device_allocator=device_allocator, layout=layout)
        for s in wl.segments:
            lat.set_segment(s.id, s.kind, s.normal, s.u_max, s.c_in,
                            getattr(s, "rho", 1.0), getattr(s, "fix_c", False))
        if wl.schedule:
            lat.set_schedule(wl.schedule, wl.t_origin)
        if wl.region is not None:
            lat.set_region(wl.region)
        if init:
            lat.init(**(wl.init or {}))
        return lat

    @property
    def handle(self):
        return self._h

    def set_segment(self, sid: int, kind: str, normal, u_max: float = 0.0,
                    c_in: float = 0.0, rho: float = 1.0, fix_c: bool = False) -> None:
        """Configure a segment: "inlet" and "outlet" (gg_set_segment, with
        u_max and c_in) or "pressure" (gg_set_pressure_segment: density rho,
        and the compound held at c_in when fix_c)."""
        if kind == "pressure":
            A.call("gg_set_pressure_segment", self._h, int(sid), int(normal[0]), int(normal[1]),
                   float(rho), float(c_in), int(bool(fix_c)))
            self.segments[int(sid)] = (kind, tuple(normal), rho, c_in, fix_c)
            return
        k = {"inlet": A.GG_SEG_INLET, "outlet": A.GG_SEG_OUTLET}[kind]
        A.call("gg_set_segment", self._h, int(sid), k, int(normal[0]),
               int(normal[1]), float(u_max), float(c_in))

    def set_schedule(self, schedule: Optional[Sequence], t_origin: int = 0) -> None:
        if not schedule:
            A.call("gg_set_schedule", self._h, None, 0, int(t_origin))
            return
        arr = make_phases(schedule)
        A.call("gg_set_schedule", self._h, arr, len(schedule), int(t_origin))

    def set_source(self, R: Optional[np.ndarray]) -> None:
        if R is None:
            A.call("gg_set_source", self._h, None, A.GG_HOST)
            return
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(self.ny, self.nx)
        A.call("gg_set_source", self._h, _dptr(R), A.GG_HOST)

    def set_region(self, region: Optional[np.ndarray]) -> None:
        if region is None:
            A.call("gg_set_region", self._h, None)
            return
        r = np.ascontiguousarray(region, dtype=np.uint8).reshape(self.ny, self.nx)
        A.call("gg_set_region", self._h, _dptr(r))

    def init(self, rho=None, ux=None, uy=None, C=None) -> None:
        arrs = []
        for a in (rho, ux, uy, C):
            arrs.append(None if a is None else
                        np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny, self.nx))
        ptrs = [None if a is None else _dptr(a) for a in arrs]
        A.call("gg_init", self._h, *ptrs, A.GG_HOST)

    def step(self, n: int = 1) -> None:
        A.call("gg_step", self._h, int(n))

    def set_launch(self, tile_x: int = 64, tile_y: int = 4, graph_chunk: int = 64) -> None:
        A.call("gg_set_launch", self._h, int(tile_x), int(tile_y), int(graph_chunk))

    def set_two_step(self, fuse: int = 3, strip_h: int = 6) -> None:
        """Two steps per pass over memory (fuse = 2: walking strips of
        strip_h rows; 3, the default: row-parallel tiles of 6 or 14 rows with
        the boundary kernel apart; 4: the same in one kernel), four steps per
        pass in runs of 8k steps (fuse = 5; other runs as fuse = 3) or
        single steps (fuse = 1); include/gg.h,
        gg_set_two_step."""
        A.call("gg_set_two_step", self._h, int(fuse), int(strip_h))

    def set_layout(self, layout: str) -> None:
        """Population layout in device memory: "paired" (f_i and g_i side by
        side for i = 0..4, a new lattice's layout, the faster one for coupled
        steps) or "planes" (one plane per population, the faster one for the
        compound-only steps); the stored state is converted, the results of
        every step are the same bits in either; include/gg.h,
        gg_set_layout."""
        code = {"planes": A.GG_LAYOUT_PLANES, "paired": A.GG_LAYOUT_PAIRED}[layout]
        A.call("gg_set_layout", self._h, code)

    @property
    def layout(self) -> str:
        v = ctypes.c_int32()
        A.call("gg_get_layout", self._h, ctypes.byref(v))
        return "paired" if v.value == A.GG_LAYOUT_PAIRED else "planes"

    def step2_timed(self, n_pairs: int) -> float:
        """Run 2 * n_pairs two-step passes between HIP events; mean duration
        of one pass in milliseconds."""
        a = ctypes.c_double()
        A.call("gg_step2_timed", self._h, int(n_pairs), ctypes.byref(a))
        return a.value

    def step_timed(self, n: int) -> Tuple[float, float]:
        """Advance n steps with every step kernel between HIP events; mean
        (even-step, odd-step) kernel durations in milliseconds."""
        a, b = ctypes.c_double(), ctypes.c_double()
        A.call("gg_step_timed", self._h, int(n), ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def step_profile(self, n: int) -> dict:
        """gg_step_profile: n steps of gg_step with HIP events around every
        plain launch of the dominant kernel (two-step pass or single step)
        and around every graph replay; durations in milliseconds."""
        p = A.gg_profile()
        A.call("gg_step_profile", self._h, int(n), ctypes.byref(p))
        return {"ms_total": p.ms_total, "n_pass": p.n_pass, "ms_pass": p.ms_pass,
                "n_graph": p.n_graph, "ms_graph": p.ms_graph, "graph_passes": p.graph_passes,
                "graph_singles": p.graph_singles,
                "n_single": list(p.n_single), "ms_single": list(p.ms_single),
                "n_monitor": p.n_monitor, "pass_fluid": p.pass_fluid,
                "pass_side_fluid": p.pass_side_fluid, "pass_tiles": p.pass_tiles,
                "pass_side_tiles": p.pass_side_tiles, "fuse": p.fuse, "rows": p.rows,
                "steps_per_pass": p.steps_per_pass, "n_pass2": p.n_pass2,
                "ms_pass2": p.ms_pass2}

    def set_monitor(self, every: int) -> None:
        """FP64 diagnostics reduced on the GPU after every `every` steps of
        gg_step, without waiting (0 turns the monitor off)."""
        A.call("gg_set_monitor", self._h, int(every))

    def monitor(self, check_finite: bool = True) -> dict:
        """The last monitor reduction (gg_monitor_read) and the number of
        reductions since set_monitor."""
        d = A.gg_diag()
        cnt = ctypes.c_int64()
        st = A.lib().gg_monitor_read(self._h, ctypes.byref(d), ctypes.byref(cnt))
        if st != A.GG_OK and (check_finite or st != A.GG_ERR_NONFINITE):
            A.check(st, "gg_monitor_read")
        out = {k: getattr(d, k) for k, _ in A.gg_diag._fields_
               if k not in ("seg_mass", "seg_solute")}
        out["seg_mass"] = np.array(d.seg_mass[:])
        out["seg_solute"] = np.array(d.seg_solute[:])
        out["count"] = cnt.value
        return out

    def sync(self) -> None:
        A.call("gg_sync", self._h)

    def set_wall_scheme(self, scheme: str) -> None:
        """"bounce_back" (halfway bounce-back, the default) or "equilibrium"
        (the paper's walls: ghost cells emitting the fluid equilibrium at the
        extrapolated density and the momentum that vanishes at the halfway
        wall, Guo's non-equilibrium extrapolation for the compound; the
        Boundary Conditions section). Steps then run one at a time."""
        if scheme not in A.WALL_SCHEMES:
            raise ValueError(f"unknown wall scheme {scheme!r}")
        A.call("gg_set_wall_scheme", self._h, A.WALL_SCHEMES[scheme])

    def permute_tiles(self, seed: int) -> None:
        """Shuffle the launch order of the tiles and strips (instrumentation)."""
        A.call("gg_permute_tiles", self._h, int(seed))

    # compound alone on frozen velocity fields (include/gg.h, gg_cde_step)
    def set_velocity_field(self, slot: int, ux: Optional[np.ndarray] = None,
                           uy: Optional[np.ndarray] = None, scale: float = 1.0) -> None:
        """Store scale * (ux, uy) (host arrays, shape (ny, nx)) in field slot
        `slot`; with neither given, scale times the velocity of the current
        fluid state."""
        if ux is None and uy is None:
            A.call("gg_set_velocity_field", self._h, int(slot), None, None, float(scale),
                   A.GG_HOST)
            return
        a = np.ascontiguousarray(ux, np.float64).reshape(self.ny, self.nx)
        b = np.ascontiguousarray(uy, np.float64).reshape(self.ny, self.nx)
        A.call("gg_set_velocity_field", self._h, int(slot), _dptr(a), _dptr(b), float(scale),
               A.GG_HOST)

    def set_phase_fields(self, slots: Optional[Sequence[int]]) -> None:
        """slots[k]: field slot used in schedule phase k (None: slot 0)."""
        if not slots:
            A.call("gg_set_phase_fields", self._h, None, 0)
            return
        arr = (ctypes.c_int32 * len(slots))(*[int(v) for v in slots])
        A.call("gg_set_phase_fields", self._h, arr, len(slots))

    def set_cde_launch(self, rows: int = 14) -> None:
        """Two-step passes over tiles of 6 or 14 rows for cde_step,
        four-step passes over 58-column tiles of 6 or 10 rows (rows = -6,
        -10), or single steps (rows = 0); include/gg.h, gg_set_cde_launch."""
        A.call("gg_set_cde_launch", self._h, int(rows))

    def cde_step(self, n: int = 2) -> None:
        """Advance the compound alone n (even) steps on the frozen fields."""
        A.call("gg_cde_step", self._h, int(n))

    def adjoint(self, n_steps: int, weight: np.ndarray, target: np.ndarray,
                r_box: Optional[Sequence[int]] = None, ckpt_every: int = 0) -> dict:
        """Advance n_steps and return L = 1/2 sum weight (C - target)^2 with
        its gradients (include/gg.h, gg_adjoint)."""
        w = np.ascontiguousarray(weight, np.float64).reshape(self.ny, self.nx)
        t = np.ascontiguousarray(target, np.float64).reshape(self.ny, self.nx)
        out = A.gg_grads()
        box = None
        dR = None
        if r_box is not None:
            box = (ctypes.c_int32 * 4)(*[int(v) for v in r_box])
            dR = np.zeros((int(r_box[3]), int(r_box[2])))
        A.call("gg_adjoint", self._h, int(n_steps), int(ckpt_every), _dptr(w), _dptr(t),
               box, None if dR is None else _dptr(dR), ctypes.byref(out))
        return {"loss": out.loss, "d_c_in": np.array(out.d_c_in[:]), "d_D": out.d_D,
                "d_omega_g": out.d_omega_g, "d_R": dR, "ckpt_every": out.ckpt_every,
                "n_checkpoints": out.n_checkpoints}

    # ------------------------------------------------------------------
    def read(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        """(rho, ux, uy, C) on the host, shape (ny, nx), NaN off the fluid."""
        out = [np.empty((self.ny, self.nx)) for _ in range(4)]
        A.call("gg_read", self._h, *[_dptr(a) for a in out], A.GG_HOST)
        return tuple(out)

    def read_device(self, rho, ux, uy, C) -> None:
        """Write the fields into device buffers (torch tensors or None)."""
        ptrs = [None if a is None else ctypes.c_void_p(a.data_ptr()) for a in (rho, ux, uy, C)]
        A.call("gg_read", self._h, *ptrs, A.GG_DEVICE)

    def populations(self) -> Tuple[np.ndarray, np.ndarray]:
        """f (9, ny, nx) and g (5, ny, nx) in natural order, FP64."""
        f = np.empty((9, self.ny, self.nx))
        g = np.empty((5, self.ny, self.nx))
        A.call("gg_read_populations", self._h, _dptr(f), _dptr(g), A.GG_HOST)
        return f, g

    def diagnostics(self, check_finite: bool = True, noalloc: bool = False) -> dict:
        """FP64 diagnostics (gg_diagnostics, or gg_diagnostics_noalloc with
        the reduction in the library's fixed device array)."""
        d = A.gg_diag()
        fn = "gg_diagnostics_noalloc" if noalloc else "gg_diagnostics"
        st = getattr(A.lib(), fn)(self._h, ctypes.byref(d))
        if st != A.GG_OK and (check_finite or st != A.GG_ERR_NONFINITE):
            A.check(st, fn)
        out = {k: getattr(d, k) for k, _ in A.gg_diag._fields_
               if k not in ("seg_mass", "seg_solute")}
        out["seg_mass"] = np.array(d.seg_mass[:])
        out["seg_solute"] = np.array(d.seg_solute[:])
        return out

    def info(self) -> dict:
        nf, nt, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        A.call("gg_info", self._h, ctypes.byref(nf), ctypes.byref(nt), ctypes.byref(t))
        return {"n_fluid": nf.value, "n_tiles": nt.value, "t": t.value}

    def save(self) -> bytes:
        n = ctypes.c_size_t(0)
        A.call("gg_save", self._h, None, ctypes.byref(n))
        buf = ctypes.create_string_buffer(n.value)
        A.call("gg_save", self._h, buf, ctypes.byref(n))
        return buf.raw[: n.value]

    def load(self, snap: bytes) -> None:
        A.call("gg_load", self._h, snap, len(snap))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            A.lib().gg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several lattices advanced by one flat launch per step (gg_batch_*).

    The lattices keep their own state; after ``step(n)`` each of them is n
    steps further, exactly as after ``Lattice.step(n)``.
    """

    def __init__(self, lattices: Sequence[Lattice], tile: Optional[Tuple[int, int]] = (64, 4),
                 persist: int = 0, graph_chunk: int = 64, fuse: int = 1, rows: int = 6):
        """tile=None: the library's autotuner picks the launch form
        (gg_batch_create with GG_AUTOTUNE; the members are left as they
        were); fuse and rows are then ignored."""
        self.lattices = list(lattices)
        arr = (ctypes.c_void_p * len(self.lattices))(*[l.handle.value for l in self.lattices])
        h = ctypes.c_void_p()
        tx, ty = tile if tile is not None else (0, 0)
        A.call("gg_batch_create", arr, len(self.lattices), int(tx), int(ty),
               A.GG_AUTOTUNE if tile is None else int(persist), int(graph_chunk), ctypes.byref(h))
        self._h = h
        if tile is None:
            f = self.form()
            self.tile, self.persist = (f["tile_x"], f["tile_y"]), f["persist"]
            return
        self.tile = tuple(tile)
        self.persist = int(persist)
        if fuse != 1:
            self.set_two_step(fuse, rows)

    def form(self) -> dict:
        """The launch form in use (gg_batch_form)."""
        v = [ctypes.c_int32() for _ in range(5)]
        A.call("gg_batch_form", self._h, *[ctypes.byref(x) for x in v])
        return dict(zip(("tile_x", "tile_y", "persist", "fuse", "rows"), [x.value for x in v]))

    def set_two_step(self, fuse: int = 4, rows: int = 6) -> None:
        """Two-step passes over all members (fuse 3 or 4), four-step passes
        (fuse 5) or single steps (fuse 1);
        include/gg.h, gg_batch_set_two_step."""
        A.call("gg_batch_set_two_step", self._h, int(fuse), int(rows))

    def step(self, n: int = 1) -> None:
        A.call("gg_batch_step", self._h, int(n))

    def info(self) -> dict:
        nt, nf = ctypes.c_int64(), ctypes.c_int64()
        A.call("gg_batch_info", self._h, ctypes.byref(nt), ctypes.byref(nf))
        return {"n_tiles": nt.value, "n_fluid": nf.value}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            A.lib().gg_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
