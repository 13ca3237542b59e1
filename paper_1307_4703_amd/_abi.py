"""ctypes binding of the C ABI in include/gg.h (argument marshalling only).

The names mirror the C functions. Loading fails loudly when libgg.so has not
been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgg.so")

GG_OK = 0
GG_ERR_ARG = 1
GG_ERR_MASK = 2
GG_ERR_OOM = 3
GG_ERR_HIP = 4
GG_ERR_NONFINITE = 5
GG_ERR_STATE = 6

GG_F64, GG_F32, GG_F16_SHIFTED = 0, 1, 2
GG_HOST, GG_DEVICE = 0, 1
GG_SEG_INLET, GG_SEG_OUTLET, GG_SEG_PRESSURE = 1, 2, 3
GG_FIRST_SEGMENT = 2
GG_WALL_BOUNCE_BACK, GG_WALL_PAPER = 0, 1
GG_LAYOUT_PLANES, GG_LAYOUT_PAIRED = 0, 1
WALL_SCHEMES = {"bounce_back": GG_WALL_BOUNCE_BACK, "equilibrium": GG_WALL_PAPER}
GG_MAX_SEGMENTS = 16
GG_MAX_PHASES = 64

STORAGE = {"f64": GG_F64, "f32": GG_F32, "f16": GG_F16_SHIFTED}


class gg_params(ctypes.Structure):
    _fields_ = [("tau_f", ctypes.c_double), ("D", ctypes.c_double),
                ("w0", ctypes.c_double), ("rho0", ctypes.c_double),
                ("k_decay", ctypes.c_double), ("c_shift", ctypes.c_double),
                ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32)]


GG_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
GG_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class gg_alloc(ctypes.Structure):
    _fields_ = [("alloc", GG_ALLOC_FN), ("release", GG_RELEASE_FN), ("ctx", ctypes.c_void_p)]


class gg_phase(ctypes.Structure):
    _fields_ = [("duration", ctypes.c_int64), ("open_mask", ctypes.c_uint32),
                ("c_in_set", ctypes.c_uint32),
                ("c_in", ctypes.c_double * GG_MAX_SEGMENTS)]


class gg_diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("n_fluid", ctypes.c_int64),
                ("n_nonfinite", ctypes.c_int64),
                ("mass", ctypes.c_double), ("solute", ctypes.c_double),
                ("mass_in", ctypes.c_double), ("mass_out", ctypes.c_double),
                ("solute_in", ctypes.c_double), ("solute_out", ctypes.c_double),
                ("max_u", ctypes.c_double), ("max_u_region", ctypes.c_double),
                ("max_pe_region", ctypes.c_double),
                ("seg_mass", ctypes.c_double * GG_MAX_SEGMENTS),
                ("seg_solute", ctypes.c_double * GG_MAX_SEGMENTS)]


class gg_grads(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_double),
                ("d_c_in", ctypes.c_double * GG_MAX_SEGMENTS),
                ("d_D", ctypes.c_double), ("d_omega_g", ctypes.c_double),
                ("ckpt_every", ctypes.c_int64), ("n_checkpoints", ctypes.c_int64)]


class gg_profile(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("n_pass", ctypes.c_int64),
                ("ms_pass", ctypes.c_double), ("n_graph", ctypes.c_int64),
                ("ms_graph", ctypes.c_double), ("graph_passes", ctypes.c_int64),
                ("graph_singles", ctypes.c_int64), ("n_single", ctypes.c_int64 * 2),
                ("ms_single", ctypes.c_double * 2), ("n_monitor", ctypes.c_int64),
                ("pass_fluid", ctypes.c_int64), ("pass_side_fluid", ctypes.c_int64),
                ("pass_tiles", ctypes.c_int64), ("pass_side_tiles", ctypes.c_int64),
                ("n_pass2", ctypes.c_int64), ("ms_pass2", ctypes.c_double),
                ("fuse", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("steps_per_pass", ctypes.c_int32)]


class GGError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where} failed with status {status}: {message}")
        self.status = status


_LIB = None

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
D = ctypes.c_double
SIGS = {
    "gg_create": [P, I32, I32, ctypes.POINTER(gg_params), ctypes.c_int, P, ctypes.POINTER(P)],
    "gg_create_ex": [P, I32, I32, ctypes.POINTER(gg_params), ctypes.c_int, P,
                     ctypes.POINTER(gg_alloc), ctypes.POINTER(P)],
    "gg_set_segment": [P, I32, ctypes.c_int, I32, I32, D, D],
    "gg_set_pressure_segment": [P, I32, I32, I32, D, D, I32],
    "gg_set_schedule": [P, ctypes.POINTER(gg_phase), I32, I64],
    "gg_set_source": [P, P, ctypes.c_int],
    "gg_set_region": [P, P],
    "gg_init": [P, P, P, P, P, ctypes.c_int],
    "gg_step": [P, I64],
    "gg_read": [P, P, P, P, P, ctypes.c_int],
    "gg_read_populations": [P, P, P, ctypes.c_int],
    "gg_diagnostics": [P, ctypes.POINTER(gg_diag)],
    "gg_save": [P, P, ctypes.POINTER(ctypes.c_size_t)],
    "gg_load": [P, P, ctypes.c_size_t],
    "gg_set_launch": [P, I32, I32, I32],
    "gg_info": [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)],
    "gg_sync": [P],
    "gg_step_timed": [P, I64, ctypes.POINTER(D), ctypes.POINTER(D)],
    "gg_set_two_step": [P, I32, I32],
    "gg_set_layout": [P, I32],
    "gg_get_layout": [P, ctypes.POINTER(I32)],
    "gg_step2_timed": [P, I64, ctypes.POINTER(D)],
    "gg_set_velocity_field": [P, I32, P, P, D, ctypes.c_int],
    "gg_set_phase_fields": [P, P, I32],
    "gg_cde_step": [P, I64],
    "gg_set_cde_launch": [P, I32],
    "gg_adjoint": [P, I64, I64, P, P, P, P, ctypes.POINTER(gg_grads)],
    "gg_batch_create": [ctypes.POINTER(P), I32, I32, I32, I32, I32, ctypes.POINTER(P)],
    "gg_batch_step": [P, I64],
    "gg_batch_set_two_step": [P, I32, I32],
    "gg_batch_info": [P, ctypes.POINTER(I64), ctypes.POINTER(I64)],
    "gg_permute_tiles": [P, ctypes.c_uint64],
    "gg_set_wall_scheme": [P, I32],
    "gg_stream_copy": [P, P, ctypes.c_size_t, I32, P, ctypes.POINTER(D)],
    "gg_set_monitor": [P, I64],
    "gg_monitor_read": [P, ctypes.POINTER(gg_diag), ctypes.POINTER(I64)],
    "gg_step_profile": [P, I64, ctypes.POINTER(gg_profile)],
    "gg_diagnostics_noalloc": [P, ctypes.POINTER(gg_diag)],
    "gg_batch_form": [P] + [ctypes.POINTER(I32)] * 5,
}
GG_AUTOTUNE = -1


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.gg_destroy.argtypes = [P]
        L.gg_destroy.restype = None
        L.gg_batch_destroy.argtypes = [P]
        L.gg_batch_destroy.restype = None
        L.gg_last_error.argtypes = []
        L.gg_last_error.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


def check(status: int, where: str) -> None:
    if status != GG_OK:
        msg = lib().gg_last_error().decode(errors="replace")
        raise GGError(status, where, msg)


def call(name: str, *args) -> None:
    check(getattr(lib(), name)(*args), name)
