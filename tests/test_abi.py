"""The C ABI library: it loads, exports every function include/gg.h declares,
and its host-side validation rejects bad input before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1307_4703_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(gg_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gg_create", "gg_set_segment", "gg_set_schedule", "gg_step",
                 "gg_read", "gg_diagnostics", "gg_destroy", "gg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = A.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def _params(**kw):
    p = dict(tau_f=0.8, D=0.01, w0=1 / 3, rho0=1.0, k_decay=0.0, c_shift=0.0,
             periodic_x=0, periodic_y=0)
    p.update(kw)
    return A.gg_params(**p)


def _create(mask, **kw):
    mask = np.ascontiguousarray(mask, np.uint8)
    h = ctypes.c_void_p()
    p = _params(**kw)
    st = A.lib().gg_create(mask.ctypes.data_as(ctypes.c_void_p), mask.shape[1],
                           mask.shape[0], ctypes.byref(p), A.GG_F32, None, ctypes.byref(h))
    return st, A.lib().gg_last_error().decode()


@pytest.mark.parametrize("kw,msg", [(dict(tau_f=0.5), "tau_f"), (dict(D=0.0), "D must"),
                                    (dict(w0=1.0), "w0"), (dict(rho0=-1.0), "rho0"),
                                    (dict(k_decay=-1e-3), "k_decay")])
def test_create_rejects_bad_parameters(kw, msg):
    st, err = _create(np.zeros((8, 8)), **kw)
    assert st == A.GG_ERR_ARG and msg in err


def test_create_rejects_bad_masks():
    m = np.zeros((8, 8), np.uint8)
    m[3, 3] = 200
    st, err = _create(m)
    assert st == A.GG_ERR_MASK and "mask value 200" in err
    m = np.ones((8, 8), np.uint8)
    m[4, 4] = 0  # isolated fluid cell
    st, err = _create(m)
    assert st == A.GG_ERR_MASK and "no fluid neighbour" in err
    m2 = np.zeros((7, 7), np.uint8)
    m2[2, 3], m2[4, 3], m2[3, 2] = 2, 3, 4  # node (3,3) touches three segments
    st, err = _create(m2)
    assert st == A.GG_ERR_MASK and "more than two segments" in err


def test_null_arguments():
    h = ctypes.c_void_p()
    assert A.lib().gg_create(None, 4, 4, None, A.GG_F32, None, ctypes.byref(h)) == A.GG_ERR_ARG
    assert A.lib().gg_step(None, 1) == A.GG_ERR_ARG
    assert A.lib().gg_read(None, None, None, None, None, A.GG_HOST) == A.GG_ERR_ARG


def test_create_rejects_a_lattice_too_large():
    """One FP32 population plane must stay below 4 GiB (the kernels address
    it with 32-bit byte offsets); the check comes before any allocation."""
    big = np.zeros((30000, 40000), np.uint8)  # zero pages, never touched
    st, err = _create(big)
    assert st == A.GG_ERR_ARG and "too large" in err


def test_null_arguments_of_the_later_calls():
    assert A.lib().gg_cde_step(None, 2) == A.GG_ERR_ARG
    assert A.lib().gg_set_velocity_field(None, 0, None, None, 1.0, A.GG_HOST) == A.GG_ERR_ARG
    assert A.lib().gg_set_phase_fields(None, None, 0) == A.GG_ERR_ARG
    assert A.lib().gg_set_cde_launch(None, 14) == A.GG_ERR_ARG
    assert A.lib().gg_set_pressure_segment(None, 2, 1, 0, 1.0, 0.0, 0) == A.GG_ERR_ARG
    assert A.lib().gg_set_two_step(None, 3, 6) == A.GG_ERR_ARG
    assert A.lib().gg_set_layout(None, A.GG_LAYOUT_PAIRED) == A.GG_ERR_ARG
    assert A.lib().gg_get_layout(None, None) == A.GG_ERR_ARG


def test_create_ex_rejects_an_incomplete_allocator():
    """An allocator needs both functions; the check comes before any device
    work."""
    mask = np.zeros((8, 8), np.uint8)
    p = A.gg_params(0.8, 0.02, 1.0 / 3.0, 1.0, 0.0, 0.0, 1, 1)
    h = ctypes.c_void_p()
    al = A.gg_alloc(A.GG_ALLOC_FN(lambda n, c: None), A.GG_RELEASE_FN(), None)
    st = A.lib().gg_create_ex(mask.ctypes.data_as(ctypes.c_void_p), 8, 8, ctypes.byref(p),
                              A.STORAGE["f32"], None, ctypes.byref(al), ctypes.byref(h))
    assert st == A.GG_ERR_ARG and not h.value
    assert b"alloc" in A.lib().gg_last_error()
