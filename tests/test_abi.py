"""The C-ABI library loads and exports every entry point of include/fofse.h;
host-side argument checks that run before any HIP call (no GPU needed)."""

import ctypes
import os
import re

import pytest

from paper_2207_01205_amd import fofse as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fofse.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fofse_[a-z_]+)\s*\(", text)))


def test_library_is_built():
    assert os.path.exists(F.LIB_PATH), "run __graft_entry__.build() first"


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(F.LIB_PATH)
    names = declared_functions()
    assert set(F.EXPORTED) <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    for st in range(6):
        assert F.fofse_status_str(st) != "unknown status"
    assert F.fofse_status_str(99) == "unknown status"


def test_null_arguments_rejected_without_gpu():
    L = F.load_library()
    out = ctypes.c_void_p()
    assert L.fofse_create(None, 0, ctypes.byref(out)) == F.FOFSE_ERR_ARG
    tm = (ctypes.c_uint8 * 4)(1, 0, 0, 0)
    bad = [F.fofse_geometry(2, 2, 3, 5, tm),       # T not a power of two
           F.fofse_geometry(2, 2, 4, -1, tm),      # K < 0
           F.fofse_geometry(8, 2, 4, 5, tm),       # area larger than T
           F.fofse_geometry(0, 2, 4, 5, tm),
           F.fofse_geometry(2, 2, 4, 5, None)]
    for g in bad:
        assert L.fofse_create(ctypes.byref(g), 0, ctypes.byref(out)) == F.FOFSE_ERR_ARG
    assert L.fofse_extrapolate_batch(None, 1, None, None, None, None, None, None, None, None) == F.FOFSE_ERR_ARG
    assert L.fofse_extrapolate_batch_noalloc(None, 1, *([None] * 8)) == F.FOFSE_ERR_ARG
    assert L.fofse_extrapolate_multi(None, 1, *([None] * 8)) == F.FOFSE_ERR_ARG
    assert L.fofse_create_multi(None, 1, 0, ctypes.byref(out)) == F.FOFSE_ERR_ARG
    assert L.fofse_multi_geometry_plan(None, 0) is None
    L.fofse_destroy_multi(None)
    assert L.fofse_target_count(None) == 0
    assert L.fofse_set_path(None, 0) == F.FOFSE_ERR_ARG
    assert L.fofse_set_waves(None, 2) == F.FOFSE_ERR_ARG
    assert L.fofse_set_basis(None, F.FOFSE_BASIS_DCT) == F.FOFSE_ERR_ARG
    assert L.fofse_set_compensation(None, F.FOFSE_COMP_FULL) == F.FOFSE_ERR_ARG
    assert L.fofse_backward(None, 1, *([None] * 10)) == F.FOFSE_ERR_ARG
    assert L.fofse_backward(None, 0, *([None] * 10)) == F.FOFSE_ERR_ARG
    assert L.fofse_set_timing(None, 1) == F.FOFSE_ERR_ARG
    buf = (ctypes.c_float * 4)()
    assert L.fofse_kernel_times(None, buf, 4) == 0
    L.fofse_destroy(None)


def test_binding_fails_loudly_without_library(tmp_path):
    saved = F._lib
    try:
        F._lib = None
        with pytest.raises(RuntimeError):
            F.load_library(str(tmp_path / "missing.so"))
    finally:
        F._lib = saved
