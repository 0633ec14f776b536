"""The C-ABI library builds, loads and exports every symbol the header
declares; host-side argument checks answer without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdd.h")


def _lib():
    from paper_2311_17604_amd import build, pdd
    if not os.path.exists(pdd.LIB_PATH):
        build.build()
    return pdd.load()


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pdd_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("pdd_build_grid", "pdd_knn_cost", "pdd_decimate", "pdd_ctx_create", "pdd_strerror"):
        assert n in names


def test_every_declared_symbol_is_exported():
    lib = _lib()
    for n in declared():
        assert hasattr(lib, n), n


def test_host_side_argument_errors():
    from paper_2311_17604_amd import pdd
    lib = _lib()
    assert lib.pdd_ctx_create(None, 0, None) == pdd.PDD_EINVAL
    o = pdd.Opts(k=8)
    assert lib.pdd_decimate(None, None, 10, 5, ctypes.byref(o), None, None, None) == pdd.PDD_EINVAL
    assert lib.pdd_knn_cost(None, None, 8, 0, None, None, None) == pdd.PDD_EINVAL
    assert lib.pdd_build_grid(None, None, 10, 12, 0, None) == pdd.PDD_EINVAL
    assert lib.pdd_strerror(pdd.PDD_ERANGE).decode().startswith("coordinate extent")
    assert lib.pdd_last_error(None) == b""
    lib.pdd_ctx_destroy(None)
    lib.pdd_grid_free(None, None)
