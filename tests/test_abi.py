"""CPU checks of the C-ABI library: it loads and exports every symbol the header declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clot.h")
PKG = os.path.join(ROOT, "paper_2304_09180_amd")
LIB = os.path.join(PKG, "libclot.so")
VARIANTS = {256: LIB, 512: os.path.join(PKG, "libclot_t512.so"), 1024: os.path.join(PKG, "libclot_t1024.so")}


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(clot_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared()
    for n in ("clot_create", "clot_step", "clot_get_field", "clot_set_field", "clot_destroy", "clot_init_state"):
        assert n in names


@pytest.mark.parametrize("tile", sorted(VARIANTS))
def test_library_exports_every_declared_symbol(tile):
    path = VARIANTS[tile]
    if not os.path.exists(path):
        pytest.skip(f"{os.path.basename(path)} not built")
    lib = ctypes.CDLL(path)
    for n in declared():
        assert hasattr(lib, n), n
    lib.clot_tile_cells.restype = ctypes.c_int32
    assert lib.clot_tile_cells() == tile


@pytest.mark.skipif(not os.path.exists(LIB), reason="libclot.so not built")
def test_params_default_and_argument_checks_without_gpu():
    from paper_2304_09180_amd import clot
    lib = clot.load()
    p = clot.Params()
    assert lib.clot_params_default(ctypes.byref(p)) == 0
    assert p.nu == 2.62507 and p.M_rxn == 2 and p.P_max == 6.67e7
    assert lib.clot_params_default(None) == -1
    # workspace query is host-only arithmetic
    import clot_inputs as ci
    d = ci.workload("channel2d_64x16")
    arr = (clot.Channel * 1)(clot.channel_struct(d))
    n = ctypes.c_size_t(0)
    assert lib.clot_query_workspace(arr, 1, clot.FP64, ctypes.byref(n)) == 0
    assert n.value > 64 * 16 * 8 * 80
    n32 = ctypes.c_size_t(0)
    assert lib.clot_query_workspace(arr, 1, clot.FP32_MIXED, ctypes.byref(n32)) == 0
    assert n32.value < n.value
    bad = clot.channel_struct(dict(d, nx=1))
    assert lib.clot_query_workspace((clot.Channel * 1)(bad), 1, clot.FP64, ctypes.byref(n)) == -1
    assert lib.clot_query_workspace(arr, 0, clot.FP64, ctypes.byref(n)) == -1
    assert lib.clot_query_workspace(arr, 1, 7, ctypes.byref(n)) == -1
