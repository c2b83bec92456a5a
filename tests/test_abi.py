"""CPU checks of the C-ABI library: it loads and exports every symbol the header declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clot.h")
PKG = os.path.join(ROOT, "paper_2304_09180_amd")
LIB = os.path.join(PKG, "libclot.so")
# (cells per tile, cell species) of every library built
VARIANTS = {"libclot.so": (256, 15), "libclot_t512.so": (512, 15), "libclot_t1024.so": (1024, 15),
            "libclot_inh.so": (256, 17)}


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(clot_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared()
    for n in ("clot_create", "clot_step", "clot_get_field", "clot_set_field", "clot_destroy", "clot_init_state"):
        assert n in names


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_library_exports_every_declared_symbol(name):
    path = os.path.join(PKG, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not built")
    lib = ctypes.CDLL(path)
    for n in declared():
        assert hasattr(lib, n), n
    lib.clot_tile_cells.restype = ctypes.c_int32
    lib.clot_cell_species.restype = ctypes.c_int32
    assert (lib.clot_tile_cells(), lib.clot_cell_species()) == VARIANTS[name]


def test_binding_knows_every_declared_symbol():
    from paper_2304_09180_amd import clot
    assert set(declared()) == set(clot.exported_symbols())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libclot.so not built")
def test_params_default_and_argument_checks_without_gpu():
    from paper_2304_09180_amd import clot
    lib = clot.load()
    p = clot.Params()
    assert lib.clot_params_default(ctypes.byref(p)) == 0
    assert p.nu == 2.62507 and p.M_rxn == 2 and p.P_max == 6.67e7
    assert p.rtol_s == 1e-13 and p.rtol_tr == 1e-13 and p.I_0 == 3.4e-3 and p.mom_mg == 1 and p.mg_brick == 1   # the last fields
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


@pytest.mark.skipif(not os.path.exists(os.path.join(PKG, "libclot_inh.so")), reason="libclot_inh.so not built")
def test_inhibitor_build_defaults_workspace_and_refusals_without_gpu():
    """The inhibitor build's defaults carry the inhibitor's constants, its workspace holds
    two more cell species and two more transport systems than the base build's, and the
    batch entry points of the base model's reaction network refuse before any GPU work."""
    from paper_2304_09180_amd import clot
    lib = clot.load(256, inhibitor=True)
    p = clot.Params()
    assert lib.clot_params_default(ctypes.byref(p)) == 0
    assert p.k_I == 7.1 and p.I_0 == 3.4e-3
    import clot_inputs as ci
    d = ci.workload("channel2d_64x16")
    arr = (clot.Channel * 1)(clot.channel_struct(d))
    n_inh, n_base = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.clot_query_workspace(arr, 1, clot.FP64, ctypes.byref(n_inh)) == 0
    assert clot.load().clot_query_workspace(arr, 1, clot.FP64, ctypes.byref(n_base)) == 0
    # per cell at least: 2 species + 2 x (transport solution, diagonal, rhs, 6 couplings,
    # history) + 2 x 7 Krylov vectors, 8 bytes each
    assert n_inh.value - n_base.value >= 64 * 16 * 8 * (2 + 2 * 10 + 2 * 7)
    rows = (ctypes.c_double * 64)()
    inc = (ctypes.c_double * 64)()
    assert lib.clot_rxn_rk4_batch(ctypes.byref(p), rows, 1, inc, None) == -1
    assert lib.clot_surr_dataset(ctypes.byref(p), rows, inc, 1, None, None, None, rows, None) == -1
    for bad in (dict(k_I=-1.0), dict(I_0=float("nan"))):
        q = clot.Params()
        lib.clot_params_default(ctypes.byref(q))
        for k, v in bad.items():
            setattr(q, k, v)
        ctx = ctypes.c_void_p()
        assert lib.clot_create(arr, 1, ctypes.byref(q), clot.FP64, ctypes.c_void_p(256), 1 << 30, None,
                               ctypes.byref(ctx)) == -1


def test_binding_refuses_libraries_that_are_not_built():
    from paper_2304_09180_amd import clot
    with pytest.raises(clot.ClotError):
        clot.load(512, inhibitor=True)      # the inhibitor model is built at 256 cells per tile only
    with pytest.raises(clot.ClotError):
        clot.load(384)
    assert clot.lib_path(256, True).endswith("libclot_inh.so")
    assert clot.lib_path(1024).endswith("libclot_t1024.so")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libclot.so not built")
def test_multigrid_sweep_count_is_checked_without_gpu():
    from paper_2304_09180_amd import clot
    import clot_inputs as ci
    lib = clot.load()
    arr = (clot.Channel * 1)(clot.channel_struct(ci.workload("channel2d_64x16")))
    for field, bad in (("mg_sweeps", 5), ("mg_sweeps", -1), ("mg_brick", 2), ("mg_brick", -1)):
        q = clot.Params()
        lib.clot_params_default(ctypes.byref(q))
        setattr(q, field, bad)
        ctx = ctypes.c_void_p()
        assert lib.clot_create(arr, 1, ctypes.byref(q), clot.FP64, ctypes.c_void_p(256), 1 << 30, None,
                               ctypes.byref(ctx)) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libclot.so not built")
def test_brick_shapes_without_gpu():
    from paper_2304_09180_amd import clot
    for kernel in clot.BRICK_KERNELS:
        for dim in (2, 3):
            for q in range(clot.N_BRICK_SHAPES):
                bx, by, bz = clot.brick_dims(dim, q, kernel)
                assert bx * by * bz == 1024 and (dim == 3 or bz == 1)
                assert bx % 2 == 0 and by % 2 == 0 and (dim == 2 or bz % 2 == 0)   # whole aggregates
    assert clot.brick_dims(3, 0, "p_down") == (16, 8, 8) and clot.brick_dims(3, 0) == (32, 8, 4)
    lib = clot.load()
    v = (ctypes.c_int32 * 3)()
    assert lib.clot_brick_dims(3, 4, v) == -1 and lib.clot_brick_dims(1, 0, v) == -1
    assert lib.clot_brick_kernel_dims(5, 3, 0, v) == -1 and lib.clot_brick_kernel_dims(-1, 3, 0, v) == -1
    assert lib.clot_set_brick_shape(None, 0, 0) == -1


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on exactly one GPU: with --gpus 2 it prints one JSON line naming
    the reason and exits with status 2, before touching a device."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2, (r.returncode, r.stderr[-500:])
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
