"""ctypes binding of the clotting-step C ABI (include/clot.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
libclot.so.  PyTorch supplies the device workspace (a uint8 tensor) and the HIP
stream; it does no model arithmetic here.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
TILES = (256, 512, 1024)


def lib_path(tile: int = 256, inhibitor: bool = False) -> str:
    """The library built for `tile` cells per block, with the inhibitor model or
    without (see build.py)."""
    stem = "libclot_inh" if inhibitor else "libclot"
    return os.path.join(_HERE, f"{stem}.so" if tile == 256 else f"{stem}_t{tile}.so")


LIB_PATH = lib_path(256)

FP64, FP32_MIXED = 0, 1
PLAIN, SURROGATE = 0, 1

FIELDS = ["UX", "UY", "UZ", "P", "PHIX", "PHIY", "PHIZ",
          "PMU", "PMA", "PBA", "PBSE", "ADP", "S1", "S2", "E1", "E2",
          "S1B", "S2B", "E1B", "E2B", "C1", "C2", "E0", "C0", "ETA", "THETAB", "SIGMA", "HADH",
          "I", "E2I"]                # the last two: inhibitor build only
FIELD = {n: i for i, n in enumerate(FIELDS)}
SPECIES_FIELDS = FIELDS[7:22]
INHIBITOR_FIELDS = ["I", "E2I"]

STATUS = {0: "OK", 1: "W_NOTCONV", 2: "W_FALLBACK", 3: "W_NONFINITE", -1: "EINVAL", -2: "ENOMEM", -3: "EWORKSPACE",
          -4: "EHIP", -5: "ESTATE", -6: "ENAN"}


class Channel(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("Lx", C.c_double), ("Ly", C.c_double), ("Lz", C.c_double),
                ("inj_x0", C.c_double), ("inj_x1", C.c_double), ("inj_z0", C.c_double), ("inj_z1", C.c_double),
                ("shear", C.c_double), ("K_y", C.c_double), ("K_z", C.c_double), ("dt", C.c_double)]


_PARAM_DOUBLES_A = ["nu", "C_CK", "D_P", "D_ADP", "D_chem", "P_diam", "P_max", "P_0", "k_adh", "kcoh_Pmax",
                    "eta_t", "eta_star", "L_eta_over_Pdiam", "k_adp", "adp_crit", "k_e2", "e2_crit",
                    "A_hat", "tau_f", "dtau", "N_A", "N1", "N2",
                    "kC0p", "kC0m", "kC0cat", "kC1p", "kC1m", "kC1cat", "kC2p", "kC2m", "kC2cat",
                    "kS1p", "kS1m", "kE1p", "kE1m", "kS2p", "kS2m", "kE2p", "kE2m",
                    "S1_0", "S2_0", "E0_0", "p_out"]


class Params(C.Structure):
    _fields_ = ([(n, C.c_double) for n in _PARAM_DOUBLES_A] +
                [("M_rxn", C.c_int32), ("n_corr", C.c_int32), ("max_iter", C.c_int32),
                 ("marg_m", C.c_int32), ("marg_n", C.c_int32),
                 ("rtol_p", C.c_double), ("rtol_s", C.c_double), ("rtol_inner", C.c_double),
                 ("mg_tail", C.c_int32), ("mg_sweeps", C.c_int32),
                 ("ddt_psi", C.c_double), ("max_co", C.c_double), ("dt_growth", C.c_double),
                 ("k_I", C.c_double), ("I_0", C.c_double), ("rtol_tr", C.c_double),
                 ("mom_mg", C.c_int32), ("mg_brick", C.c_int32)])


class Stats(C.Structure):
    _fields_ = [("it_mom", C.c_int32), ("it_p", C.c_int32 * 8), ("it_eta", C.c_int32), ("it_tr", C.c_int32),
                ("refine_p", C.c_int32 * 8),
                ("res_mom", C.c_double), ("res_p", C.c_double), ("res_eta", C.c_double), ("res_tr", C.c_double),
                ("fallback_frac", C.c_double), ("steps", C.c_int64), ("t", C.c_double), ("dt", C.c_double),
                ("div_rel", C.c_double), ("min_species", C.c_double), ("sysit_tr", C.c_int32)]


class ClotError(RuntimeError):
    pass


_libs = {}


def load(tile: int = 256, inhibitor: bool = False):
    """Load the library built for `tile` cells per block (with the inhibitor model:
    256 only); raises if it has not been built."""
    key = (tile, bool(inhibitor))
    if key in _libs:
        return _libs[key]
    if tile not in TILES or (inhibitor and tile != 256):
        raise ClotError(f"no library for tile {tile}{' with the inhibitor' if inhibitor else ''}")
    path = lib_path(tile, inhibitor)
    if not os.path.exists(path):
        raise ClotError(f"HIP library not built: {path} (run __graft_entry__.build())")
    # One HIP runtime per process: torch's bundled runtime carries the soname this
    # library links against, so loading torch first binds the library to it.  The
    # other order loads a second HIP/HSA runtime next to torch's (torch names the
    # unversioned file), and that second runtime finds no device.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P = C.c_void_p
    sig = {
        "clot_params_default": ([C.POINTER(Params)], C.c_int),
        "clot_query_workspace": ([C.POINTER(Channel), C.c_int32, C.c_int, C.POINTER(C.c_size_t)], C.c_int),
        "clot_create": ([C.POINTER(Channel), C.c_int32, C.POINTER(Params), C.c_int, P, C.c_size_t, P, C.POINTER(P)],
                        C.c_int),
        "clot_init_state": ([P, C.c_int32, P, C.c_size_t, P, C.c_size_t], C.c_int),
        "clot_field_count": ([P, C.c_int32, C.c_int, C.POINTER(C.c_size_t)], C.c_int),
        "clot_set_field": ([P, C.c_int32, C.c_int, P, C.c_size_t], C.c_int),
        "clot_get_field": ([P, C.c_int32, C.c_int, P, C.c_size_t], C.c_int),
        "clot_step": ([P, C.c_int32], C.c_int),
        "clot_step_async": ([P, C.c_int32], C.c_int),
        "clot_sync": ([P], C.c_int),
        "clot_get_stats": ([P, C.c_int32, C.POINTER(Stats)], C.c_int),
        "clot_state_size": ([P, C.POINTER(C.c_size_t)], C.c_int),
        "clot_save_state": ([P, P, C.c_size_t], C.c_int),
        "clot_load_state": ([P, P, C.c_size_t], C.c_int),
        "clot_set_reaction_mode": ([P, C.c_int, P, C.c_size_t, C.c_double], C.c_int),
        "clot_probe": ([P, C.c_int32], C.c_int),
        "clot_probe_read": ([P, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
        "clot_set_graph_mode": ([P, C.c_int32, C.c_double, C.c_int32], C.c_int),
        "clot_graph_info": ([P, C.POINTER(C.c_int64)], C.c_int),
        "clot_set_brick_shape": ([P, C.c_int32, C.c_int32], C.c_int),
        "clot_brick_dims": ([C.c_int32, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
        "clot_brick_kernel_dims": ([C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
        "clot_mlp_nparam": ([], C.c_int64),
        "clot_mlp_backward_workspace": ([C.c_int64], C.c_size_t),
        "clot_mlp_forward": ([P, P, P, C.c_int64, P, P, P], C.c_int),
        "clot_mlp_backward": ([P, P, P, P, P, C.c_int64, P, P, P], C.c_int),
        "clot_mlp_backward_noalloc": ([P, P, P, P, P, C.c_int64, P, P], C.c_int),
        "clot_mlp_adam": ([P, P, P, P, P, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double, P], C.c_int),
        "clot_mlp_mse": ([P, P, C.c_int64, C.c_int32, P, P, P], C.c_int),
        "clot_rxn_rk4_batch": ([C.POINTER(Params), P, C.c_int64, P, P], C.c_int),
        "clot_surr_dataset": ([C.POINTER(Params), P, P, C.c_int64, P, P, P, P, P], C.c_int),
        "clot_mfma_selftest": ([P, P, P, P], C.c_int),
        "clot_tile_cells": ([], C.c_int32),
        "clot_cell_species": ([], C.c_int32),
        "clot_destroy": ([P], None),
        "clot_last_error": ([P], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    if lib.clot_tile_cells() != tile:
        raise ClotError(f"{path} was built for {lib.clot_tile_cells()} cells per tile, not {tile}")
    if lib.clot_cell_species() != (17 if inhibitor else 15):
        raise ClotError(f"{path} carries {lib.clot_cell_species()} species")
    _libs[key] = lib
    return lib


def exported_symbols():
    """Names the C header declares (for the load/export check)."""
    return ["clot_params_default", "clot_query_workspace", "clot_create", "clot_init_state", "clot_field_count",
            "clot_set_field", "clot_get_field", "clot_step", "clot_step_async", "clot_sync", "clot_get_stats",
            "clot_set_reaction_mode", "clot_probe", "clot_probe_read", "clot_destroy", "clot_last_error",
            "clot_mlp_nparam", "clot_mlp_backward_workspace", "clot_mlp_forward", "clot_mlp_backward",
            "clot_mlp_adam", "clot_mlp_mse", "clot_rxn_rk4_batch", "clot_surr_dataset", "clot_mfma_selftest",
            "clot_cell_species", "clot_tile_cells", "clot_set_graph_mode", "clot_graph_info", "clot_state_size",
            "clot_save_state", "clot_load_state", "clot_mlp_backward_noalloc", "clot_set_brick_shape",
            "clot_brick_dims", "clot_brick_kernel_dims"]


BRICK_KERNELS = {"restrict": 0, "prolong": 1, "sweep": 2, "p_down": 3, "p_up": 4}
N_BRICK_SHAPES = 4


def brick_dims(dim, shape, kernel="restrict"):
    """(BX, BY, BZ) of a bricked kernel's shape for channels of dimension dim."""
    k = BRICK_KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    v = (C.c_int32 * 3)()
    st = load().clot_brick_kernel_dims(k, int(dim), int(shape), v)
    if st != 0:
        raise ClotError(f"brick_dims({dim}, {shape}, {kernel}): status {st}")
    return tuple(v)


PROBES = {"p_cg_a": 1, "p_cg_b": 2, "tr_b1": 3, "tr_b2": 4, "tr_b3": 5, "mom_b1": 6, "mom_b2": 7, "mom_b3": 8,
          "rxn": 9, "tr_asm": 10, "eta_cg_a": 11, "eta_cg_b": 12, "p_resid": 13, "correct": 14, "hbya": 15,
          "prhs": 16, "mom_asm": 17, "p_mg_post": 18, "rxn_fallback": 19, "mom_mg_r": 20, "mom_mg_p1": 21,
          "mom_mg_p2": 22, "p_mg_down": 23, "p_mg_up": 24,
          "p_mg_mesh_down": 25, "p_mg_mesh_up": 26}


def default_params(precision=FP64, **over) -> Params:
    p = Params()
    load().clot_params_default(C.byref(p))
    if precision == FP32_MIXED:
        p.rtol_s = 1e-7
        p.rtol_tr = 1e-8
        p.rtol_p = 1e-8
        p.rtol_inner = 1e-4
        p.max_iter = 400
    for k, v in over.items():
        setattr(p, k, v)
    return p


def channel_struct(d: dict) -> Channel:
    return Channel(d["dim"], d["nx"], d["ny"], d["nz"], d["Lx"], d["Ly"], d["Lz"], d["inj_x0"], d["inj_x1"],
                   d["inj_z0"], d["inj_z1"], d["shear"], d["K_y"], d["K_z"], d["dt"])


def ptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def check(st, what):
    if st != 0:
        raise ClotError(f"{what} failed: {STATUS.get(st, st)}")


def _check(lib, ctx, st, what):
    if st < 0:
        msg = lib.clot_last_error(ctx).decode()
        raise ClotError(f"{what} failed: {STATUS.get(st, st)} {msg}")
    return st


class Solver:
    """One context over a list of channel descriptors.

    The workspace is a torch uint8 CUDA tensor; the stream is torch's current
    stream (or the one passed in).
    """

    def __init__(self, descs, precision=FP64, params: Params | None = None, device="cuda", stream=None, tile=256,
                 inhibitor=False):
        import torch
        self.tile = tile
        self.inhibitor = bool(inhibitor)
        self.lib = load(tile, inhibitor)
        if not torch.cuda.is_available():
            raise ClotError("no GPU visible: the clotting-step library runs only on the GPU")
        self.descs = list(descs)
        self.precision = precision
        self.params = params if params is not None else default_params(precision)
        arr = (Channel * len(self.descs))(*[channel_struct(d) for d in self.descs])
        self._chs = arr
        nbytes = C.c_size_t(0)
        _check(self.lib, None, self.lib.clot_query_workspace(arr, len(self.descs), precision, C.byref(nbytes)),
               "query_workspace")
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        ctx = C.c_void_p()
        _check(self.lib, None, self.lib.clot_create(arr, len(self.descs), C.byref(self.params), precision,
                                                    C.c_void_p(self.ws.data_ptr()), nbytes,
                                                    C.c_void_p(self.stream.cuda_stream), C.byref(ctx)), "create")
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.clot_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_state(self, ch, xi_cell, xi_face):
        xc = np.ascontiguousarray(xi_cell, dtype=np.float64)
        xf = np.ascontiguousarray(xi_face, dtype=np.float64)
        _check(self.lib, self.ctx, self.lib.clot_init_state(self.ctx, ch, xc.ctypes.data, xc.size, xf.ctypes.data,
                                                            xf.size), "init_state")

    def count(self, ch, name):
        n = C.c_size_t(0)
        _check(self.lib, self.ctx, self.lib.clot_field_count(self.ctx, ch, FIELD[name], C.byref(n)), "field_count")
        return int(n.value)

    def get(self, ch, name):
        n = self.count(ch, name)
        out = np.empty(n, dtype=np.float64)
        _check(self.lib, self.ctx, self.lib.clot_get_field(self.ctx, ch, FIELD[name], out.ctypes.data, n), "get_field")
        return out

    def set(self, ch, name, values):
        v = np.ascontiguousarray(values, dtype=np.float64)
        return _check(self.lib, self.ctx, self.lib.clot_set_field(self.ctx, ch, FIELD[name], v.ctypes.data, v.size),
                      "set_field")

    def step(self, n=1):
        return _check(self.lib, self.ctx, self.lib.clot_step(self.ctx, n), "step")

    def step_async(self, n=1):
        return _check(self.lib, self.ctx, self.lib.clot_step_async(self.ctx, n), "step_async")

    def sync(self):
        return _check(self.lib, self.ctx, self.lib.clot_sync(self.ctx), "sync")

    def stats(self, ch=0):
        s = Stats()
        st = self.lib.clot_get_stats(self.ctx, ch, C.byref(s))
        _check(self.lib, self.ctx, st, "get_stats")
        return {"status": STATUS.get(st, st), "it_mom": s.it_mom, "it_p": list(s.it_p), "it_eta": s.it_eta,
                "it_tr": s.it_tr, "refine_p": list(s.refine_p), "res_mom": s.res_mom, "res_p": s.res_p,
                "res_eta": s.res_eta, "res_tr": s.res_tr, "fallback_frac": s.fallback_frac, "steps": s.steps,
                "t": s.t, "dt": s.dt, "div_rel": s.div_rel, "min_species": s.min_species, "sysit_tr": s.sysit_tr}

    def save_state(self) -> np.ndarray:
        """The context's state (device workspace and host side) as a uint8 host array."""
        n = C.c_size_t(0)
        _check(self.lib, self.ctx, self.lib.clot_state_size(self.ctx, C.byref(n)), "state_size")
        buf = np.empty(int(n.value), dtype=np.uint8)
        _check(self.lib, self.ctx, self.lib.clot_save_state(self.ctx, buf.ctypes.data, buf.size), "save_state")
        return buf

    def load_state(self, buf) -> None:
        """Restores a state saved from a context of the same channels and precision."""
        b = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(self.lib, self.ctx, self.lib.clot_load_state(self.ctx, b.ctypes.data, b.size), "load_state")

    def set_reaction_mode(self, mode, blob=None, tol=1e-3):
        """PLAIN, or SURROGATE with a float32 blob (MLP parameters + 28 scales)."""
        if mode == PLAIN:
            return _check(self.lib, self.ctx, self.lib.clot_set_reaction_mode(self.ctx, PLAIN, None, 0, 0.0), "rxn mode")
        b = np.ascontiguousarray(blob, dtype=np.float32)
        return _check(self.lib, self.ctx, self.lib.clot_set_reaction_mode(self.ctx, SURROGATE, b.ctypes.data, b.nbytes,
                                                                         float(tol)), "rxn mode")

    def probe(self, name):
        """Start timing every launch of one kernel phase (name in PROBES, or None to stop)."""
        kid = 0 if name is None else PROBES[name]
        return _check(self.lib, self.ctx, self.lib.clot_probe(self.ctx, kid), "probe")

    def probe_read(self):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        _check(self.lib, self.ctx, self.lib.clot_probe_read(self.ctx, C.byref(ms), C.byref(n)), "probe_read")
        return ms.value, n.value

    def set_graph_mode(self, on=True, budget_scale=1.1, budget_pad=1):
        """Replay whole steps as HIP graphs after two calibrating eager steps (each
        Krylov solve then runs a fixed iteration budget; see clot_set_graph_mode)."""
        return _check(self.lib, self.ctx, self.lib.clot_set_graph_mode(self.ctx, 1 if on else 0, float(budget_scale),
                                                                      int(budget_pad)), "graph mode")

    def set_brick_shape(self, kernel, shape):
        """Tile shape (0..3) of one LDS-staged momentum kernel: 'restrict', 'prolong' or 'sweep'."""
        k = BRICK_KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        return _check(self.lib, self.ctx, self.lib.clot_set_brick_shape(self.ctx, k, int(shape)), "brick shape")

    def graph_info(self):
        v = (C.c_int64 * 20)()
        _check(self.lib, self.ctx, self.lib.clot_graph_info(self.ctx, v), "graph_info")
        keys = ("mom", "p1", "p2", "p3", "eta", "tr", "passes")
        return {"on": bool(v[0]), "captures": v[1], "replays": v[2], "overflows": v[3],
                "budgets": dict(zip(keys, v[4:11])), "seen": dict(zip(keys, v[11:18])), "nodes": v[18],
                "graphs": v[19]}

    def fields(self, ch=0):
        names = ["UX", "UY", "P", "PHIX", "PHIY", "E0", "C0", "ETA", "SIGMA"] + SPECIES_FIELDS
        if self.inhibitor:
            names += INHIBITOR_FIELDS
        if self.descs[ch]["dim"] == 3:
            names += ["UZ", "PHIZ"]
        return {n: self.get(ch, n) for n in names}
