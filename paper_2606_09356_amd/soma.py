"""Python binding of libsoma_mi355x (the C-ABI in include/soma.h).

Argument marshalling only: every step of the sweep runs in the library's HIP
kernels.  PyTorch provides the device workspace (one uint8 tensor owned by
the Python object) and the HIP stream.  The library must be built
(``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

from .workloads import SystemDesc

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsoma_mi355x.so")

SOMA_OK, SOMA_EINVAL, SOMA_ENOMEM, SOMA_EDEVICE, SOMA_EOVERFLOW, SOMA_ENONFINITE, SOMA_ESTATE = \
    0, -1, -2, -3, -4, -5, -6
POS_F32, POS_CELL_F32 = 0, 1
COUNT_U16, COUNT_U32 = 0, 1
_STATUS_NAMES = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EOVERFLOW", -5: "ENONFINITE",
                 -6: "ESTATE"}


class SomaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"soma {_STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class soma_system_desc(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("N", C.c_int32), ("n_chains_a", C.c_int32),
                ("ham_form", C.c_int32), ("pattern_a", C.c_void_p), ("pattern_b", C.c_void_p),
                ("chiN", C.c_double), ("kappaN", C.c_double), ("Re", C.c_double),
                ("box", C.c_double * 3), ("grid", C.c_int32 * 3), ("move_halfwidth", C.c_double),
                ("smc_A", C.c_double), ("walls", C.c_int32 * 2), ("zones", C.c_int32 * 2)]


class soma_options(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("pos_repr", C.c_int32), ("count_width", C.c_int32),
                ("use_graph", C.c_int32), ("density_mode", C.c_int32), ("reorder_every", C.c_int32),
                ("waves_per_block", C.c_int32), ("waves_per_cu", C.c_int32), ("sys_id_base", C.c_int32),
                ("launch_order", C.c_int32),
                ("hip_stream", C.c_void_p), ("coupling", C.c_int32), ("packed_tiles", C.c_int32)]


class soma_obs(C.Structure):
    _fields_ = [("Re2", C.c_double), ("Re2_err", C.c_double), ("Rg2", C.c_double),
                ("Rg2_err", C.c_double), ("Ebond_per_chain", C.c_double),
                ("Enb_per_chain", C.c_double), ("accept_ratio", C.c_double),
                ("n_moves", C.c_uint64), ("n_accepted", C.c_uint64), ("sweep", C.c_uint64),
                ("converted_to_a", C.c_uint64), ("converted_to_b", C.c_uint64)]


class soma_info(C.Structure):
    _fields_ = [("n_systems", C.c_int32), ("n_tiles", C.c_int32), ("n_beads", C.c_int64),
                ("n_cells", C.c_int64), ("sweep", C.c_uint64), ("bytes_per_sweep", C.c_int64),
                ("density_mode", C.c_int32), ("waves_per_block", C.c_int32),
                ("waves_per_cu", C.c_int32), ("xcd_remap", C.c_int32), ("packed_tiles", C.c_int32)]


class soma_tune(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("waves_per_cu", C.c_int32), ("xcd_remap", C.c_int32),
                ("density_mode", C.c_int32), ("n_candidates", C.c_int32), ("us_per_sweep", C.c_double),
                ("us_per_sweep_before", C.c_double), ("from_cache", C.c_int32), ("packed_tiles", C.c_int32)]


class soma_ktimes(C.Structure):
    _fields_ = [("n_sweeps", C.c_int32), ("density_mode", C.c_int32), ("sweep_kernel_us", C.c_double),
                ("fold_kernel_us", C.c_double), ("sweep_us", C.c_double)]


EXPORTS = ("soma_workspace_size", "soma_create", "soma_destroy", "soma_mc_sweep", "soma_sync",
           "soma_density", "soma_fields", "soma_observables", "soma_get_positions",
           "soma_set_positions", "soma_get_state", "soma_set_state", "soma_set_fields",
           "soma_release_fields", "soma_set_sweep", "soma_get_info", "soma_autotune", "soma_tune_cache_clear",
           "soma_time_kernels", "soma_place_from_fields", "soma_set_umbrella", "soma_get_classes",
           "soma_set_classes", "soma_observables_noalloc", "soma_last_error")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # torch brings its own HIP runtime (libamdhip64.so.7); importing it first
    # makes the library bind to that same runtime, so torch streams and device
    # pointers are valid in both and only one runtime owns the device.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    L = C.CDLL(path)
    P, I32 = C.c_void_p, C.c_int32
    sig = {
        "soma_workspace_size": ([P, I32, P, P], C.c_int),
        "soma_create": ([P, I32, P, P, C.c_size_t, P], C.c_int),
        "soma_destroy": ([P], C.c_int),
        "soma_mc_sweep": ([P, I32], C.c_int),
        "soma_sync": ([P], C.c_int),
        "soma_density": ([P, I32, P, I32], C.c_int),
        "soma_fields": ([P, I32, P, I32], C.c_int),
        "soma_observables": ([P, I32, P], C.c_int),
        "soma_observables_noalloc": ([P, I32, P], C.c_int),
        "soma_get_positions": ([P, I32, P], C.c_int),
        "soma_set_positions": ([P, I32, P], C.c_int),
        "soma_get_state": ([P, I32, P, P], C.c_int),
        "soma_set_state": ([P, I32, P, P], C.c_int),
        "soma_set_fields": ([P, I32, P], C.c_int),
        "soma_release_fields": ([P, I32], C.c_int),
        "soma_set_sweep": ([P, C.c_uint64], C.c_int),
        "soma_get_info": ([P, P], C.c_int),
        "soma_autotune": ([P, I32, P], C.c_int),
        "soma_tune_cache_clear": ([], None),
        "soma_time_kernels": ([P, I32, P], C.c_int),
        "soma_place_from_fields": ([P, I32, P], C.c_int),
        "soma_set_umbrella": ([P, I32, C.c_double], C.c_int),
        "soma_get_classes": ([P, I32, P], C.c_int),
        "soma_set_classes": ([P, I32, P], C.c_int),
        "soma_last_error": ([P], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _desc_array(systems: Sequence[SystemDesc]):
    arr = (soma_system_desc * len(systems))()
    keep = []
    for k, s in enumerate(systems):
        pa = np.ascontiguousarray(s.pattern_a, dtype=np.uint8)
        pb = np.ascontiguousarray(s.pattern_b, dtype=np.uint8)
        keep += [pa, pb]
        d = arr[k]
        d.n_chains, d.N, d.n_chains_a, d.ham_form = s.n_chains, s.N, s.n_chains_a, s.ham_form
        d.pattern_a, d.pattern_b = pa.ctypes.data, pb.ctypes.data
        d.chiN, d.kappaN, d.Re = s.chiN, s.kappaN, s.Re
        d.box = (C.c_double * 3)(*s.box)
        d.grid = (C.c_int32 * 3)(*s.grid)
        d.move_halfwidth = s.move_halfwidth
        d.smc_A = float(getattr(s, "smc_A", 0.0))
        d.walls = (C.c_int32 * 2)(*(getattr(s, "walls", None) or (0, 0)))
        d.zones = (C.c_int32 * 2)(*(getattr(s, "zones", None) or (0, 0)))
    return arr, keep


class Soma:
    """A context over a batch of independent systems on one GPU."""

    def __init__(self, systems: Sequence[SystemDesc], seed: int = 0, pos_repr: str = "f32",
                 count_width: int = 16, use_graph: bool = True, density_mode: int = 0,
                 reorder_every: int = 0, waves_per_block: int = 0, waves_per_cu: int = 0,
                 sys_id_base: int = 0, launch_order: int = 0, coupling: bool = False, packed_tiles: int = 0,
                 device: str = "cuda:0", stream=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.systems: List[SystemDesc] = list(systems)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        o = soma_options()
        o.seed = seed
        o.pos_repr = POS_CELL_F32 if pos_repr in ("cell", POS_CELL_F32) else POS_F32
        if int(count_width) not in (16, 32):
            raise ValueError("count_width must be 16 or 32")
        o.count_width = COUNT_U32 if int(count_width) == 32 else COUNT_U16
        o.use_graph = int(bool(use_graph))
        o.density_mode = density_mode
        o.reorder_every = reorder_every
        o.waves_per_block = waves_per_block
        o.waves_per_cu = waves_per_cu
        o.sys_id_base = sys_id_base
        o.launch_order = launch_order
        o.coupling = int(bool(coupling))
        o.packed_tiles = int(packed_tiles)
        o.hip_stream = self.stream.cuda_stream
        self.options = o
        self.pos_repr = o.pos_repr
        arr, self._keep = _desc_array(self.systems)
        self._desc = arr
        nbytes = C.c_size_t(0)
        self._check(self.lib.soma_workspace_size(arr, len(self.systems), C.byref(o), C.byref(nbytes)), None)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        ctx = C.c_void_p()
        self._check(self.lib.soma_create(arr, len(self.systems), C.byref(o), self.workspace.data_ptr(),
                                         self.workspace.numel(), C.byref(ctx)), None)
        self.ctx = ctx

    # -- plumbing -----------------------------------------------------------
    def _check(self, rc: int, ctx):
        if rc != SOMA_OK:
            msg = self.lib.soma_last_error(ctx if ctx is not None else None)
            raise SomaError(rc, msg.decode() if msg else "")

    def _c(self, rc):
        self._check(rc, self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.soma_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- API ----------------------------------------------------------------
    def sweep(self, n: int = 1):
        self._c(self.lib.soma_mc_sweep(self.ctx, n))

    def sync(self):
        self._c(self.lib.soma_sync(self.ctx))

    def info(self) -> dict:
        i = soma_info()
        self._c(self.lib.soma_get_info(self.ctx, C.byref(i)))
        return {f: getattr(i, f) for f, _ in soma_info._fields_}

    def autotune(self, trial_sweeps: int = 5) -> dict:
        """Time every launch shape and keep the fastest (or take the cached
        shape of a context with the same key); trial sweeps are undone."""
        t = soma_tune()
        self._c(self.lib.soma_autotune(self.ctx, trial_sweeps, C.byref(t)))
        return {f: getattr(t, f) for f, _ in soma_tune._fields_}

    def time_kernels(self, n_sweeps: int = 5) -> dict:
        """Run n real sweeps eagerly with HIP events around each kernel; average durations."""
        t = soma_ktimes()
        self._c(self.lib.soma_time_kernels(self.ctx, n_sweeps, C.byref(t)))
        return {f: getattr(t, f) for f, _ in soma_ktimes._fields_}

    def density(self, sys: int = 0) -> np.ndarray:
        M = self.systems[sys].n_cells
        out = np.zeros((2, M), np.uint32)
        self._c(self.lib.soma_density(self.ctx, sys, out.ctypes.data, 0))
        return out

    def density_device(self, sys: int, dst) -> None:
        self._c(self.lib.soma_density(self.ctx, sys, dst.data_ptr(), 1))

    def fields(self, sys: int = 0) -> np.ndarray:
        M = self.systems[sys].n_cells
        out = np.zeros((2, M), np.float32)
        self._c(self.lib.soma_fields(self.ctx, sys, out.ctypes.data, 0))
        return out

    def observables(self, sys: int = 0) -> dict:
        o = soma_obs()
        self._c(self.lib.soma_observables(self.ctx, sys, C.byref(o)))
        return {f: getattr(o, f) for f, _ in soma_obs._fields_}

    def positions(self, sys: int = 0) -> np.ndarray:
        out = np.zeros((3, self.systems[sys].n_beads), np.float64)
        self._c(self.lib.soma_get_positions(self.ctx, sys, out.ctypes.data))
        return out

    def set_positions(self, sys: int, xyz: np.ndarray):
        a = np.ascontiguousarray(xyz, dtype=np.float64)
        if a.shape != (3, self.systems[sys].n_beads):
            raise ValueError("positions must have shape [3, n_chains * N]")
        self._c(self.lib.soma_set_positions(self.ctx, sys, a.ctypes.data))

    def state(self, sys: int = 0):
        B = self.systems[sys].n_beads
        f = np.zeros((3, B), np.float32)
        c = np.zeros((3, B), np.int32) if self.pos_repr == POS_CELL_F32 else None
        self._c(self.lib.soma_get_state(self.ctx, sys, f.ctypes.data, c.ctypes.data if c is not None else None))
        return (f, c) if c is not None else f

    def set_state(self, sys: int, f32: np.ndarray, cell: Optional[np.ndarray] = None):
        B = self.systems[sys].n_beads
        f = np.ascontiguousarray(f32, dtype=np.float32).reshape(3, B)
        c = np.ascontiguousarray(cell, dtype=np.int32).reshape(3, B) if cell is not None else None
        self._c(self.lib.soma_set_state(self.ctx, sys, f.ctypes.data, c.ctypes.data if c is not None else None))

    def set_fields(self, sys: int, omega: np.ndarray):
        w = np.ascontiguousarray(omega, dtype=np.float32).reshape(2, self.systems[sys].n_cells)
        self._c(self.lib.soma_set_fields(self.ctx, sys, w.ctypes.data))

    def place_from_fields(self, sys: int, phi_target: np.ndarray):
        """Place the chains of `sys` from target fields [2][M] (needs coupling=True)."""
        t = np.ascontiguousarray(phi_target, dtype=np.float32).reshape(2, self.systems[sys].n_cells)
        self._c(self.lib.soma_place_from_fields(self.ctx, sys, t.ctypes.data))

    def set_umbrella(self, sys: int, lam: float):
        self._c(self.lib.soma_set_umbrella(self.ctx, sys, float(lam)))

    def classes(self, sys: int = 0) -> np.ndarray:
        out = np.zeros(self.systems[sys].n_chains, np.uint8)
        self._c(self.lib.soma_get_classes(self.ctx, sys, out.ctypes.data))
        return out

    def set_classes(self, sys: int, cls: np.ndarray):
        c = np.ascontiguousarray(cls, dtype=np.uint8).reshape(self.systems[sys].n_chains)
        self._c(self.lib.soma_set_classes(self.ctx, sys, c.ctypes.data))

    def set_sweep(self, sweep: int):
        self._c(self.lib.soma_set_sweep(self.ctx, sweep))

    def release_fields(self, sys: int):
        self._c(self.lib.soma_release_fields(self.ctx, sys))


def tune_cache_clear():
    """Empty the library's process-wide autotune cache."""
    load_library().soma_tune_cache_clear()
