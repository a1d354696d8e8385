"""CPU oracle of the SCMF Monte-Carlo sweep (ctypes wrapper over soma_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
CPU-baseline leg of the benchmark may use this package; the GPU product path
never imports it.  It shares no code with the GPU library: the only common
inputs are the seeded workloads in ``paper_2606_09356_amd.workloads``.

Modes: 0 = FP64 positions, 1 = FP32-stored positions, 2 = int32 cell + FP32
offset stored positions (energies always FP64).  Coupling extensions: target
fields with placement and an umbrella potential, walls and conversion zones.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "soma_oracle.c")
LIB = os.path.join(HERE, "_soma_oracle.so")

MODE_F64, MODE_F32, MODE_CELL = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11 + OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _System(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("N", C.c_int32), ("n_chains_a", C.c_int32),
                ("ham_form", C.c_int32), ("pattern_a", C.c_void_p), ("pattern_b", C.c_void_p),
                ("chiN", C.c_double), ("kappaN", C.c_double), ("Re", C.c_double),
                ("box", C.c_double * 3), ("grid", C.c_int32 * 3),
                ("move_halfwidth", C.c_double), ("sys_id", C.c_uint32), ("smc_A", C.c_double),
                ("umb_lambda", C.c_double), ("umb_target", C.c_void_p),
                ("wall", C.c_int32 * 2), ("zone", C.c_int32 * 2)]


class _State(C.Structure):
    _fields_ = [("mode", C.c_int32), ("x", C.c_void_p), ("xf", C.c_void_p),
                ("cell", C.c_void_p), ("off", C.c_void_p), ("chain_class", C.c_void_p),
                ("conv", C.c_uint64 * 2)]


class _Obs(C.Structure):
    _fields_ = [("Re2", C.c_double), ("Re2_err", C.c_double), ("Rg2", C.c_double),
                ("Rg2_err", C.c_double), ("Ebond_per_chain", C.c_double),
                ("Enb_per_chain", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_set_positions.argtypes = [P, P, P]
        L.orc_get_positions.argtypes = [P, P, P]
        L.orc_density.argtypes = [P, P, P]
        L.orc_energy_nb.argtypes = [P, P]
        L.orc_energy_nb.restype = C.c_double
        L.orc_fields.argtypes = [P, P, P]
        L.orc_sweep.argtypes = [P, P, C.c_uint64, C.c_uint32, P, P]
        L.orc_sweep.restype = C.c_uint64
        L.orc_run.argtypes = [P, P, C.c_uint64, C.c_uint32, C.c_int32, P, P, C.c_int32]
        L.orc_run.restype = C.c_uint64
        L.orc_init_walks.argtypes = [P, C.c_uint64, P]
        L.orc_init_walks.restype = C.c_int
        L.orc_place_from_fields.argtypes = [P, P, C.c_uint64, P, P, P]
        L.orc_place_from_fields.restype = C.c_int
        L.orc_convert.argtypes = [P, P]
        L.orc_convert.restype = None
        L.orc_observables.argtypes = [P, P, P, P, P]
        L.orc_neumaier_sum.argtypes = [P, C.c_int64]
        L.orc_neumaier_sum.restype = C.c_double
        L.orc_smc_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, P, P]
        L.orc_smc_draw.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data if a is not None else None


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def neumaier_sum(v) -> float:
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    return lib().orc_neumaier_sum(_ptr(a), a.size)


def smc_draw(seed: int, sweep: int, chain: int, bead: int, sys_id: int = 0):
    """The three standard normals and the acceptance variate of one smart move."""
    xi = np.zeros(3)
    u = C.c_double(0.0)
    lib().orc_smc_draw(seed, sweep, chain, bead, sys_id, _ptr(xi), C.byref(u))
    return xi, u.value


class OracleSystem:
    """One system of the oracle: its description, stored positions, counts and fields."""

    def __init__(self, desc, sys_id: int = 0, mode: int = MODE_F64):
        """Walls and conversion zones come from the descriptor's optional
        ``walls`` ((lo, hi) z-cell faces) and ``zones`` ((lower, upper) widths
        in z cells) attributes."""
        self.desc = desc
        self.mode = mode
        self._pa = np.ascontiguousarray(desc.pattern_a, dtype=np.uint8)
        self._pb = np.ascontiguousarray(desc.pattern_b, dtype=np.uint8)
        s = _System()
        s.n_chains, s.N, s.n_chains_a = desc.n_chains, desc.N, desc.n_chains_a
        s.ham_form = desc.ham_form
        s.pattern_a, s.pattern_b = _ptr(self._pa), _ptr(self._pb)
        s.chiN, s.kappaN, s.Re = desc.chiN, desc.kappaN, desc.Re
        s.box = (C.c_double * 3)(*desc.box)
        s.grid = (C.c_int32 * 3)(*desc.grid)
        s.move_halfwidth = desc.move_halfwidth
        s.smc_A = float(getattr(desc, "smc_A", 0.0))
        s.sys_id = sys_id
        walls = getattr(desc, "walls", None) or (0, 0)
        zones = getattr(desc, "zones", None) or (0, 0)
        s.wall = (C.c_int32 * 2)(*walls)
        s.zone = (C.c_int32 * 2)(*zones)
        s.umb_lambda = 0.0
        s.umb_target = None
        self._target = None
        self._sys = s
        B, M = desc.n_beads, desc.n_cells
        self.x = np.zeros((3, B), np.float64) if mode == MODE_F64 else None
        self.xf = np.zeros((3, B), np.float32) if mode == MODE_F32 else None
        self.cell = np.zeros((3, B), np.int32) if mode == MODE_CELL else None
        self.off = np.zeros((3, B), np.float32) if mode == MODE_CELL else None
        self.chain_class = (np.arange(desc.n_chains) >= desc.n_chains_a).astype(np.uint8)
        st = _State()
        st.mode = mode
        st.x, st.xf, st.cell, st.off = _ptr(self.x), _ptr(self.xf), _ptr(self.cell), _ptr(self.off)
        st.chain_class = _ptr(self.chain_class)
        self._st = st
        self.counts = np.zeros((2, M), np.uint32)
        self.omega = np.zeros((2, M), np.float64)

    @property
    def sp(self):
        return C.byref(self._sys)

    @property
    def stp(self):
        return C.byref(self._st)

    # -- state --------------------------------------------------------------
    def set_positions(self, xyz: np.ndarray, refresh: bool = True):
        a = np.ascontiguousarray(xyz, dtype=np.float64)
        assert a.shape == (3, self.desc.n_beads)
        lib().orc_set_positions(self.sp, self.stp, _ptr(a))
        if refresh:
            self.density()
            self.fields()

    def positions(self) -> np.ndarray:
        out = np.zeros((3, self.desc.n_beads), np.float64)
        lib().orc_get_positions(self.sp, self.stp, _ptr(out))
        return out

    def init_walks(self, seed: int) -> np.ndarray:
        out = np.zeros((3, self.desc.n_beads), np.float64)
        rc = lib().orc_init_walks(self.sp, seed, _ptr(out))
        if rc != 0:
            raise ValueError(f"initial walks failed ({rc}): chains do not fit between the walls")
        return out

    # -- coupling: target fields, umbrella, conversion zones ----------------
    def set_target(self, phi_target: np.ndarray):
        """Target concentration fields [2][M] (phi_A, phi_B) for placement and umbrella."""
        self._target = np.ascontiguousarray(np.asarray(phi_target, dtype=np.float64).reshape(2, -1))
        self._sys.umb_target = _ptr(self._target)

    def set_umbrella(self, lam: float):
        """Umbrella strength lambda (0 switches it off); needs set_target."""
        if lam > 0 and self._target is None:
            raise ValueError("set_target first")
        self._sys.umb_lambda = float(lam)

    def place_from_fields(self, seed: int):
        """Positions of the placement from the target fields; returns (xyz, targets, cells)."""
        B, n = self.desc.n_beads, self.desc.n_chains
        xyz = np.zeros((3, B), np.float64)
        tg = np.zeros((3, n), np.float64)
        cells = np.zeros(n, np.int64)
        rc = lib().orc_place_from_fields(self.sp, self.stp, seed, _ptr(xyz), _ptr(tg), _ptr(cells))
        if rc != 0:
            raise ValueError(f"placement failed ({rc})")
        return xyz, tg, cells

    def convert(self):
        lib().orc_convert(self.sp, self.stp)

    @property
    def conversions(self):
        return int(self._st.conv[0]), int(self._st.conv[1])

    # -- steps --------------------------------------------------------------
    def density(self) -> np.ndarray:
        lib().orc_density(self.sp, self.stp, _ptr(self.counts))
        return self.counts

    def fields(self) -> np.ndarray:
        lib().orc_fields(self.sp, _ptr(self.counts), _ptr(self.omega))
        return self.omega

    def set_fields(self, omega: np.ndarray):
        self.omega[...] = np.asarray(omega, dtype=np.float64).reshape(2, -1)

    def energy_nb(self) -> float:
        return lib().orc_energy_nb(self.sp, _ptr(self.counts))

    def sweep(self, seed: int, sweep: int, decisions: bool = False):
        """One move sweep with the current (frozen) fields; no density/field refresh."""
        acc = np.zeros(self.desc.n_beads, np.uint8) if decisions else None
        n = lib().orc_sweep(self.sp, self.stp, seed, sweep, _ptr(self.omega), _ptr(acc))
        return (n, acc) if decisions else n

    def run(self, seed: int, first_sweep: int, n_sweeps: int, refresh: bool = True) -> int:
        return lib().orc_run(self.sp, self.stp, seed, first_sweep, n_sweeps,
                             _ptr(self.counts), _ptr(self.omega), int(refresh))

    def observables(self, per_chain: bool = False):
        o = _Obs()
        pc = np.zeros((3, self.desc.n_chains), np.float64) if per_chain else None
        lib().orc_observables(self.sp, self.stp, _ptr(self.counts), C.byref(o), _ptr(pc))
        d = {f: getattr(o, f) for f, _ in _Obs._fields_}
        if per_chain:
            d["per_chain"] = pc
        return d
