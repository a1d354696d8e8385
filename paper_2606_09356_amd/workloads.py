"""Seeded synthetic workloads for the SCMF Monte-Carlo sweep.

This module only draws inputs: system descriptors (chain counts, chain
length, block pattern, chiN, kappaN, box and grid) and, for tests, bead
positions as Gaussian random walks.  It holds none of the sweep's
arithmetic, so both the GPU path and the CPU oracle can consume it.

The paper states the model in words only (Sec. 2, SOMA paragraph: soft
coarse-grained polymers, single-chain-in-mean-field propagation); it prints
no system sizes for its SOMA runs.  The five workloads below are synthetic
stand-ins at 128 beads per Re^3 with a grid cell of Re/4:

  plain_small    256 AB diblocks, N=32, f=0.5, chiN=20, kappaN=50, 4^3 box, 16^3 grid
  plain_large    131072 AB diblocks, N=32, 32^3 box, 128^3 grid
  mixed_large    262144 AB diblocks, N=64, chiN=30, 64x64x32 box, 256x256x128 grid
  batched_uneven 64 diblock systems, chains ~U{512..16384}, N in {16,32,64},
                 f ~U[0.3,0.7], chiN ~U[10,40], kappaN=50
  batched_mixed  256 systems mixing A/B blends, AB diblocks and ABA triblocks,
                 N ~U{8..128}, beads ~U[1e4,1e6], chiN ~U[0,50], kappaN ~U[25,100]
  plain_large_smc  plain_large with bond-force-biased (smart) moves, A = 4e-4 Re^2
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

TYPE_A = 0
TYPE_B = 1

WORKLOAD_NAMES = ("plain_small", "plain_large", "mixed_large",
                  "batched_uneven", "batched_mixed", "plain_large_smc")
BASE_SEED = 20260609


@dataclasses.dataclass
class SystemDesc:
    """One independent polymer system.

    Chains ``[0, n_chains_a)`` carry bead types ``pattern_a``; the remaining
    chains carry ``pattern_b``.  A diblock or triblock melt has
    ``n_chains_a == n_chains``; an A/B homopolymer blend has an all-A
    ``pattern_a`` and an all-B ``pattern_b``.
    """
    n_chains: int
    N: int
    pattern_a: np.ndarray          # uint8 [N], 0 = A, 1 = B
    pattern_b: np.ndarray          # uint8 [N]
    n_chains_a: int
    chiN: float
    kappaN: float
    box: tuple                     # (Lx, Ly, Lz) in Re
    grid: tuple                    # (nx, ny, nz)
    Re: float = 1.0
    move_halfwidth: float = 0.05   # half-width of the uniform trial cube, in Re
    ham_form: int = 0              # 0: Helfand form, 1: chiN*phiA*phiB form
    label: str = ""
    smc_A: float = 0.0             # > 0: bond-force-biased moves with this A (Re^2); 0: uniform moves
    walls: Optional[tuple] = None  # (lo, hi): hard walls at these z-cell faces; None: periodic z
    zones: Optional[tuple] = None  # (lower, upper): z-cell widths of the conversion zones at the walls

    @property
    def n_beads(self) -> int:
        return self.n_chains * self.N

    @property
    def n_cells(self) -> int:
        return int(self.grid[0]) * int(self.grid[1]) * int(self.grid[2])

    def bead_types(self) -> np.ndarray:
        """Per-bead types, chain-major, as uint8 [n_chains * N]."""
        t = np.empty((self.n_chains, self.N), dtype=np.uint8)
        t[: self.n_chains_a] = self.pattern_a
        t[self.n_chains_a:] = self.pattern_b
        return t.reshape(-1)


def _round_half_up(v: float) -> int:
    return int(math.floor(v + 0.5))


def diblock_pattern(N: int, f: float) -> np.ndarray:
    n_a = min(max(_round_half_up(f * N), 1), N - 1) if N > 1 else 1
    p = np.full(N, TYPE_B, dtype=np.uint8)
    p[:n_a] = TYPE_A
    return p


def triblock_pattern(N: int, f: float) -> np.ndarray:
    """Symmetric ABA: the A beads are split over both ends."""
    n_a = min(max(_round_half_up(f * N), 2), N - 1) if N > 2 else 1
    left = n_a // 2
    right = n_a - left
    p = np.full(N, TYPE_B, dtype=np.uint8)
    p[:left] = TYPE_A
    if right:
        p[N - right:] = TYPE_A
    return p


def diblock_system(n_chains, N, f, chiN, kappaN, box, grid, label="", **kw) -> SystemDesc:
    pat = diblock_pattern(N, f)
    return SystemDesc(n_chains=int(n_chains), N=int(N), pattern_a=pat, pattern_b=pat.copy(),
                      n_chains_a=int(n_chains), chiN=float(chiN), kappaN=float(kappaN),
                      box=tuple(float(b) for b in box), grid=tuple(int(g) for g in grid),
                      label=label, **kw)


def cubic_box_for(n_beads: int, rho=128.0, cells_per_re=4):
    """Cubic box at bead density ``rho`` per Re^3 with cell Re/cells_per_re."""
    n = max(1, int(round(cells_per_re * (n_beads / rho) ** (1.0 / 3.0))))
    L = n / cells_per_re
    return (L, L, L), (n, n, n)


def plain_small() -> List[SystemDesc]:
    return [diblock_system(256, 32, 0.5, 20.0, 50.0, (4, 4, 4), (16, 16, 16), "plain_small")]


def plain_large() -> List[SystemDesc]:
    return [diblock_system(131072, 32, 0.5, 20.0, 50.0, (32, 32, 32), (128, 128, 128), "plain_large")]


def mixed_large() -> List[SystemDesc]:
    return [diblock_system(262144, 64, 0.5, 30.0, 50.0, (64, 64, 32), (256, 256, 128), "mixed_large")]


def plain_large_smc() -> List[SystemDesc]:
    """plain_large with bond-force-biased moves, A = 4e-4 Re^2: the Gaussian
    part of the displacement has the rms per axis of the uniform cube."""
    s = plain_large()[0]
    s.smc_A = 4.0e-4
    s.label = "plain_large_smc"
    return [s]


def batched_uneven(n_systems: int = 64, seed: Optional[int] = None,
                   chain_range=(512, 16384)) -> List[SystemDesc]:
    rng = np.random.default_rng(BASE_SEED + 4 if seed is None else seed)
    out = []
    for k in range(n_systems):
        n_chains = int(rng.integers(chain_range[0], chain_range[1] + 1))
        N = int(rng.choice([16, 32, 64]))
        f = float(rng.uniform(0.3, 0.7))
        chiN = float(rng.uniform(10.0, 40.0))
        box, grid = cubic_box_for(n_chains * N)
        out.append(diblock_system(n_chains, N, f, chiN, 50.0, box, grid, f"batched_uneven[{k}]"))
    return out


def batched_mixed(n_systems: int = 256, seed: Optional[int] = None,
                  bead_range=(1.0e4, 1.0e6)) -> List[SystemDesc]:
    rng = np.random.default_rng(BASE_SEED + 5 if seed is None else seed)
    out = []
    for k in range(n_systems):
        arch = int(rng.integers(0, 3))            # 0 blend, 1 AB, 2 ABA
        N = int(rng.integers(8, 129))
        n_beads = float(rng.uniform(*bead_range))
        n_chains = max(1, int(round(n_beads / N)))
        chiN = float(rng.uniform(0.0, 50.0))
        kappaN = float(rng.uniform(25.0, 100.0))
        box, grid = cubic_box_for(n_chains * N)
        label = f"batched_mixed[{k}]"
        if arch == 0:
            phi_a = float(rng.uniform(0.2, 0.8))
            pa = np.full(N, TYPE_A, dtype=np.uint8)
            pb = np.full(N, TYPE_B, dtype=np.uint8)
            out.append(SystemDesc(n_chains, N, pa, pb, int(round(phi_a * n_chains)), chiN, kappaN,
                                  box, grid, label=label + ":blend"))
        else:
            f = float(rng.uniform(0.3, 0.7))
            pat = diblock_pattern(N, f) if arch == 1 else triblock_pattern(N, f)
            out.append(SystemDesc(n_chains, N, pat, pat.copy(), n_chains, chiN, kappaN, box, grid,
                                  label=label + (":AB" if arch == 1 else ":ABA")))
    return out


def workload(name: str, **kw) -> List[SystemDesc]:
    return {"plain_small": plain_small, "plain_large": plain_large, "mixed_large": mixed_large,
            "batched_uneven": batched_uneven, "batched_mixed": batched_mixed,
            "plain_large_smc": plain_large_smc}[name](**kw)


# Options per workload: position representation and count width.
WORKLOAD_OPTIONS = {
    "plain_small": dict(pos_repr="f32", count_width=16, sweeps=1000, reorder_every=100),
    "plain_large": dict(pos_repr="f32", count_width=16, sweeps=200, reorder_every=100),
    "mixed_large": dict(pos_repr="cell", count_width=32, sweeps=100, reorder_every=100),
    "batched_uneven": dict(pos_repr="f32", count_width=16, sweeps=500, reorder_every=100),
    "batched_mixed": dict(pos_repr="cell", count_width=16, sweeps=200, reorder_every=100),
    "plain_large_smc": dict(pos_repr="f32", count_width=16, sweeps=200, reorder_every=100),
}


def gaussian_walks(sys: SystemDesc, seed: int) -> np.ndarray:
    """Gaussian random-walk chains, FP64, shape [3, n_chains * N] (unwrapped).

    The first bead of each chain is uniform in the box; each bond component
    is N(0, Re^2 / (3 (N - 1))).  Used as a common starting state for the
    GPU path and the oracle in tests.
    """
    rng = np.random.default_rng(seed)
    box = np.asarray(sys.box, dtype=np.float64)
    start = rng.uniform(0.0, 1.0, size=(sys.n_chains, 3)) * box
    sigma = sys.Re / math.sqrt(3.0 * max(sys.N - 1, 1))
    bonds = rng.normal(0.0, sigma, size=(sys.n_chains, sys.N - 1, 3))
    pos = np.empty((sys.n_chains, sys.N, 3), dtype=np.float64)
    pos[:, 0] = start
    if sys.N > 1:
        pos[:, 1:] = start[:, None, :] + np.cumsum(bonds, axis=1)
    return np.ascontiguousarray(pos.reshape(-1, 3).T)
