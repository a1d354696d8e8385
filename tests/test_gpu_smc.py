"""Bond-force-biased ("smart") moves on the GPU against the oracle.

Parity: batches that mix smart-move and uniform-move systems, in both
position representations and both density modes, compared with the oracle
bead by bead after each sweep (the Gaussian draws are FP64 Box-Muller on
both sides; the FP32 displacement can differ only when the two math
libraries' last-bit differences straddle an FP32 rounding boundary).
Statistics: the acceptance of N = 2 ideal chains against the numpy estimate,
and the two-bead frozen-field Boltzmann occupancy.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2606_09356_amd import workloads as W
from paper_2606_09356_amd.soma import Soma
from tests.helpers.closed_forms import smart_acceptance_two_beads, two_bead_cell_probabilities
from tests.test_gpu_parity import oracle_density_of_gpu_state, same_state

pytestmark = pytest.mark.gpu
SEED = 20260609


def mixed_batch(seed):
    systems = W.batched_mixed(n_systems=5, seed=seed, bead_range=(2000, 12000))
    for k, s in enumerate(systems):
        if k != 1:
            s.smc_A = 0.002 if k % 2 == 0 else 0.0004
    return systems


@pytest.mark.parametrize("r,cw,dm,pk", [("f32", 16, 0, 0), ("f32", 16, 1, 0), ("f32", 16, 2, 0), ("cell", 32, 0, 0),
                                        ("cell", 16, 1, 0), ("cell", 16, 2, 0), ("cell", 32, 2, 0), ("f32", 16, 0, 1),
                                        ("cell", 16, 2, 1), ("cell", 16, 3, 0), ("f32", 16, 3, 1)])
def test_smart_move_parity(r, cw, dm, pk):
    systems = mixed_batch(61)
    print(f"[smc parity] {r}/u{cw}/mode {dm}/packed {pk}: {sum(s.n_beads for s in systems)} beads", flush=True)
    g = Soma(systems, seed=SEED, pos_repr=r, count_width=cw, density_mode=dm, reorder_every=2, packed_tiles=pk,
             waves_per_block=5 if pk else 0)
    mode = oracle.MODE_F32 if r == "f32" else oracle.MODE_CELL
    orcs = []
    for k, s in enumerate(systems):
        xyz = W.gaussian_walks(s, seed=70 + k)
        g.set_positions(k, xyz)
        o = oracle.OracleSystem(s, sys_id=k, mode=mode)
        o.set_positions(xyz)
        orcs.append(o)
    total, mism = 0, 0
    for sweep in range(3):
        g.sweep(1)
        for k, o in enumerate(orcs):
            o.sweep(SEED, sweep)
            o.density()
            o.fields()
            eq = same_state(g, k, o)
            total += eq.size
            mism += int((~eq).sum())
            assert (g.density(k) == oracle_density_of_gpu_state(g, k, o)).all()
            if eq.all():
                assert (g.density(k) == o.counts).all()
    acc = [g.observables(k)["accept_ratio"] for k in range(len(systems))]
    print(f"[smc parity] {mism} differing beads of {total}; acceptance {np.round(acc, 4)}", flush=True)
    assert mism <= max(1, int(1e-6 * total)), (mism, total)
    g.close()


def test_smart_acceptance_two_beads_on_gpu():
    A, box, grid = 0.05, 8.0, 8
    s = W.diblock_system(65536, 2, 0.5, 0.0, 0.0, (box, box, box), (grid, grid, grid))
    s.smc_A = A
    g = Soma([s], seed=SEED, pos_repr="f32", count_width=16)
    g.sweep(10)
    ob = g.observables(0)
    expect, se_mc = smart_acceptance_two_beads(A, box / grid)
    se = math.sqrt(expect * (1 - expect) / ob["n_moves"] + se_mc ** 2)
    print(f"[smc acceptance] gpu {ob['accept_ratio']:.5f} estimate {expect:.5f} se {se:.1e}", flush=True)
    assert abs(ob["accept_ratio"] - expect) < 6 * se
    g.close()


def test_smart_two_bead_frozen_field_boltzmann_on_gpu():
    n_chains, L, n = 32768, 1.0, 4
    s = W.SystemDesc(n_chains=n_chains, N=2, pattern_a=np.array([0, 1], np.uint8),
                     pattern_b=np.array([0, 1], np.uint8), n_chains_a=n_chains, chiN=0.0, kappaN=0.0,
                     box=(L, L, L), grid=(n, n, n), smc_A=0.004)
    M = n ** 3
    omega = np.random.default_rng(4).uniform(-1.0, 1.0, size=(2, M)).astype(np.float32)
    g = Soma([s], seed=SEED, pos_repr="cell", count_width=32)
    g.set_fields(0, omega)
    g.sweep(150)
    acc = np.zeros((2, M))
    for _ in range(50):
        g.sweep(5)
        acc += g.density(0)
    P, idx = two_bead_cell_probabilities(omega.astype(np.float64), n, L, 3.0)
    pA, pB = P.sum(axis=1), P.sum(axis=0)
    assert np.abs(acc[0] / acc[0].sum() / pA - 1).max() < 0.06
    assert np.abs(acc[1] / acc[1].sum() / pB - 1).max() < 0.06
    assert 0.5 * np.abs(acc[0] / acc[0].sum() - pA).sum() < 0.012
    g.close()


@pytest.mark.parametrize("shape", ["auto", "dm0", "dm2", "dm3"])
def test_full_size_smart_move_parity(shape):
    """plain_large with smart moves, in the benchmark's configuration (the
    autotuner's choice) and in density modes 0, 2 and 3: every decision of two
    sweeps compared with the oracle, density bit-exact."""
    systems = W.workload("plain_large_smc")
    s = systems[0]
    print(f"[full-size] plain_large_smc ({shape}): {s.n_beads} beads", flush=True)
    xyz = W.gaussian_walks(s, seed=11)
    dm = int(shape[2]) if shape.startswith("dm") else 0
    g = Soma(systems, seed=SEED, pos_repr="f32", count_width=16, density_mode=dm,
             reorder_every=W.WORKLOAD_OPTIONS["plain_large_smc"]["reorder_every"])
    if shape == "auto":
        print(f"[shape] autotuned: {g.autotune(2)}", flush=True)
    g.set_positions(0, xyz)
    o = oracle.OracleSystem(s, sys_id=0, mode=oracle.MODE_F32)
    o.set_positions(xyz)
    del xyz
    total, mism = 0, 0
    for sweep in range(2):
        g.sweep(1)
        o.sweep(SEED, sweep)
        eq = same_state(g, 0, o)
        total += eq.size
        mism += int((~eq).sum())
        assert (g.density(0) == oracle_density_of_gpu_state(g, 0, o)).all()
        o.density()
        o.fields()
    print(f"[full-size] plain_large_smc: {mism} differing beads of {total} decisions", flush=True)
    assert mism / total <= 1e-6, (mism, total)
    g.close()
