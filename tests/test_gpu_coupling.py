"""GPU parity of the coupling steps (Sec. 3.2, "Coupling") against the oracle:
placement from target fields, the umbrella potential, walls and the
molecular-type conversion zones, through the C-ABI.

Bars as for the sweep: stored state after the same sweeps compared bead by
bead (mismatch rate at most 1e-6, both sides in the same storage mode), the
density bit-exact from the GPU's own state, chain classes and conversion
counters exact.  Placement and initial walks use FP64 transcendental
functions whose last bits differ between the two libraries, so positions
are compared to 1e-9 Re and the stored values for at least 99.99 % of the
beads (as for the initial walks).
"""
import numpy as np
import pytest

import oracle
from paper_2606_09356_amd import workloads as W
from paper_2606_09356_amd.soma import Soma, SomaError, SOMA_EINVAL
from tests.helpers.closed_forms import two_bead_cell_probabilities_walls

pytestmark = pytest.mark.gpu
SEED = 20260609


def omode(r):
    return oracle.MODE_F32 if r == "f32" else oracle.MODE_CELL


def oracle_from_gpu(g, k, desc, r):
    """An oracle system holding exactly the GPU's stored state and classes."""
    o = oracle.OracleSystem(desc, sys_id=k, mode=omode(r))
    st = g.state(k)
    if r == "f32":
        o.xf[...] = st
    else:
        o.off[...], o.cell[...] = st
    o.chain_class[...] = g.classes(k)
    o.density()
    o.fields()
    return o


def same_state(g, k, o, r):
    st = g.state(k)
    if r == "f32":
        return (st == o.xf).all(axis=0)
    return ((st[0] == o.off) & (st[1] == o.cell)).all(axis=0)


def targets_for(s, seed):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, 2.0, size=(2, s.n_cells)).astype(np.float32)
    t[:, rng.random(s.n_cells) < 0.2] = 0.0
    if s.walls:
        iz = np.arange(s.n_cells) % s.grid[2]
        t[:, (iz < s.walls[0] + 1) | (iz >= s.walls[1] - 1)] = 0.0
    return t


def coupling_batch():
    a = W.diblock_system(3000, 16, 0.4, 12.0, 40.0, (3.0, 3.0, 3.0), (12, 12, 12), "walls+zones")
    a.pattern_b = W.diblock_pattern(16, 0.7)
    a.n_chains_a = 1800
    a.walls, a.zones = (1, 11), (2, 3)
    b = W.diblock_system(2000, 9, 0.5, 20.0, 50.0, (2.5, 2.5, 2.5), (10, 10, 10), "periodic")
    c = W.SystemDesc(1500, 12, np.zeros(12, np.uint8), np.ones(12, np.uint8), 700, 8.0, 30.0,
                     (2.25, 2.25, 2.25), (9, 9, 9), label="blend with walls")
    c.walls = (0, 9)
    return [a, b, c]


@pytest.mark.parametrize("r", ["f32", "cell"])
def test_initial_walks_with_walls_match_oracle(r):
    systems = coupling_batch()
    g = Soma(systems, seed=SEED, pos_repr=r, count_width=16)
    for k, s in enumerate(systems):
        o = oracle.OracleSystem(s, sys_id=k, mode=omode(r))
        o.set_positions(o.init_walks(SEED))
        eq = same_state(g, k, o, r)
        assert eq.mean() > 0.9999, (k, eq.mean())
        assert np.abs(g.positions(k) - o.positions()).max() < 1e-5
        if s.walls:
            e = s.box[2] / s.grid[2]
            z = g.positions(k)[2]
            assert (z >= s.walls[0] * e).all() and (z < s.walls[1] * e).all()
    g.close()


@pytest.mark.parametrize("r", ["f32", "cell"])
def test_placement_matches_oracle(r):
    systems = coupling_batch()
    g = Soma(systems, seed=SEED, pos_repr=r, count_width=16, coupling=True)
    for k, s in enumerate(systems):
        t = targets_for(s, 30 + k)
        g.place_from_fields(k, t)
        o = oracle.OracleSystem(s, sys_id=k, mode=omode(r))
        o.set_target(t.astype(np.float64))
        xyz, _, _ = o.place_from_fields(SEED)
        o.set_positions(xyz)
        eq = same_state(g, k, o, r)
        print(f"[placement {r}] system {k}: {eq.mean():.6f} of stored beads equal", flush=True)
        assert eq.mean() > 0.9999, (k, eq.mean())
        assert np.abs(g.positions(k) - xyz).max() < 1e-5
        t2 = oracle_from_gpu(g, k, s, r)
        assert (g.density(k) == t2.counts).all()
    g.close()


def test_placement_errors():
    systems = coupling_batch()
    g = Soma(systems, seed=SEED, pos_repr="f32", count_width=16)
    with pytest.raises(SomaError) as e:                 # no coupling workspace
        g.place_from_fields(0, targets_for(systems[0], 1))
    assert e.value.code == SOMA_EINVAL
    g.close()
    g = Soma(systems, seed=SEED, pos_repr="f32", count_width=16, coupling=True)
    t = targets_for(systems[2], 2)
    t[1] = 0.0                                          # the B homopolymers have no weight
    with pytest.raises(SomaError) as e:
        g.place_from_fields(2, t)
    assert e.value.code == SOMA_EINVAL
    bad = targets_for(systems[1], 3)
    bad[0, 5] = -1.0
    with pytest.raises(SomaError):
        g.place_from_fields(1, bad)
    with pytest.raises(SomaError):                      # umbrella without targets
        g.set_umbrella(1, 5.0)
    g.close()


@pytest.mark.parametrize("r,cw,dm", [("f32", 16, 0), ("cell", 32, 1), ("cell", 16, 0), ("cell", 16, 3)])
def test_umbrella_and_walls_sweep_parity(r, cw, dm):
    systems = coupling_batch()
    g = Soma(systems, seed=SEED, pos_repr=r, count_width=cw, density_mode=dm, coupling=True, reorder_every=2)
    lam = [25.0, 10.0, 0.0]
    targets = []
    for k, s in enumerate(systems):
        t = targets_for(s, 50 + k)
        targets.append(t)
        g.place_from_fields(k, t)
        g.set_umbrella(k, lam[k])
    orcs = []
    for k, s in enumerate(systems):
        o = oracle_from_gpu(g, k, s, r)
        o.set_target(targets[k].astype(np.float64))
        o.set_umbrella(lam[k])
        o.fields()
        # fields and energy with the umbrella, from identical counts
        wg = g.fields(k).astype(np.float64)
        assert np.abs(wg - o.omega).max() <= 4e-6 * max(1.0, np.abs(o.omega).max()), k
        assert g.observables(k)["Enb_per_chain"] == pytest.approx(o.observables()["Enb_per_chain"], rel=1e-11)
        orcs.append(o)
    total = mism = 0
    for sweep in range(3):
        g.sweep(1)
        for k, o in enumerate(orcs):
            o.sweep(SEED, sweep)
            o.density()
            o.fields()
            eq = same_state(g, k, o, r)
            total += eq.size
            mism += int((~eq).sum())
            assert (g.classes(k) == o.chain_class).all(), (sweep, k)
            ob = g.observables(k)
            assert (ob["converted_to_a"], ob["converted_to_b"]) == o.conversions, (sweep, k)
            assert (g.density(k) == oracle_from_gpu(g, k, systems[k], r).counts).all()
            if eq.all():
                assert (g.density(k) == o.counts).all()
    print(f"[umbrella/walls {r}/u{cw}/dm{dm}] {mism} differing beads of {total}; conversions "
          f"{orcs[0].conversions}", flush=True)
    assert mism <= max(1, int(1e-6 * total)), (mism, total)
    assert sum(orcs[0].conversions) > 0
    g.close()


@pytest.mark.parametrize("r,dm", [("f32", 0), ("cell", 1), ("f32", 3)])
def test_zones_with_smart_moves_parity(r, dm):
    systems = coupling_batch()
    systems[0].smc_A = 0.002
    g = Soma(systems, seed=SEED, pos_repr=r, count_width=16, density_mode=dm)
    orcs = [oracle_from_gpu(g, k, s, r) for k, s in enumerate(systems)]
    total = mism = 0
    for sweep in range(4):
        g.sweep(1)
        for k, o in enumerate(orcs):
            o.sweep(SEED, sweep)
            o.density()
            o.fields()
            eq = same_state(g, k, o, r)
            total += eq.size
            mism += int((~eq).sum())
            assert (g.classes(k) == o.chain_class).all(), (sweep, k)
    assert mism <= max(1, int(1e-6 * total)), (mism, total)
    g.close()


def test_zones_long_run_invariants_and_checkpoint():
    systems = coupling_batch()
    a = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, density_mode=1, reorder_every=5)
    a.sweep(40)
    b = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, density_mode=0, reorder_every=5)
    b.sweep(20)
    saved = [(b.state(k), b.classes(k)) for k in range(len(systems))]
    b.close()
    c = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, density_mode=1, reorder_every=5)
    for k, ((f, cl), cls) in enumerate(saved):
        c.set_state(k, f, cl)
        c.set_classes(k, cls)
    c.set_sweep(20)
    c.sweep(20)
    for k, s in enumerate(systems):
        fa, ca = a.state(k)
        fc, cc = c.state(k)
        assert (fa == fc).all() and (ca == cc).all(), k
        assert (a.classes(k) == c.classes(k)).all(), k
        assert (a.density(k) == c.density(k)).all(), k
        d = a.density(k)
        assert d.sum() == s.n_beads
        if s.walls:
            iz = np.arange(s.n_cells) % s.grid[2]
            assert d[:, (iz < s.walls[0]) | (iz >= s.walls[1])].sum() == 0
    ob = a.observables(0)
    cls0 = (np.arange(systems[0].n_chains) >= systems[0].n_chains_a).astype(int)
    assert ob["converted_to_b"] - ob["converted_to_a"] == int(a.classes(0).sum()) - int(cls0.sum())
    a.close()
    c.close()


def test_positions_outside_walls_rejected():
    systems = coupling_batch()
    g = Soma(systems, seed=SEED, pos_repr="f32", count_width=16)
    xyz = g.positions(0)
    xyz[2, 7] = 0.05                                   # below the wall at z cell 1 (edge 0.25)
    with pytest.raises(SomaError) as e:
        g.set_positions(0, xyz)
    assert e.value.code == SOMA_EINVAL
    g.close()


def test_autotune_with_zones_keeps_trajectory():
    from paper_2606_09356_amd.soma import tune_cache_clear
    systems = coupling_batch()
    tune_cache_clear()
    a = Soma(systems, seed=SEED, pos_repr="f32", count_width=16)
    b = Soma(systems, seed=SEED, pos_repr="f32", count_width=16)
    a.sweep(3)
    b.sweep(3)
    t = a.autotune(2)
    assert t["density_mode"] != 2 and t["n_candidates"] == 90
    a.sweep(4)
    b.sweep(4)
    for k in range(len(systems)):
        assert (a.state(k) == b.state(k)).all()
        assert (a.classes(k) == b.classes(k)).all()
        assert a.observables(k)["converted_to_a"] == b.observables(k)["converted_to_a"]
    a.close()
    b.close()


def test_two_bead_boltzmann_with_walls_on_gpu():
    n_chains, L, n, lo, hi = 32768, 1.0, 4, 1, 4
    s = W.SystemDesc(n_chains=n_chains, N=2, pattern_a=np.array([0, 1], np.uint8),
                     pattern_b=np.array([0, 1], np.uint8), n_chains_a=n_chains, chiN=0.0, kappaN=0.0,
                     box=(L, L, L), grid=(n, n, n), move_halfwidth=0.2)
    s.walls = (lo, hi)
    M = n ** 3
    omega = np.random.default_rng(6).uniform(-1.0, 1.0, size=(2, M)).astype(np.float32)
    g = Soma([s], seed=SEED, pos_repr="cell", count_width=32)
    g.set_fields(0, omega)
    g.sweep(150)
    acc = np.zeros((2, M))
    for _ in range(50):
        g.sweep(5)
        acc += g.density(0)
    P, idx = two_bead_cell_probabilities_walls(omega.astype(np.float64), n, L, 3.0, lo, hi)
    inside = (idx[2] >= lo) & (idx[2] < hi)
    assert acc[:, ~inside].sum() == 0
    pA = P.sum(axis=1)
    oa = acc[0] / acc[0].sum()
    assert np.abs(oa[inside] / pA[inside] - 1).max() < 0.06
    assert 0.5 * np.abs(oa - pA).sum() < 0.012
    g.close()
