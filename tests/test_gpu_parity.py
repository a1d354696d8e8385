"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Bars (from the task's definition of the hot path):
  * density histogram from identical positions: bit-exact;
  * one sweep from identical stored state under the shared Philox stream:
    fraction of beads whose stored state differs (a decision mismatch) at
    most 1e-6 -- the oracle runs in the storage mode of the GPU
    representation (FP32 positions, or int32 cell + FP32 offset) with FP64
    energies, so a mismatch can only come from FP32 energy rounding near
    u = exp(-dE);
  * observables from identical positions: FP64 compensated sums, relative
    difference below 1e-12 (rounding order only).
Small cases span many wave tiles and ragged tails (odd N, partial tiles,
N up to 128, blends, triblocks); full-size cases run the workloads the
benchmark times, in its launch configuration.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2606_09356_amd import workloads as W
from paper_2606_09356_amd.soma import Soma, SomaError, SOMA_EOVERFLOW, SOMA_ESTATE, SOMA_ENONFINITE, tune_cache_clear
from tests.helpers.closed_forms import acceptance_closed_form, two_bead_cell_probabilities

pytestmark = pytest.mark.gpu
SEED = 20260609


def small_cases():
    return {
        "plain_small/f32/u16": (W.plain_small(), "f32", 16),
        "plain_small/cell/u32": (W.plain_small(), "cell", 32),
        "batched_uneven_small/f32/u16": (W.batched_uneven(n_systems=6, seed=41, chain_range=(60, 700)), "f32", 16),
        "batched_mixed_small/cell/u16": (W.batched_mixed(n_systems=10, seed=42, bead_range=(2000, 20000)), "cell", 16),
        "batched_mixed_small/f32/u32": (W.batched_mixed(n_systems=5, seed=43, bead_range=(3000, 9000)), "f32", 32),
        # 16384 beads in 8 cells: every wave's density updates hit a handful of
        # count words, the worst case for the per-wave merge of the delta
        "crowded/f32/u16": ([crowded()], "f32", 16),
        "crowded/cell/u32": ([crowded()], "cell", 32),
        # cell edge just above the move half-width: almost every accepted move
        # changes cell, so a wave's merge table holds up to 256 distinct words
        "fine_grid/f32/u16": ([fine_grid()], "f32", 16),
        "fine_grid/cell/u16": ([fine_grid()], "cell", 16),
    }


def fine_grid():
    return W.diblock_system(1024, 32, 0.5, 20.0, 50.0, (1.275, 1.275, 1.275), (25, 25, 25), "fine_grid")


def crowded():
    return W.diblock_system(512, 32, 0.5, 20.0, 50.0, (0.5, 0.5, 0.5), (2, 2, 2), "crowded")


def make_pair(systems, pos_repr, cw, pos_seed=7, **kw):
    print(f"[case] {len(systems)} systems, {sum(s.n_beads for s in systems)} beads, {pos_repr}/u{cw}", flush=True)
    g = Soma(systems, seed=SEED, pos_repr=pos_repr, count_width=cw, **kw)
    mode = oracle.MODE_F32 if pos_repr == "f32" else oracle.MODE_CELL
    orcs = []
    for k, s in enumerate(systems):
        xyz = W.gaussian_walks(s, seed=pos_seed + k)
        g.set_positions(k, xyz)
        o = oracle.OracleSystem(s, sys_id=k, mode=mode)
        o.set_positions(xyz)
        orcs.append(o)
    return g, orcs


def same_state(g, k, o):
    """Per-bead boolean: stored GPU state equals the oracle's stored state."""
    if o.mode == oracle.MODE_F32:
        return (g.state(k) == o.xf).all(axis=0)
    f, c = g.state(k)
    return ((f == o.off) & (c == o.cell)).all(axis=0)


def oracle_density_of_gpu_state(g, k, o):
    s = o.desc
    t = oracle.OracleSystem(s, sys_id=k, mode=o.mode)
    if o.mode == oracle.MODE_F32:
        t.xf[...] = g.state(k)
    else:
        f, c = g.state(k)
        t.off[...] = f
        t.cell[...] = c
    return t.density().copy()


@pytest.mark.parametrize("name", list(small_cases()))
def test_density_bit_exact_from_identical_positions(name):
    systems, r, cw = small_cases()[name]
    g, orcs = make_pair(systems, r, cw)
    for k, o in enumerate(orcs):
        assert (g.density(k) == o.counts).all(), (name, k)
    g.close()


def test_density_faces_negative_and_images():
    s = W.diblock_system(64, 32, 0.5, 20.0, 50.0, (4, 4, 4), (16, 16, 16))
    rng = np.random.default_rng(3)
    xyz = W.gaussian_walks(s, seed=2)
    # beads exactly on cell faces, at L - ulp, at negative unwrapped coordinates, far images
    xyz[:, :200] = rng.integers(-40, 40, size=(3, 200)) * 0.25
    xyz[:, 200:210] = np.nextafter(np.float32(4.0), np.float32(0.0))
    xyz[:, 210:400] -= 12.0
    xyz[:, 400:600] += 40.0
    for r, cw in [("f32", 16), ("cell", 32)]:
        g = Soma([s], seed=1, pos_repr=r, count_width=cw)
        g.set_positions(0, xyz)
        o = oracle.OracleSystem(s, mode=oracle.MODE_F32 if r == "f32" else oracle.MODE_CELL)
        o.set_positions(xyz)
        assert (g.density(0) == o.counts).all(), r
        assert g.density(0).sum() == s.n_beads
        g.close()


@pytest.mark.parametrize("name", list(small_cases()))
def test_fields_match_oracle(name):
    systems, r, cw = small_cases()[name]
    g, orcs = make_pair(systems, r, cw)
    for k, o in enumerate(orcs):
        wg = g.fields(k).astype(np.float64)
        wo = o.omega
        scale = max(1.0, np.abs(wo).max())
        # FP32 coefficients and two FMAs: a few FP32 ulps of the largest term
        assert np.abs(wg - wo).max() <= 4e-6 * scale, (name, k, np.abs(wg - wo).max())
    g.close()


@pytest.mark.parametrize("reorder,dm,pk", [(0, 0, 0), (1, 0, 0), (0, 2, 0), (1, 1, 0), (0, 0, 1), (1, 2, 1),
                                           (0, 3, 0), (1, 3, 1), (1, 3, 2), (0, 2, 2), (1, 1, 2)])
@pytest.mark.parametrize("name", list(small_cases()))
def test_single_and_multi_sweep_parity(name, reorder, dm, pk):
    systems, r, cw = small_cases()[name]
    g, orcs = make_pair(systems, r, cw, reorder_every=reorder, density_mode=dm, packed_tiles=pk,
                        waves_per_block=3 if pk else 0)
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
            # the density is bit-exact from the GPU's own positions in every case
            assert (g.density(k) == oracle_density_of_gpu_state(g, k, o)).all()
            if eq.all():
                assert (g.density(k) == o.counts).all()
    print(f"[{name}] {mism} differing beads of {total}")
    assert mism <= max(1, int(1e-6 * total)), (mism, total)
    g.close()


def stream_systems():
    """Chains that cross wave boundaries in stream tiles: P = ceil(N/2) lanes
    per chain does not divide 64 (odd and even N, 33..63 lanes, and short
    chains), with chiN > 0 so the field term decides moves too."""
    out = []
    for k, (N, nch) in enumerate([(67, 300), (100, 200), (125, 160), (9, 2000), (2, 5000), (41, 500)]):
        box = round((N * nch / 128.0) ** (1.0 / 3.0) * 4) / 4
        n = int(box * 4)
        out.append(W.diblock_system(nch, N, 0.4 + 0.05 * k, 15.0 + 3 * k, 50.0, (box, box, box), (n, n, n), f"stream{k}"))
    return out


@pytest.mark.parametrize("r,cw,dm", [("cell", 16, 3), ("f32", 16, 0), ("cell", 32, 1), ("f32", 16, 2)])
def test_stream_tile_parity(r, cw, dm):
    """Stream tiles: every decision of three sweeps equals the oracle's and
    the density is bit-exact, on chains that cross wave boundaries (the
    wave repeats the even move of the bead after its last lane); the same
    context in wave tiles runs the identical trajectory."""
    systems = stream_systems()
    g, orcs = make_pair(systems, r, cw, density_mode=dm, packed_tiles=2, waves_per_block=4)
    assert g.info()["packed_tiles"] == 2
    h = Soma(systems, seed=SEED, pos_repr=r, count_width=cw, density_mode=dm)
    for k, s in enumerate(systems):
        h.set_positions(k, W.gaussian_walks(s, seed=7 + k))
    total = mism = 0
    for sweep in range(3):
        g.sweep(1)
        h.sweep(1)
        for k, o in enumerate(orcs):
            o.sweep(SEED, sweep)
            o.density()
            o.fields()
            eq = same_state(g, k, o)
            total += eq.size
            mism += int((~eq).sum())
            assert (g.density(k) == oracle_density_of_gpu_state(g, k, o)).all()
            assert _same_state(g.state(k), h.state(k)), (k, sweep)
    print(f"[stream {r}/u{cw}/dm{dm}] {mism} differing beads of {total}")
    assert mism <= max(1, int(1e-6 * total)), (mism, total)
    for k in range(len(systems)):
        assert g.observables(k)["n_accepted"] == h.observables(k)["n_accepted"]
    g.close()
    h.close()


@pytest.mark.parametrize("name,n_sys,dm", [("batched_mixed", 24, 3), ("batched_uneven", 64, 1)])
def test_stream_tiles_match_wave_tiles_at_scale(name, n_sys, dm):
    """Stream tiles on a batch of millions of beads, where the waves of one
    sweep run far apart in time: the overlap lanes read the pairs of their
    neighbouring tiles from the copy taken before the sweep, never from
    pairs the owning wave has already rewritten, so 30 sweeps (two calls,
    a chain reorder every 10 sweeps) leave every system's state, density and
    acceptance count bit-identical to wave tiles, on repeated runs too."""
    systems = W.workload(name)[:n_sys]
    opts = W.WORKLOAD_OPTIONS[name]
    r, cw = opts["pos_repr"], opts["count_width"]
    print(f"[stream at scale] {name}: {len(systems)} systems, {sum(s.n_beads for s in systems)} beads, dm {dm}",
          flush=True)
    h = Soma(systems, seed=SEED, pos_repr=r, count_width=cw, reorder_every=10)
    h.sweep(30)
    for run in range(2):
        g = Soma(systems, seed=SEED, pos_repr=r, count_width=cw, reorder_every=10, density_mode=dm, packed_tiles=2,
                 waves_per_block=4)
        assert g.info()["packed_tiles"] == 2
        g.sweep(12)
        g.sweep(18)
        bad = [k for k in range(len(systems)) if not _same_state(g.state(k), h.state(k))]
        print(f"[stream at scale] run {run}: {len(bad)} of {len(systems)} systems differ from wave tiles", flush=True)
        assert not bad, bad[:8]
        for k in range(len(systems)):
            assert (g.density(k) == h.density(k)).all(), k
            assert g.observables(k)["n_accepted"] == h.observables(k)["n_accepted"], k
        g.close()
    h.close()


def test_stream_tiles_refresh_the_halo_after_new_positions():
    """The halo copy is refilled when positions change outside a stream-tile
    sweep (set_positions, set_state, set_sweep) and reused between calls
    otherwise: a stream-tile context and a wave-tile context given the same
    new positions mid-run stay bit-identical."""
    systems = stream_systems()
    g = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, density_mode=3, packed_tiles=2, waves_per_block=4)
    h = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, density_mode=3)
    assert g.info()["packed_tiles"] == 2
    for x in (g, h):
        x.sweep(3)
    for k, s in enumerate(systems):
        xyz = W.gaussian_walks(s, seed=99 + k)
        g.set_positions(k, xyz)
        h.set_positions(k, xyz)
    for x in (g, h):
        x.sweep(2)
        x.sweep(2)
    st = h.state(1)
    g.set_state(1, *st)
    h.set_state(1, *st)
    for x in (g, h):
        x.set_sweep(50)
        x.sweep(3)
    for k in range(len(systems)):
        assert _same_state(g.state(k), h.state(k)), k
        assert (g.density(k) == h.density(k)).all(), k
    g.close()
    h.close()


def test_acceptance_counts_across_tilings_and_reads():
    """Wave- and stream-tile sweeps count accepted moves per tile and fold
    them into the per-system counters before the tiling changes or the
    counters are read; block tiles count with device atomics.  Contexts that
    read their observables between sweeps, switch tilings through the
    autotuner and sweep on must count exactly what a block-tile context
    counts over the same trajectory."""
    systems = stream_systems()
    ref = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, density_mode=3, packed_tiles=1,
               waves_per_block=4)
    ref.sweep(9)
    want = [ref.observables(k)["n_accepted"] for k in range(len(systems))]
    assert all(w > 0 for w in want)
    for pk in (0, 2):
        tune_cache_clear()
        g = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, density_mode=3, packed_tiles=pk,
                 waves_per_block=4)
        g.sweep(3)
        mid = [g.observables(k)["n_accepted"] for k in range(len(systems))]
        g.sweep(2)
        t = g.autotune(1)
        g.sweep(4)
        got = [g.observables(k)["n_accepted"] for k in range(len(systems))]
        print(f"[acceptance] start tiling {pk}, tuned to {t['packed_tiles']}: {got[:3]} vs {want[:3]}")
        assert got == want, (pk, t)
        assert all(0 < m < w for m, w in zip(mid, want))
        assert _same_state(g.state(0), ref.state(0))
        g.close()
    ref.close()


def test_stream_tiles_fall_back_with_smart_moves():
    """Stream tiles are asked for but the context moves with smart moves: the
    shape reports wave tiles and the sweep matches a wave-tile context."""
    systems = stream_systems()[:2]
    systems[0].smc_A = 0.001
    g = Soma(systems, seed=SEED, pos_repr="f32", count_width=16, packed_tiles=2)
    h = Soma(systems, seed=SEED, pos_repr="f32", count_width=16)
    assert g.info()["packed_tiles"] == 0
    g.sweep(2)
    h.sweep(2)
    for k in range(len(systems)):
        assert _same_state(g.state(k), h.state(k))
    g.close()
    h.close()


def test_zero_sweeps_change_nothing_and_negative_counts_are_rejected():
    """soma_mc_sweep(0) is a no-op in every tiling (state, density, sweep
    and move counters unchanged); a negative count is SOMA_EINVAL."""
    systems = stream_systems()[:3]
    for pk in (0, 1, 2):
        g = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, density_mode=3, packed_tiles=pk,
                 waves_per_block=4)
        g.sweep(2)
        before = [(g.state(k), g.density(k), g.observables(k)) for k in range(len(systems))]
        g.sweep(0)
        for k, (st, dens, ob) in enumerate(before):
            assert _same_state(g.state(k), st) and (g.density(k) == dens).all()
            after = g.observables(k)
            assert (after["sweep"], after["n_moves"], after["n_accepted"]) == (ob["sweep"], ob["n_moves"],
                                                                             ob["n_accepted"])
        with pytest.raises(SomaError):
            g.sweep(-1)
        g.close()


def test_accept_counter_matches_oracle():
    systems = W.batched_uneven(n_systems=4, seed=44, chain_range=(100, 400))
    g, orcs = make_pair(systems, "f32", 16)
    g.sweep(1)
    for k, o in enumerate(orcs):
        n = o.sweep(SEED, 0)
        ob = g.observables(k)
        assert ob["n_moves"] == systems[k].n_beads
        assert abs(int(ob["n_accepted"]) - int(n)) <= 1
    g.close()


@pytest.mark.parametrize("name", list(small_cases()))
def test_observables_match_oracle(name):
    systems, r, cw = small_cases()[name]
    g, orcs = make_pair(systems, r, cw)
    g.sweep(2)
    for k, o in enumerate(orcs):
        # oracle evaluated on the GPU's own state and counts
        t = oracle.OracleSystem(o.desc, sys_id=k, mode=o.mode)
        if o.mode == oracle.MODE_F32:
            t.xf[...] = g.state(k)
        else:
            t.off[...], t.cell[...] = g.state(k)
        t.density()
        go, oo = g.observables(k), t.observables()
        for key in ("Re2", "Rg2", "Ebond_per_chain", "Enb_per_chain", "Re2_err", "Rg2_err"):
            assert go[key] == pytest.approx(oo[key], rel=1e-11, abs=1e-12), (name, k, key)
    g.close()


@pytest.mark.parametrize("r", ["f32", "cell"])
def test_gpu_init_matches_oracle_walks(r):
    systems = W.batched_mixed(n_systems=4, seed=45, bead_range=(3000, 30000))
    g = Soma(systems, seed=SEED, pos_repr=r, count_width=16)
    for k, s in enumerate(systems):
        o = oracle.OracleSystem(s, sys_id=k, mode=oracle.MODE_F32 if r == "f32" else oracle.MODE_CELL)
        walks = o.init_walks(SEED)
        o.set_positions(walks)
        eq = same_state(g, k, o)
        # FP64 transcendental functions of the two libraries may differ in the
        # last bit, which changes a stored FP32 value only at a rounding tie
        assert eq.mean() > 0.9999, (k, eq.mean())
        assert np.abs(g.positions(k) - o.positions()).max() < 1e-5
        assert (g.density(k) == oracle_density_of_gpu_state(g, k, o)).all()
    g.close()


def test_graph_tiling_and_xcd_invariance():
    systems = W.batched_mixed(n_systems=6, seed=46, bead_range=(2000, 15000))
    ref = None
    for use_graph, wpb, wpcu, reorder, dm, pk in [
            (False, 1, 0, 0, 0, 0), (True, 4, 0, 0, 0, 0), (True, 16, 0, 0, 0, 0),
            (False, 7, 0, 0, 0, 0), (True, 4, 1, 0, 0, 0), (True, 2, 8, 0, 0, 0),
            (True, 4, 0, 1, 0, 0), (False, 4, 0, 2, 0, 0), (True, 4, 0, 3, 0, 0),
            (True, 4, 0, 0, 1, 0), (False, 1, 0, 2, 1, 0), (True, 2, 8, 3, 1, 0),
            (True, 16, 32, 0, 1, 0), (True, 4, 0, 0, 2, 0), (False, 1, 0, 2, 2, 0),
            (True, 2, 8, 3, 2, 0), (True, 16, 32, 0, 2, 0),
            # block tiles: chains packed over the waves of a workgroup
            (True, 2, 0, 0, 0, 1), (False, 4, 0, 2, 0, 1), (True, 16, 0, 0, 1, 1), (True, 3, 0, 1, 2, 1),
            (True, 8, 0, 0, 2, 1)]:
        g = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, use_graph=use_graph, waves_per_block=wpb,
                 waves_per_cu=wpcu, reorder_every=reorder, density_mode=dm, packed_tiles=pk)
        g.sweep(2)
        g.sweep(3)
        st = [g.state(k) for k in range(len(systems))]
        den = [g.density(k) for k in range(len(systems))]
        if ref is None:
            ref, ref_den = st, den
        else:
            for a, b, da, db in zip(ref, st, ref_den, den):
                assert (a[0] == b[0]).all() and (a[1] == b[1]).all(), (use_graph, wpb, wpcu, reorder, dm, pk)
                assert (da == db).all(), (use_graph, wpb, wpcu, reorder, dm, pk)
        g.close()


def _same_state(x, y):
    if isinstance(x, tuple):
        return all(np.array_equal(a, b) for a, b in zip(x, y))
    return np.array_equal(x, y)


@pytest.mark.parametrize("r", ["f32", "cell"])
def test_autotune_keeps_the_trajectory(r):
    """Autotuning times every launch shape on trial sweeps and undoes them:
    the tuned context then continues exactly like an untuned one."""
    systems = W.batched_mixed(n_systems=4, seed=48, bead_range=(2000, 12000))
    tune_cache_clear()
    a = Soma(systems, seed=SEED, pos_repr=r, count_width=16, reorder_every=3)
    b = Soma(systems, seed=SEED, pos_repr=r, count_width=16, reorder_every=3)
    a.sweep(2)
    b.sweep(2)
    t = a.autotune(trial_sweeps=2)
    print(f"[autotune {r}] {t}", flush=True)
    assert t["n_candidates"] == 192 and 0 < t["us_per_sweep"] and 0 < t["us_per_sweep_before"]
    i = a.info()
    assert (i["waves_per_block"], i["waves_per_cu"], i["xcd_remap"], i["density_mode"], i["packed_tiles"]) == \
        (t["waves_per_block"], t["waves_per_cu"], t["xcd_remap"], t["density_mode"], t["packed_tiles"])
    assert i["sweep"] == 2
    # a second context with the same key takes the cached shape without timing
    c = Soma(systems, seed=SEED, pos_repr=r, count_width=16, reorder_every=3)
    tc = c.autotune(trial_sweeps=2)
    assert tc["from_cache"] == 1 and tc["n_candidates"] == 0
    ic = c.info()
    assert (ic["waves_per_block"], ic["waves_per_cu"], ic["xcd_remap"], ic["density_mode"], ic["packed_tiles"]) == \
        (t["waves_per_block"], t["waves_per_cu"], t["xcd_remap"], t["density_mode"], t["packed_tiles"])
    c.sweep(2)
    c.sweep(5)
    a.sweep(5)
    b.sweep(5)
    for k in range(len(systems)):
        assert _same_state(a.state(k), b.state(k)), k
        assert (a.density(k) == b.density(k)).all(), k
        assert _same_state(c.state(k), b.state(k)), k
        oa, ob = a.observables(k), b.observables(k)
        assert (oa["n_moves"], oa["n_accepted"], oa["sweep"]) == (ob["n_moves"], ob["n_accepted"], ob["sweep"]), k
    a.close()
    b.close()
    c.close()


@pytest.mark.parametrize("dm", [0, 1, 2, 3])
def test_kernel_timing_sweeps_are_real_sweeps(dm):
    """soma_time_kernels runs real sweeps (eager, with events around each
    kernel): the trajectory equals plain sweeps, and the durations are positive."""
    systems = W.batched_mixed(n_systems=4, seed=49, bead_range=(2000, 12000))
    a = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, density_mode=dm, reorder_every=2)
    b = Soma(systems, seed=SEED, pos_repr="cell", count_width=16, density_mode=dm, reorder_every=2)
    a.sweep(1)
    t = a.time_kernels(3)
    a.sweep(1)
    b.sweep(5)
    assert t["n_sweeps"] == 3 and t["density_mode"] == dm and t["sweep_kernel_us"] > 0
    assert (t["fold_kernel_us"] > 0) == (dm != 1)
    for k in range(len(systems)):
        assert _same_state(a.state(k), b.state(k)), k
        assert (a.density(k) == b.density(k)).all(), k
        assert a.observables(k)["n_accepted"] == b.observables(k)["n_accepted"]
    a.close()
    b.close()


def test_batched_equals_each_system_alone():
    systems = W.batched_uneven(n_systems=5, seed=47, chain_range=(64, 500))
    g = Soma(systems, seed=SEED, pos_repr="f32", count_width=16)
    g.sweep(4)
    for k, s in enumerate(systems):
        a = Soma([s], seed=SEED, pos_repr="f32", count_width=16, sys_id_base=k)
        a.sweep(4)
        assert (a.state(0) == g.state(k)).all(), k
        assert (a.density(0) == g.density(k)).all(), k
        a.close()
    g.close()


@pytest.mark.parametrize("r,dm", [("f32", 0), ("cell", 0), ("f32", 1), ("cell", 1), ("f32", 2), ("cell", 2),
                                  ("f32", 3), ("cell", 3)])
def test_checkpoint_resume_bit_exact(r, dm):
    """A checkpoint taken in one density mode resumes bit-exactly in another."""
    systems = W.batched_mixed(n_systems=3, seed=48, bead_range=(2000, 8000))
    a = Soma(systems, seed=SEED, pos_repr=r, count_width=16, density_mode=dm)
    a.sweep(3)
    acc3 = [a.observables(k)["n_accepted"] for k in range(len(systems))]
    a.sweep(3)
    acc6 = [a.observables(k)["n_accepted"] for k in range(len(systems))]
    b = Soma(systems, seed=SEED, pos_repr=r, count_width=16, density_mode=(dm + 1) % 4)
    b.sweep(3)
    saved = [b.state(k) for k in range(len(systems))]
    b.close()
    c = Soma(systems, seed=SEED, pos_repr=r, count_width=16, density_mode=dm)
    for k, st in enumerate(saved):
        if r == "f32":
            c.set_state(k, st)
        else:
            c.set_state(k, st[0], st[1])
    c.set_sweep(3)
    c.sweep(3)
    for k, sysd in enumerate(systems):
        # acceptance counts the three sweeps run on the resumed context
        oc = c.observables(k)
        assert oc["n_moves"] == 3 * sysd.n_beads and oc["sweep"] == 6
        assert oc["n_accepted"] == acc6[k] - acc3[k]
        assert oc["accept_ratio"] == (acc6[k] - acc3[k]) / (3 * sysd.n_beads)
        assert 0.3 < oc["accept_ratio"] < 1.0
    for k in range(len(systems)):
        sa, sc = a.state(k), c.state(k)
        if r == "f32":
            assert (sa == sc).all()
        else:
            assert (sa[0] == sc[0]).all() and (sa[1] == sc[1]).all()
        assert (a.density(k) == c.density(k)).all()
    a.close()
    c.close()


@pytest.mark.parametrize("dm", [0, 1, 2, 3])
def test_count_overflow_in_a_sweep_is_latched(dm):
    """A packed 16-bit count pushed past 65535 by a sweep latches
    SOMA_EOVERFLOW in every density mode, reported by the next call that
    reads the counts (density mode 1 folds a sweep's changes only then).
    65534 A beads sit at the centre of one cell (a move of at most 0.05 Re
    cannot take them out of a 0.25 Re cell) and 1000 two-bead chains sit
    0.001 Re outside its lower x face, so about half of them cross in and the
    count passes 65535."""
    inner, outer = 32767, 1000                 # two-bead chains
    n = inner + outer
    s = W.SystemDesc(n, 2, np.zeros(2, np.uint8), np.zeros(2, np.uint8), n, 0.0, 0.0,
                     (8.0, 8.0, 8.0), (32, 32, 32))
    xyz = np.empty((3, 2 * n))
    xyz[:, : 2 * inner] = 3.125                # centre of cell (12, 12, 12)
    xyz[0, 2 * inner:] = 2.999                 # cell 11, next to the face at x = 3.0
    xyz[1:, 2 * inner:] = 3.125
    g = Soma([s], seed=1, pos_repr="f32", count_width=16, density_mode=dm)
    g.set_positions(0, xyz)
    d = g.density(0)
    assert d[0].max() == 65534 and d[0].sum() == 2 * n
    g.sweep(1)
    with pytest.raises(SomaError) as e:
        g.density(0)
    assert e.value.code == SOMA_EOVERFLOW
    g.close()


def test_count_overflow_is_latched_not_wrapped():
    n_chains, N = 2200, 32                       # 70400 A beads > 65535
    s = W.SystemDesc(n_chains, N, np.zeros(N, np.uint8), np.zeros(N, np.uint8), n_chains, 0.0, 0.0,
                     (8.0, 8.0, 8.0), (32, 32, 32))
    g = Soma([s], seed=1, pos_repr="f32", count_width=16)
    xyz = np.full((3, s.n_beads), 3.1)
    with pytest.raises(SomaError) as e:
        g.set_positions(0, xyz)
    assert e.value.code == SOMA_EOVERFLOW
    with pytest.raises(SomaError) as e:
        g.sweep(1)
    assert e.value.code == SOMA_ESTATE
    g.close()
    # uint32 counts hold it
    g = Soma([s], seed=1, pos_repr="f32", count_width=32)
    g.set_positions(0, xyz)
    d = g.density(0)
    assert d[0].max() == s.n_beads
    g.close()


def test_nonfinite_fields_rejected():
    g = Soma(W.plain_small(), seed=1)
    w = np.zeros((2, 4096), np.float32)
    w[1, 17] = np.nan
    with pytest.raises(SomaError) as e:
        g.set_fields(0, w)
    assert e.value.code == SOMA_ENONFINITE
    g.close()


def test_ideal_chain_acceptance_closed_form_on_gpu():
    N, n_chains = 32, 16384
    s = W.diblock_system(n_chains, N, 0.5, 0.0, 0.0, (16, 16, 16), (64, 64, 64))
    g = Soma([s], seed=SEED, pos_repr="f32", count_width=16)
    g.sweep(20)
    ob = g.observables(0)
    expect = acceptance_closed_form(N, 0.05)
    se = math.sqrt(expect * (1 - expect) / ob["n_moves"])
    assert abs(ob["accept_ratio"] - expect) < max(6 * se, 4e-4), (ob["accept_ratio"], expect)
    assert ob["Ebond_per_chain"] == pytest.approx(1.5 * (N - 1), abs=5 * math.sqrt(1.5 * (N - 1) / n_chains))
    assert ob["Re2"] == pytest.approx(1.0, abs=5 * math.sqrt(2 / 3 / n_chains))
    g.close()


def test_two_bead_frozen_field_boltzmann_on_gpu():
    n_chains, L, n = 32768, 1.0, 4
    s = W.SystemDesc(n_chains=n_chains, N=2, pattern_a=np.array([0, 1], np.uint8),
                     pattern_b=np.array([0, 1], np.uint8), n_chains_a=n_chains, chiN=0.0, kappaN=0.0,
                     box=(L, L, L), grid=(n, n, n), move_halfwidth=0.2)
    M = n ** 3
    omega = np.random.default_rng(4).uniform(-1.0, 1.0, size=(2, M)).astype(np.float32)
    g = Soma([s], seed=SEED, pos_repr="cell", count_width=32)
    g.set_fields(0, omega)
    g.sweep(150)
    acc = np.zeros((2, M))
    for _ in range(50):
        g.sweep(5)
        acc += g.density(0)
    assert np.abs(g.fields(0) - omega).max() == 0.0       # frozen: never refreshed
    P, idx = two_bead_cell_probabilities(omega.astype(np.float64), n, L, 3.0)
    pA, pB = P.sum(axis=1), P.sum(axis=0)
    assert np.abs(acc[0] / acc[0].sum() / pA - 1).max() < 0.06
    assert np.abs(acc[1] / acc[1].sum() / pB - 1).max() < 0.06
    assert 0.5 * np.abs(acc[0] / acc[0].sum() - pA).sum() < 0.012
    g.release_fields(0)
    g.close()


def apply_shape(g, shape):
    """"auto": the benchmark's launch configuration (the autotuner's choice);
    "dmK": the library's default shape in density mode K."""
    if shape == "auto":
        t = g.autotune(2)
        print(f"[shape] autotuned: {t}", flush=True)
    return g


@pytest.mark.parametrize("shape", ["auto", "dm0", "dm1", "dm2", "dm3", "stream"])
@pytest.mark.parametrize("name", ["plain_large", "mixed_large"])
def test_full_size_single_sweep_parity(name, shape):
    """Full-size workloads, in the benchmark's launch configuration (the
    autotuner's choice) and in each density mode: every bead's decision
    compared, mismatch rate <= 1e-6, density bit-exact after each sweep."""
    systems = W.workload(name)
    opts = W.WORKLOAD_OPTIONS[name]
    r, cw = opts["pos_repr"], opts["count_width"]
    s = systems[0]
    print(f"[full-size] {name} ({shape}): {s.n_beads} beads", flush=True)
    xyz = W.gaussian_walks(s, seed=11)
    dm = int(shape[2]) if shape.startswith("dm") else (3 if shape == "stream" else 0)
    g = apply_shape(Soma(systems, seed=SEED, pos_repr=r, count_width=cw, density_mode=dm,
                         packed_tiles=2 if shape == "stream" else 0, reorder_every=opts["reorder_every"]), shape)
    g.set_positions(0, xyz)
    o = oracle.OracleSystem(s, sys_id=0, mode=oracle.MODE_F32 if r == "f32" else oracle.MODE_CELL)
    o.set_positions(xyz)
    del xyz
    assert (g.density(0) == o.counts).all()
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
    print(f"[full-size] {name} ({shape}, density mode {g.info()['density_mode']}): "
          f"{mism} differing beads of {total} decisions", flush=True)
    assert mism / total <= 1e-6, (mism, total)
    g.close()


def face_system():
    # cell edge 1.275 / 25 = 0.051: not a power of two, so the GPU's product
    # with the FP32 reciprocal needs its correction next to every face
    return W.diblock_system(2048, 8, 0.5, 20.0, 50.0, (1.275, 1.275, 1.275), (25, 25, 25), "faces")


def face_positions(s, seed=5):
    from tests.helpers.positions import face_adjacent_fp32
    edge32 = np.float32(s.box[0] / s.grid[0])
    rng = np.random.default_rng(seed)
    xs = face_adjacent_fp32(edge32, list(range(-30, 60, 3)), rng)
    xyz = W.gaussian_walks(s, seed=seed)
    # bead 0 of each chain on a face-adjacent coordinate in every axis; the
    # walk around it shifted with it
    shift = np.stack([rng.choice(xs, size=s.n_chains) for _ in range(3)]) - xyz[:, 0::s.N]
    return xyz + np.repeat(shift, s.N, axis=1)


@pytest.mark.parametrize("r,cw", [("f32", 16), ("cell", 32)])
def test_non_dyadic_edge_faces_density_and_sweep(r, cw):
    s = face_system()
    xyz = face_positions(s)
    g = Soma([s], seed=SEED, pos_repr=r, count_width=cw)
    g.set_positions(0, xyz)
    o = oracle.OracleSystem(s, mode=oracle.MODE_F32 if r == "f32" else oracle.MODE_CELL)
    o.set_positions(xyz)
    assert (g.density(0) == o.counts).all()
    g.sweep(1)
    o.sweep(SEED, 0)
    o.density()
    assert same_state(g, 0, o).all()
    assert (g.density(0) == o.counts).all()
    g.close()
