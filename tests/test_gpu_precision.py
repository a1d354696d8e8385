"""Precision of the two position representations, equilibrium agreement with
the FP64 oracle, and sampled full-size parity of the batched workloads.

* Precision error: the GPU (FP32 positions, and int32 cell + FP32 offset)
  and the FP64-position oracle start from the same positions in a 64 Re
  wide box and run the same sweeps with the same random numbers.  The
  relative error of Re^2, Rg^2 and the bond energy per chain is printed
  for each representation and bounded.  Far from the origin FP32 keeps
  about 4e-6 Re, while the cell form keeps 1.5e-8 Re.
* Equilibrium: in a disordered melt, after equilibration, time averages of
  Re^2, Rg^2, bond and non-bonded energy per chain agree with the FP64
  oracle within two combined standard errors (block averages over blocks
  of at least twice the correlation time) and within 0.5 %.
* Full size, batched: one sweep of the 64- and 256-system workloads in the
  benchmark's launch configuration (autotuned) and in density modes 1 and 2;
  for sampled systems the oracle starts
  from the GPU's own stored state, and the density and the next stored
  state are compared bead by bead.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2606_09356_amd import workloads as W
from paper_2606_09356_amd.soma import Soma

pytestmark = pytest.mark.gpu
SEED = 20260609


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# Measured errors of the two representations on this case (10 sweeps): FP32
# Re^2 1.5e-5, Rg^2 2.0e-6, E_b 9.4e-6; cell + offset 1.1e-10, 1.7e-10,
# 1.9e-9.  Each bound sits about 10x above its measurement, so a regression
# of one representation toward the other's precision fails.
PRECISION_BOUND = {"f32": {"Re2": 1.5e-4, "Rg2": 2e-5, "Ebond_per_chain": 1e-4},
                   "cell": {"Re2": 1e-9, "Rg2": 2e-9, "Ebond_per_chain": 2e-8}}


def test_precision_error_against_fp64_positions():
    # 1M beads in a 64 x 64 x 2 Re slab: coordinates up to 64 Re
    s = W.diblock_system(32768, 32, 0.5, 20.0, 50.0, (64.0, 64.0, 2.0), (256, 256, 8))
    xyz = W.gaussian_walks(s, seed=21)
    o = oracle.OracleSystem(s, sys_id=0, mode=oracle.MODE_F64)
    o.set_positions(xyz)
    g32 = Soma([s], seed=SEED, pos_repr="f32", count_width=16)
    gc = Soma([s], seed=SEED, pos_repr="cell", count_width=16)
    g32.set_positions(0, xyz)
    gc.set_positions(0, xyz)
    worst = {"f32": {}, "cell": {}}
    for sweep in range(10):
        o.run(SEED, sweep, 1)
        g32.sweep(1)
        gc.sweep(1)
        oo = o.observables()
        for name, g in (("f32", g32), ("cell", gc)):
            go = g.observables(0)
            for k in ("Re2", "Rg2", "Ebond_per_chain"):
                worst[name][k] = max(worst[name].get(k, 0.0), rel(go[k], oo[k]))
    print(f"[precision] max relative error over 10 sweeps vs FP64 positions: {worst}")
    for name in worst:
        for k, v in worst[name].items():
            assert v < PRECISION_BOUND[name][k], (name, k, v)
    g32.close()
    gc.close()


def tau_int(x):
    """Integrated autocorrelation time of a series, in samples, with Sokal's
    automatic window (the smallest W with W >= 5 tau(W))."""
    x = np.asarray(x, float) - np.mean(x)
    n = len(x)
    f = np.fft.rfft(x, 2 * n)
    ac = np.fft.irfft(f * np.conj(f))[:n]
    ac = ac / ac[0]
    t = 0.5
    for w in range(1, n):
        t += ac[w]
        if w >= 5 * t:
            break
    return t


def block_mean_sigma(x, block):
    """Mean of the series and the standard error of the mean from the
    variance of its block means."""
    nb = len(x) // block
    b = np.asarray(x[: nb * block], float).reshape(nb, block).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / math.sqrt(nb)), nb


def test_equilibrium_observables_agree_with_oracle():
    """Equilibrium agreement with the FP64-position oracle (time averages of
    Re^2, Rg^2, bond and non-bonded energy per chain), for both position
    representations, in a disordered melt (chiN = 10, N = 8, 32768 chains,
    trial cube half-width 0.2 Re so the chains relax in about a hundred
    sweeps).  After 1500 sweeps of equilibration, observables are sampled
    every 5 sweeps for 6000 sweeps; the integrated autocorrelation time tau of
    the chain size (the slowest of the Re^2 and Rg^2 series, at least 200
    sweeps) sets the block length for every observable (3 tau, above the 2 tau
    the reading of the tolerance asks for, and at least 8 blocks); the standard
    error of each time average is the spread of its block means.  Pass:
    |GPU - oracle| <= 2 sqrt(s_GPU^2 + s_oracle^2) and within 0.5 %.  (The
    system is sized so that the Re^2 difference has a standard error near
    0.15 %, well inside the 0.5 % cap.)"""
    s = W.diblock_system(32768, 8, 0.5, 10.0, 50.0, (16.0, 16.0, 8.0), (64, 64, 32), move_halfwidth=0.2)
    xyz = W.gaussian_walks(s, seed=22)
    burn, total, every = 1500, 6000, 5
    keys = ("Re2", "Rg2", "Ebond_per_chain", "Enb_per_chain")
    o = oracle.OracleSystem(s, sys_id=0, mode=oracle.MODE_F64)
    o.set_positions(xyz)
    gs = {r: Soma([s], seed=SEED, pos_repr=r, count_width=16, reorder_every=50) for r in ("f32", "cell")}
    for g in gs.values():
        g.set_positions(0, xyz)
        g.sweep(burn)
    o.run(SEED, 0, burn)
    series = {"oracle": {k: [] for k in keys}, "f32": {k: [] for k in keys}, "cell": {k: [] for k in keys}}
    sweep = burn
    for _ in range(total // every):
        o.run(SEED, sweep, every)
        sweep += every
        oo = o.observables()
        for k in keys:
            series["oracle"][k].append(oo[k])
        for r, g in gs.items():
            g.sweep(every)
            go = g.observables(0)
            for k in keys:
                series[r][k].append(go[k])
    for g in gs.values():
        g.close()
    # one correlation time for every observable: the slowest of the chain-size
    # series (Re^2, Rg^2) of the three trajectories, at least 200 sweeps (the
    # energies carry the same slow chain-size modes under faster noise)
    tau = max([tau_int(series[src][k]) for src in series for k in ("Re2", "Rg2")] + [200 / every])
    block = max(int(math.ceil(3 * tau)), 1)
    for k in keys:
        assert len(series["oracle"][k]) // block >= 8, (k, tau, block)
        mo, so, nb = block_mean_sigma(series["oracle"][k], block)
        for r in ("f32", "cell"):
            mg, sg, _ = block_mean_sigma(series[r][k], block)
            diff = abs(mg - mo)
            bound = 2 * math.sqrt(sg ** 2 + so ** 2)
            print(f"[equilibrium {r}] {k}: gpu {mg:.6f} +- {sg:.1e}, oracle {mo:.6f} +- {so:.1e}, "
                  f"tau {tau * every:.0f} sweeps, {nb} blocks of {block * every} sweeps: diff {diff:.2e} "
                  f"(2 sigma {bound:.2e}, rel {diff / abs(mo):.2e})")
            assert diff <= bound, (r, k, diff, bound)
            assert diff <= 5e-3 * abs(mo), (r, k, diff)


@pytest.mark.parametrize("shape", ["auto", "dm1", "dm2", "dm3", "packed", "stream"])
@pytest.mark.parametrize("name,sample", [("batched_uneven", [0, 17, 63]), ("batched_mixed", [0, 101, 255])])
def test_full_size_batched_sampled_parity(name, sample, shape):
    """One sweep of the full batched workloads in the benchmark's launch
    configuration (autotuned) and in density modes 1 and 2."""
    systems = W.workload(name)
    opts = W.WORKLOAD_OPTIONS[name]
    r, cw = opts["pos_repr"], opts["count_width"]
    print(f"[full-size] {name} ({shape}): {len(systems)} systems, {sum(s.n_beads for s in systems)} beads",
          flush=True)
    dm = int(shape[2]) if shape.startswith("dm") else (3 if shape == "stream" else 0)
    pk = {"packed": 1, "stream": 2}.get(shape, 0)
    g = Soma(systems, seed=SEED, pos_repr=r, count_width=cw, reorder_every=opts["reorder_every"], density_mode=dm,
             packed_tiles=pk, waves_per_block=4 if pk else 0)
    if shape == "auto":
        print(f"[shape] autotuned: {g.autotune(2)}", flush=True)
    g.sweep(3)
    mode = oracle.MODE_F32 if r == "f32" else oracle.MODE_CELL
    orcs = {}
    for k in sample:
        o = oracle.OracleSystem(systems[k], sys_id=k, mode=mode)
        st = g.state(k)
        if mode == oracle.MODE_F32:
            o.xf[...] = st
        else:
            o.off[...], o.cell[...] = st
        o.density()
        o.fields()
        assert (g.density(k) == o.counts).all(), (name, k)
        orcs[k] = o
    g.sweep(1)
    total = mism = 0
    for k, o in orcs.items():
        o.sweep(SEED, 3)
        st = g.state(k)
        if mode == oracle.MODE_F32:
            eq = (st == o.xf).all(axis=0)
        else:
            eq = ((st[0] == o.off) & (st[1] == o.cell)).all(axis=0)
        total += eq.size
        mism += int((~eq).sum())
        o.density()
        if eq.all():
            assert (g.density(k) == o.counts).all(), (name, k)
    print(f"[full-size] {name}: {mism} differing beads of {total} sampled decisions", flush=True)
    assert mism <= max(1, int(1e-6 * total)), (mism, total)
    g.close()
