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
  oracle within 0.5 %, and Re^2, Rg^2 within two combined chain-level
  standard errors.
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
            assert v < 2e-3, (name, k, v)
    g32.close()
    gc.close()


@pytest.mark.parametrize("r", ["f32", "cell"])
def test_equilibrium_observables_agree_with_oracle(r):
    """Disordered melt (chiN = 10 < 10.5), N = 16, 32768 chains: after 200
    sweeps of equilibration, time averages over 400 sweeps agree within two
    combined chain-level standard errors and within 0.5 %."""
    s = W.diblock_system(32768, 16, 0.5, 10.0, 50.0, (16.0, 16.0, 16.0), (64, 64, 64))
    xyz = W.gaussian_walks(s, seed=22)
    o = oracle.OracleSystem(s, sys_id=0, mode=oracle.MODE_F64)
    o.set_positions(xyz)
    g = Soma([s], seed=SEED, pos_repr=r, count_width=16, reorder_every=50)
    g.set_positions(0, xyz)
    burn, snaps, every = 200, 20, 20
    o.run(SEED, 0, burn)
    g.sweep(burn)
    keys = ("Re2", "Rg2", "Ebond_per_chain", "Enb_per_chain")
    gs = {k: [] for k in keys + ("Re2_err", "Rg2_err")}
    os_ = {k: [] for k in keys + ("Re2_err", "Rg2_err")}
    sweep = burn
    for _ in range(snaps):
        o.run(SEED, sweep, every)
        g.sweep(every)
        sweep += every
        go, oo = g.observables(0), o.observables()
        for k in gs:
            gs[k].append(go[k])
            os_[k].append(oo[k])
    for k in keys:
        a, b = float(np.mean(gs[k])), float(np.mean(os_[k]))
        diff = abs(a - b)
        if k in ("Re2", "Rg2"):
            se = math.sqrt(np.mean(gs[k + "_err"]) ** 2 + np.mean(os_[k + "_err"]) ** 2)
            print(f"[equilibrium {r}] {k}: gpu {a:.6f} oracle {b:.6f} diff {diff:.2e} 2se {2 * se:.2e}")
            assert diff <= 2 * se, (k, diff, se)
        else:
            print(f"[equilibrium {r}] {k}: gpu {a:.6f} oracle {b:.6f} rel diff {diff / abs(b):.2e}")
        assert diff <= 5e-3 * abs(b), (k, diff)
    g.close()


@pytest.mark.parametrize("shape", ["auto", "dm1", "dm2", "packed"])
@pytest.mark.parametrize("name,sample", [("batched_uneven", [0, 17, 63]), ("batched_mixed", [0, 101, 255])])
def test_full_size_batched_sampled_parity(name, sample, shape):
    """One sweep of the full batched workloads in the benchmark's launch
    configuration (autotuned) and in density modes 1 and 2."""
    systems = W.workload(name)
    opts = W.WORKLOAD_OPTIONS[name]
    r, cw = opts["pos_repr"], opts["count_width"]
    print(f"[full-size] {name} ({shape}): {len(systems)} systems, {sum(s.n_beads for s in systems)} beads",
          flush=True)
    dm = int(shape[2]) if shape.startswith("dm") else 0
    pk = 1 if shape == "packed" else 0
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
