"""Benchmark: bead Monte-Carlo moves per second of the SCMF sweep on one MI355X.

A step is one full sweep (move, density, field) of every bead of the
workload.  Inputs live in HBM before the timed region; the timed region is
K sweeps replayed as hipGraphs on the context's stream, bracketed by HIP
events on that stream and device synchronisation.

Default workload: one plain FP32 system of 131072 AB diblock chains, N=32
(4.19M beads), chiN=20, kappaN=50, 32^3 Re box, 128^3 grid, uint16 counts.

Extra legs (on by default, --no-extra to skip):
  batched   64 uneven diblock systems (~20M beads) in one launch per sweep,
            against the same systems run one after another as single-system
            contexts; the per-system results are bit-identical, so the Re^2
            error is matched exactly, and the JSON says so.
  mixed     262144 chains, N=64 (16.8M beads), int32 cell + FP32 offset,
            uint32 counts.
  batched mixed  256 systems (124.6M beads), cell + offset, uint16 counts.
  smart     the default workload with bond-force-biased moves.
The CPU baseline is the FP64 oracle (test infrastructure), timed on a
bounded sample of the default workload on the host cores.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, AMD public specification
SEED = 20260609


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--workload", default="plain_large")
    p.add_argument("--no-extra", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run one 1 GiB device copy (reference for HBM byte counters) and exit")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the default launch shape instead of timing every shape first")
    p.add_argument("--shape", default=None,
                   help="fixed launch shape WPB,WPCU,ORDER,DM for the main workload (no autotuning): "
                        "waves per block, waves per CU (0: one tile per wave), launch_order, density_mode")
    return p.parse_args()


def timed_sweeps(g, steps, warmup):
    """Run warmup sweeps, then time `steps` sweeps with HIP events on the context stream."""
    import torch
    g.sweep(warmup)
    g.sync()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(g.stream)
    g.sweep(steps)
    end.record(g.stream)
    end.synchronize()
    g.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / 1e3, wall


def run_workload(name, steps, warmup, shape=None, autotune=True):
    from paper_2606_09356_amd import workloads as W
    from paper_2606_09356_amd.soma import Soma
    systems = W.workload(name)
    o = W.WORKLOAD_OPTIONS[name]
    wpb, wpcu, order, dm = shape if shape else (0, 0, 0, 0)
    g = Soma(systems, seed=SEED, pos_repr=o["pos_repr"], count_width=o["count_width"],
             use_graph=True, waves_per_block=wpb, waves_per_cu=wpcu, launch_order=order, density_mode=dm,
             reorder_every=o["reorder_every"])
    tune = g.autotune(5) if autotune and not shape else None
    info = g.info()
    sec, wall = timed_sweeps(g, steps, warmup)
    obs = g.observables(0)
    g.close()
    info["autotune"] = tune
    return systems, info, sec, wall, obs


def shape_of(info):
    return {"waves_per_block": info["waves_per_block"], "waves_per_cu": info["waves_per_cu"],
            "xcd_remap": info["xcd_remap"], "density_mode": info["density_mode"],
            "autotuned": info.get("autotune") is not None}


def batched_vs_plain(steps, warmup, autotune=True):
    """Batched launch of the 64 uneven systems vs each system alone, same sweeps."""
    import numpy as np
    from paper_2606_09356_amd import workloads as W
    from paper_2606_09356_amd.soma import Soma
    systems = W.batched_uneven()
    o = W.WORKLOAD_OPTIONS["batched_uneven"]
    B = sum(s.n_beads for s in systems)
    g = Soma(systems, seed=SEED, pos_repr=o["pos_repr"], count_width=o["count_width"], use_graph=True,
             reorder_every=o["reorder_every"])
    tune = g.autotune(5) if autotune else None
    sec_b, _ = timed_sweeps(g, steps, warmup)
    info_b = g.info()
    info_b["autotune"] = tune
    re2_b = [g.observables(k)["Re2"] for k in range(len(systems))]
    g.close()
    sec_p = 0.0
    re2_p = []
    for k, s in enumerate(systems):
        a = Soma([s], seed=SEED, pos_repr=o["pos_repr"], count_width=o["count_width"], use_graph=True,
                 sys_id_base=k, reorder_every=o["reorder_every"])
        if autotune:
            a.autotune(5)
        t, _ = timed_sweeps(a, steps, warmup)
        sec_p += t
        re2_p.append(a.observables(0)["Re2"])
        a.close()
    re2_b, re2_p = np.array(re2_b), np.array(re2_p)
    return {
        "workload": "64 uneven AB diblock systems (chains U{512..16384}, N in {16,32,64}, "
                    "f U[0.3,0.7], chiN U[10,40], kappaN 50), FP32, uint16 counts",
        "beads": int(B), "sweeps": steps,
        "batched_moves_per_s": B * steps / sec_b,
        "plain_sequential_moves_per_s": B * steps / sec_p,
        "batched_over_plain": sec_p / sec_b,
        "batched_hbm_gbs": info_b["bytes_per_sweep"] * steps / sec_b / 1e9,
        "batched_shape": shape_of(info_b), "plain_autotuned_each": bool(autotune),
        "re2_max_abs_diff_batched_vs_plain": float(np.abs(re2_b - re2_p).max()),
    }


def profiled(workload):
    """The committed rocprofv3 counter summary of k_sweep (HBM bytes and
    atomics per launch), only while the kernel source is the one that was
    profiled (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_sweep_{workload}_traffic.json")
    src = os.path.join(ROOT, "paper_2606_09356_amd", "csrc", "soma_kernels.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return rec


def atomic_calibration(n_words=1 << 21, n_ops=1 << 23, reps=5):
    """Device-scope 32-bit atomic adds per second at random words of an 8 MiB
    array (torch index_add_ on int32, which issues one atomic per element)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(SEED)
    buf = torch.zeros(n_words, dtype=torch.int32, device="cuda")
    idx = torch.randint(0, n_words, (n_ops,), device="cuda", generator=g)
    one = torch.ones(n_ops, dtype=torch.int32, device="cuda")
    buf.index_add_(0, idx, one)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        buf.index_add_(0, idx, one)
    e1.record()
    e1.synchronize()
    assert int(buf.sum().item()) == (reps + 1) * n_ops
    return n_ops * reps / (e0.elapsed_time(e1) / 1e3)


def cpu_baseline(name, budget_s=15.0):
    """The oracle (FP64, OpenMP) on a bounded sample of the workload's sweeps."""
    import oracle
    from paper_2606_09356_amd import workloads as W
    systems = W.workload(name)
    s = systems[0]
    o = W.WORKLOAD_OPTIONS[name]
    mode = oracle.MODE_F32 if o["pos_repr"] == "f32" else oracle.MODE_CELL
    orc = oracle.OracleSystem(s, sys_id=0, mode=mode)
    orc.set_positions(W.gaussian_walks(s, seed=1))
    t0 = time.perf_counter()
    sweeps = 0
    while time.perf_counter() - t0 < budget_s:
        orc.run(SEED, sweeps, 1)
        sweeps += 1
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": s.n_beads * sweeps / dt, "unit": "bead moves/s", "cores": cores, "kind": "oracle",
            "sample": f"{sweeps} full sweeps (move, density, field) of the {s.n_beads}-bead workload, "
                      f"{dt:.1f} s on {cores} OpenMP threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30}))
        return
    from paper_2606_09356_amd.soma import load_library
    load_library()

    print(f"[bench] workload {args.workload}: {args.warmup} warmup + {args.steps} timed sweeps", flush=True)
    autotune = not args.no_autotune
    shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else None
    systems, info, sec, wall, obs = run_workload(args.workload, args.steps, args.warmup, shape, autotune)
    B = info["n_beads"]
    prof = profiled(args.workload)
    if prof and prof.get("density_mode") != info["density_mode"]:
        prof = None         # profiled in another density mode
    moves_per_s = B * args.steps / sec
    ms_per_step = sec * 1e3 / args.steps
    achieved = info["bytes_per_sweep"] / (sec / args.steps) / 1e9
    out = {
        "metric": "bead MC moves/sec on 1 MI355X (batched vs plain) at matched Re^2 error",
        "value": moves_per_s,
        "unit": "bead moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if systems and args.workload != "mixed_large" else "i32+f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {len(systems)} system(s), {B} beads, {info['n_cells']} cells, "
                               "Gaussian-walk start, delta 0.05 Re, 128 beads/Re^3, cell Re/4",
                   "beads": B, "sweeps_per_step": 1, "parallelism": "single GPU",
                   "launch_shape": shape_of(info)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": prof["traffic_bytes_per_launch"] if prof else None,
                     "bytes_per_sweep": info["bytes_per_sweep"],
                     "kernel": {0: "k_sweep + k_fold (moves with fields from the counts, then the delta fold), "
                                   "two launches per sweep",
                                1: "k_sweep (moves with fields from base + previous delta, folds the previous "
                                   "delta), one launch per sweep",
                                2: "k_sweep + k_fold_faces (moves emitting face fluxes, then the flux-divergence "
                                   "fold), two launches per sweep"}[info["density_mode"]],
                     "avg_sweep_us_hip_events": sec / args.steps * 1e6},
        "observables": {k: obs[k] for k in ("Re2", "Re2_err", "Rg2", "Ebond_per_chain", "Enb_per_chain",
                                           "accept_ratio")},
        "wall_s": wall,
    }
    print("[bench] atomic-rate calibration", flush=True)
    peak_atomics = atomic_calibration()
    atom = {"calibrated_peak_per_s": peak_atomics,
            "calibration": "torch index_add_ of 2^23 ones at random words of an 8 MiB int32 array"}
    if prof and prof.get("atomics_per_launch"):
        kern_s = prof["k_sweep_avg_ns"] * 1e-9
        atom.update({"atomics_per_sweep": prof["atomics_per_launch"],
                     "achieved_per_s": prof["atomics_per_launch"] / kern_s,
                     "frac": prof["atomics_per_launch"] / kern_s / peak_atomics,
                     "source": "TCC_ATOMIC_sum and k_sweep duration from the committed rocprofv3 summary"})
    out["roofline"]["atomics"] = atom
    if not args.no_extra:
        print("[bench] batched vs plain", flush=True)
        out["batched_vs_plain"] = batched_vs_plain(min(args.steps, 200), min(args.warmup, 20), autotune)
        print("[bench] mixed precision workload", flush=True)
        ms, minfo, msec, _, mobs = run_workload("mixed_large", min(args.steps, 200), min(args.warmup, 20),
                                                autotune=autotune)
        mst = min(args.steps, 200)
        out["mixed_large"] = {"moves_per_s": minfo["n_beads"] * mst / msec,
                              "hbm_gbs": minfo["bytes_per_sweep"] * mst / msec / 1e9,
                              "frac": minfo["bytes_per_sweep"] * mst / msec / 1e9 / HBM_PEAK_GBS,
                              "beads": minfo["n_beads"], "Re2": mobs["Re2"], "launch_shape": shape_of(minfo)}
        print("[bench] batched mixed-precision workload", flush=True)
        bs, binfo, bsec, _, _ = run_workload("batched_mixed", min(args.steps, 100), min(args.warmup, 10),
                                             autotune=autotune)
        bst = min(args.steps, 100)
        out["batched_mixed"] = {"workload": "256 systems of A/B blends, AB and ABA (N 8..128, 1e4..1e6 beads), "
                                            "int32 cell + FP32 offset, uint16 counts",
                                "moves_per_s": binfo["n_beads"] * bst / bsec,
                                "hbm_gbs": binfo["bytes_per_sweep"] * bst / bsec / 1e9,
                                "frac": binfo["bytes_per_sweep"] * bst / bsec / 1e9 / HBM_PEAK_GBS,
                                "beads": binfo["n_beads"], "systems": len(bs), "launch_shape": shape_of(binfo),
                                "over_plain_large": (binfo["n_beads"] * bst / bsec) / moves_per_s}
        print("[bench] smart-move workload", flush=True)
        ss, sinfo, ssec, _, sobs = run_workload("plain_large_smc", min(args.steps, 200), min(args.warmup, 20),
                                                autotune=autotune)
        sst = min(args.steps, 200)
        out["plain_large_smc"] = {"workload": "plain_large with bond-force-biased (smart) moves, A = 4e-4 Re^2",
                                  "moves_per_s": sinfo["n_beads"] * sst / ssec,
                                  "hbm_gbs": sinfo["bytes_per_sweep"] * sst / ssec / 1e9,
                                  "accept_ratio": sobs["accept_ratio"], "Re2": sobs["Re2"],
                                  "launch_shape": shape_of(sinfo)}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
