"""Benchmark: bead Monte-Carlo moves per second of the SCMF sweep on one MI355X.

A step is one full sweep (move, density, field) of every bead of the
workload.  Inputs live in HBM before the timed region; each timed run is K
sweeps replayed as hipGraphs on the context's stream, bracketed by HIP
events on that stream and device synchronisation; the reported time is the
median of five such runs after W warm-up sweeps.

Headline workload (the batched mixed-precision form): 256 independent
systems of A/B homopolymer blends, AB diblocks and ABA triblocks, N 8..128,
1e4..1e6 beads each (124.6M beads), chiN U[0,50], kappaN U[25,100], int32
cell + FP32 offset positions, packed uint16 counts, all systems advanced by
one launch sequence per sweep.

Batched vs plain at matched Re^2 error:
  * the same 256 systems, each run alone in its own context (one system per
    launch): system k run alone with Philox system id k draws the same random
    numbers as in the batch, so Re^2 is bit-identical (difference 0.0);
  * the plain single-system FP32 form: one 131072-chain AB melt, N=32,
    32^3 Re box, 128^3 grid, FP32 positions (its Re^2 representation error,
    1.5e-5 relative against FP64 positions, is larger than the cell form's
    1.1e-10, so the batched form's accuracy is at least matched).
Extra legs (on by default, --no-extra to skip): the small plain system (256
chains, 8192 beads) at 1000 sweeps, the 16.8M-bead mixed-precision system, the 64
uneven systems against the same systems run one after another, and the
bond-force-biased (smart) move workload.

Roofline: algorithmic bytes per bead move of the sweep's data model
(positions read and written, field read, count write, field-kernel count
read and field write: 36 B for FP32 positions with packed uint16 counts, 60 B
for cell + offset with uint16, 64 B for cell + offset with uint32) times the
beads of one sweep, divided by the sweep's duration (HIP events on the
context stream; a sweep is the sweep kernel plus its count upkeep: the fold
kernel in density modes 0 and 2, the copy in mode 3, whose count check runs
once per batch of sweeps).  The
per-kernel split is measured with HIP events around each launch
(soma_time_kernels) after the timed runs; the HBM traffic of a sweep comes
from the committed rocprofv3 counters (profiles/sweep_<workload>_*), reported
only while they describe the current kernel source and density mode.

The CPU baseline is the FP64 oracle (test infrastructure), timed on a
bounded sample of the headline workload on the host cores.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, AMD public specification
SEED = 20260609
RUNS = 5                  # timed runs per measurement; the median is reported

# The paper's own SOMA figures (Sec. 2.2, single GPU, NVIDIA hardware); the
# paper states no system size for them, so they cannot be turned into bead
# moves per second and serve as context only.
PAPER_SOMA = {
    "source": "Sec. 2.2 (SOMA Optimization) and its time-steps-per-second figure",
    "time_steps_per_s": {"A100 baseline": 1.6, "A100 optimised": 2.5, "H100 optimised": 3.5},
    "kernel_runtime_change_A100": "-40 % after coalescing, caching and launch tuning",
    "speedup_A100_opt_over_A100_base": 2.5 / 1.6,
    "speedup_H100_opt_over_A100_base": 3.5 / 1.6,
    "note": "system size not stated in the paper; not convertible to bead moves/s",
}


def model_bytes_per_move(pos_repr, count_width):
    """Algorithmic HBM bytes per bead move: positions read and written
    (12 or 24 B each way), the field read once per cell (8 B per cell), the
    count written (4 or 8 B per cell), the field kernel's count read and its
    field write (8 B per cell), at 2 beads per cell."""
    pos = 24 if pos_repr == "f32" else 48
    cnt = 2 if int(count_width) == 16 else 4
    return pos + 4 + cnt + cnt + 4


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="batched_mixed")
    p.add_argument("--runs", type=int, default=RUNS)
    p.add_argument("--no-extra", action="store_true")
    p.add_argument("--no-plain", action="store_true", help="skip the batched-vs-plain legs")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run one 1 GiB device copy (reference for HBM byte counters) and exit")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the default launch shape instead of timing every shape first")
    p.add_argument("--shape", default=None,
                   help="fixed launch shape WPB,WPCU,ORDER,DM[,PACKED] for the main workload (no "
                        "autotuning): waves per block, waves per CU (0: one tile per wave), launch_order, "
                        "density_mode, packed_tiles (0 wave tiles, 1 block tiles, 2 stream tiles)")
    return p.parse_args()


def timed_sweeps(g, steps, warmup, runs=RUNS):
    """Warm-up sweeps, then `runs` timed runs of `steps` sweeps, each timed
    with HIP events on the context stream; returns the median seconds per
    run and the list of all runs."""
    import torch
    g.sweep(warmup)
    g.sync()
    torch.cuda.synchronize()
    secs = []
    for _ in range(runs):
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(g.stream)
        g.sweep(steps)
        end.record(g.stream)
        end.synchronize()
        g.sync()
        torch.cuda.synchronize()
        secs.append(start.elapsed_time(end) / 1e3)
    return statistics.median(secs), secs


def make_context(systems, opts, shape=None, sys_id_base=0):
    from paper_2606_09356_amd.soma import Soma
    wpb, wpcu, order, dm, packed = (tuple(shape) + (0,))[:5] if shape else (0, 0, 0, 0, 0)
    return Soma(systems, seed=SEED, pos_repr=opts["pos_repr"], count_width=opts["count_width"],
                use_graph=True, waves_per_block=wpb, waves_per_cu=wpcu, launch_order=order, density_mode=dm,
                reorder_every=opts["reorder_every"], sys_id_base=sys_id_base, packed_tiles=packed)


def shape_of(info, tune=None):
    d = {"waves_per_block": info["waves_per_block"], "waves_per_cu": info["waves_per_cu"],
         "xcd_remap": info["xcd_remap"], "density_mode": info["density_mode"],
         "packed_tiles": info["packed_tiles"], "autotuned": tune is not None}
    if tune is not None:
        d["tune_from_cache"] = bool(tune.get("from_cache", 0))
    return d


def run_workload(name, steps, warmup, shape=None, autotune=True, runs=RUNS, kernel_times=False):
    """Create, autotune, time; returns a dict with the rate and the context's info."""
    from paper_2606_09356_amd import workloads as W
    systems = W.workload(name)
    o = W.WORKLOAD_OPTIONS[name]
    g = make_context(systems, o, shape)
    tune = g.autotune(5) if autotune and not shape else None
    info = g.info()
    sec, all_secs = timed_sweeps(g, steps, warmup, runs)
    B = info["n_beads"]
    res = {"workload": name, "systems": len(systems), "beads": B, "cells": info["n_cells"], "sweeps": steps,
           "runs_s": all_secs, "median_s": sec, "moves_per_s": B * steps / sec,
           "sweep_us": sec / steps * 1e6, "launch_shape": shape_of(info, tune), "info": info,
           "pos_repr": o["pos_repr"], "count_width": o["count_width"]}
    # observables after exactly warmup + runs x steps sweeps (the trajectory
    # that a system run alone repeats), then the per-kernel timing sweeps
    res["re2"] = [g.observables(k)["Re2"] for k in range(len(systems))]
    res["obs0"] = g.observables(0)
    if kernel_times:
        # the observables leave the GPU idle between host round trips: a
        # graph-replayed warm-up brings its clocks back before the eager,
        # per-kernel timed sweeps
        g.sweep(max(warmup, 5))
        g.sync()
        res["kernel_us"] = g.time_kernels(5)
        # the K timed sweeps hold no chain reorder when K is below the
        # reorder interval R; one call of R sweeps holds exactly one, so its
        # time per sweep includes the reorder's share.  Two untimed calls of
        # R sweeps capture the graphs of the same segments (the reorder
        # splits a call, and graphs are kept per position-buffer role, which
        # each reorder swaps), so the timed one measures replays.
        R = W.WORKLOAD_OPTIONS[name]["reorder_every"]
        if R > 0:
            import torch
            g.sweep(R)
            g.sweep(R)
            g.sync()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(g.stream)
            g.sweep(R)
            e1.record(g.stream)
            e1.synchronize()
            res["reorder_every"] = R
            res["sweep_us_with_reorder"] = e0.elapsed_time(e1) * 1e3 / R
    g.close()
    return res


def roofline_of(res, prof=None):
    bpm = model_bytes_per_move(res["pos_repr"], res["count_width"])
    per_sweep = bpm * res["beads"]
    achieved = per_sweep / (res["sweep_us"] * 1e-6) / 1e9
    r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved / HBM_PEAK_GBS,
         "traffic": prof["traffic_bytes_per_sweep"] if prof else None,
        "traffic_source": ("rocprofv3 FETCH_SIZE x %.3f + WRITE_SIZE x %.3f of every sweep kernel, per sweep "
                           "(profiles/sweep_%s_counters.md)" % (prof["fetch_scale"], prof["write_scale"], res["workload"]))
        if prof else "no profile of the current kernel source and density mode",
         "bytes_per_move": bpm, "bytes_per_sweep": per_sweep,
         "launch": "one sweep: the sweep kernel, then the count upkeep (fold in density modes 0 and 2, "
                  "copy in mode 3, its count check once per batch of sweeps)",
         "sweep_us_hip_events": res["sweep_us"],
         "library_model_bytes_per_sweep": res["info"]["bytes_per_sweep"]}
    if "kernel_us" in res:
        k = res["kernel_us"]
        r["kernel_us_hip_events"] = k
        if k.get("sweep_kernel_us"):
            r["k_sweep_frac_of_sweep_bytes"] = per_sweep / (k["sweep_kernel_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
    return r


def profiled(workload, density_mode):
    """The committed rocprofv3 counter summary of the sweep kernels (HBM bytes
    and atomics per sweep, profiles/sweep_<workload>_traffic.json), only while
    the kernel source is the one that was profiled and the density mode
    matches (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"sweep_{workload}_traffic.json")
    src = os.path.join(ROOT, "paper_2606_09356_amd", "csrc", "soma_kernels.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    if rec.get("density_mode") != density_mode:
        return None
    return rec


def sequential_alone(name, steps, warmup, autotune=True, runs=RUNS):
    """Every system of a batched workload run alone (one system per context and
    launch), one after another; same Philox system ids, so the same moves."""
    from paper_2606_09356_amd import workloads as W
    systems = W.workload(name)
    o = W.WORKLOAD_OPTIONS[name]
    total, re2, tuned_from_cache = 0.0, [], 0
    for k, s in enumerate(systems):
        a = make_context([s], o, sys_id_base=k)
        if autotune:
            t = a.autotune(5)
            tuned_from_cache += int(bool(t.get("from_cache", 0)))
        sec, _ = timed_sweeps(a, steps, warmup, runs)      # median of the runs: same statistic as batched
        total += sec
        re2.append(a.observables(0)["Re2"])
        a.close()
    B = sum(s.n_beads for s in systems)
    return {"moves_per_s": B * steps / total, "seconds": total, "re2": re2, "systems": len(systems),
            "autotuned_each": bool(autotune), "tunes_from_cache": tuned_from_cache}


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(name, budget_s=15.0):
    """The oracle (FP64 energies, OpenMP over chains) on a bounded sample of
    the workload: its systems in order, one full sweep (move, density, field)
    each, until the time budget is spent."""
    import oracle
    from paper_2606_09356_amd import workloads as W
    systems = W.workload(name)
    o = W.WORKLOAD_OPTIONS[name]
    mode = oracle.MODE_F32 if o["pos_repr"] == "f32" else oracle.MODE_CELL
    moves, busy, done, sweeps = 0, 0.0, 0, 0
    k = 0
    while busy < budget_s:
        s = systems[k % len(systems)]
        orc = oracle.OracleSystem(s, sys_id=k % len(systems), mode=mode)
        orc.set_positions(W.gaussian_walks(s, seed=1 + k))
        t0 = time.perf_counter()
        orc.run(SEED, 0, 1)
        busy += time.perf_counter() - t0
        moves += s.n_beads
        sweeps += 1
        done = min(len(systems), done + 1)
        k += 1
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rate = moves / busy
    return {"value": rate, "unit": "bead moves/s", "cores": cores, "kind": "oracle",
            "per_core": rate / cores, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"one full sweep (move, density, field) per system, the {name} workload's "
                      f"{len(systems)} systems taken in order and again from the first: {sweeps} system "
                      f"sweeps, {moves} bead moves, {busy:.1f} s of oracle time on {cores} OpenMP threads "
                      "(setup excluded)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only (no multi-GPU path); "
                                   f"--gpus {args.gpus} is not supported, use --gpus 1"}))
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
    autotune = not args.no_autotune
    shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else None

    print(f"[bench] workload {args.workload}: {args.warmup} warmup + {args.runs} x {args.steps} timed sweeps",
          flush=True)
    main_res = run_workload(args.workload, args.steps, args.warmup, shape, autotune, args.runs,
                            kernel_times=True)
    B = main_res["beads"]
    prof = profiled(args.workload, main_res["info"]["density_mode"])
    out = {
        "metric": "bead MC moves/sec on 1 MI355X (batched vs plain) at matched Re^2 error",
        "value": main_res["moves_per_s"],
        "unit": "bead moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["sweep_us"] / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {main_res['systems']} system(s), {B} beads, "
                               f"{main_res['cells']} cells, Gaussian-walk start, delta 0.05 Re, "
                               "128 beads/Re^3, cell Re/4",
                   "positions": "int32 cell + fp32 offset" if main_res["pos_repr"] == "cell" else "fp32",
                   "counts": f"uint{main_res['count_width']}",
                   "beads": B, "sweeps_per_step": 1, "timed_runs": args.runs, "statistic": "median",
                   "parallelism": "single GPU, all systems in one launch per sweep",
                   "launch_shape": main_res["launch_shape"]},
        "roofline": roofline_of(main_res, prof),
        "observables_system0": {k: main_res["obs0"][k] for k in ("Re2", "Re2_err", "Rg2", "Ebond_per_chain",
                                                                  "Enb_per_chain", "accept_ratio")},
        "with_chain_reorder": ({"reorder_every": main_res["reorder_every"],
                                "sweep_us": main_res["sweep_us_with_reorder"],
                                "moves_per_s": B / (main_res["sweep_us_with_reorder"] * 1e-6),
                                "note": "one call of reorder_every sweeps, holding one spatial chain reorder "
                                        "(the timed runs of K < reorder_every sweeps hold none)"}
                               if "sweep_us_with_reorder" in main_res else None),
        "timed_runs_s": main_res["runs_s"],
        "paper_soma": PAPER_SOMA,
    }
    print("[bench] atomic-rate calibration", flush=True)
    peak_atomics = atomic_calibration()
    atom = {"calibrated_peak_per_s": peak_atomics,
            "calibration": "torch index_add_ of 2^23 ones at random words of an 8 MiB int32 array"}
    if prof and prof.get("atomics_per_sweep"):
        kern_s = prof["k_sweep_avg_ns"] * 1e-9
        atom.update({"atomics_per_sweep": prof["atomics_per_sweep"],
                     "achieved_per_s": prof["atomics_per_sweep"] / kern_s,
                     "frac": prof["atomics_per_sweep"] / kern_s / peak_atomics,
                     "source": "TCC_ATOMIC_sum and the sweep kernel's duration from the committed rocprofv3 summary"})
    out["roofline"]["atomics"] = atom

    if not args.no_plain and args.workload in ("batched_mixed", "batched_uneven"):
        print("[bench] batched vs plain: every system alone", flush=True)
        alone = sequential_alone(args.workload, args.steps, args.warmup, autotune, args.runs)
        import numpy as np
        d = float(np.abs(np.array(main_res["re2"]) - np.array(alone["re2"])).max())
        print("[bench] batched vs plain: plain single-system FP32 form (131072 chains, N=32)", flush=True)
        plain = run_workload("plain_large", args.steps, args.warmup, autotune=autotune, runs=args.runs)
        out["batched_vs_plain"] = {
            "same_systems_alone": {"moves_per_s": alone["moves_per_s"], "systems": alone["systems"],
                                   "batched_over_alone": main_res["moves_per_s"] / alone["moves_per_s"],
                                   "re2_max_abs_diff": d, "autotuned_each": alone["autotuned_each"],
                                   "tunes_from_cache": alone["tunes_from_cache"]},
            "plain_single_system_fp32": {"workload": "plain_large", "beads": plain["beads"],
                                         "moves_per_s": plain["moves_per_s"],
                                         "batched_over_plain": main_res["moves_per_s"] / plain["moves_per_s"],
                                         "re2": plain["re2"][0], "launch_shape": plain["launch_shape"],
                                         "roofline_frac": roofline_of(plain)["frac"]},
            "matched_re2": "same systems alone: the same random numbers (sys_id_base), so the same "
                           "trajectory; re2_max_abs_diff above checks it and is 0.0 when every system's Re^2 is "
                           "bit-identical; plain FP32 form: its representation error (1.5e-5 relative Re^2 "
                           "against FP64 positions) exceeds the cell form's (1.1e-10)",
        }
    if not args.no_extra:
        legs = {}
        for name, steps, warm in (("plain_small", 1000, 50), ("mixed_large", min(args.steps, 100), 10),
                                  ("batched_uneven", min(args.steps, 200), 10),
                                  ("plain_large_smc", min(args.steps, 200), 10)):
            print(f"[bench] leg {name}", flush=True)
            r = run_workload(name, steps, warm, autotune=autotune, runs=args.runs)
            legs[name] = {"beads": r["beads"], "systems": r["systems"], "sweeps": steps,
                          "moves_per_s": r["moves_per_s"], "sweep_us": r["sweep_us"],
                          "roofline_frac": roofline_of(r)["frac"], "launch_shape": r["launch_shape"],
                          "accept_ratio": r["obs0"]["accept_ratio"], "re2_system0": r["re2"][0]}
            if name == "batched_uneven":
                print("[bench] leg batched_uneven: every system alone", flush=True)
                al = sequential_alone(name, steps, warm, autotune, args.runs)
                import numpy as np
                legs[name]["alone_moves_per_s"] = al["moves_per_s"]
                legs[name]["batched_over_alone"] = r["moves_per_s"] / al["moves_per_s"]
                legs[name]["re2_max_abs_diff"] = float(np.abs(np.array(r["re2"]) - np.array(al["re2"])).max())
        out["legs"] = legs
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
        out["gpu_over_cpu_oracle"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
