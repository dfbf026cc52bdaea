"""Benchmark: SA moves/s on normalized Schwefel n=100 (65536 chains, FP32,
500 levels x 100 steps, seed 1) on one MI355X.

One step = one whole annealing run (level-0 start, 500 levels, argmin and
broadcast after each) from a reset context; the inputs are the problem
definition, already on the device.  Prints one JSON line.

Also reported (unless --no-ttt): time to |f - f*| < 1e-4 on the same
problem, plain radius moves against the learned proposal (network trained on
the GPU from accepted moves of plain runs), on the schedule extended to 8000
levels, from random starts and from a final-approach start.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-levels L] [--no-cpu] [--probe] [--no-ttt]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

# ALU roofline.  Unit: one "slot" = one lane-operation at the FP32 FMA issue
# rate.  Peak: MI355X FP32 vector 157.3 TFLOP/s = 78.6e12 lane-FMA/s.  An
# instruction class that issues r times slower than FMA costs r slots; r comes
# from the issue-rate probe (libsa_peak.so, bench.py --probe; output kept in
# profiles/valu_issue_rates.md) on MI355X: the ratio of the class's rate to
# the FMA rate at 8 waves per SIMD where the probe sweeps occupancy (FMA
# 5.43e13, v_mad_u64_u32 1.78e13, v_sin_f32 1.77e13 lane-ops/s), else with
# the grid full (FMA 5.63e13, v_mul_hi_u32 1.99e13, v_sqrt_f32 1.91e13,
# v_exp_f32 1.89e13):
#   v_mad_u64_u32 3.05, v_mul_hi_u32 2.83, v_sin/v_cos/v_sqrt/v_exp_f32 3.0,
#   FP32 add/mul/fma/med3/cvt, integer shift/xor/bitop3/compare/select 1.
# Algorithmic work of one FP32 normalized-Schwefel move with the radius rule:
CLOCK_HZ = 2.4e9  # MI355X peak engine clock
SLOT_WEIGHT = {"mad_u64": 3.05, "mul_hi": 2.83, "trans": 3.0, "valu": 1.0}
SLOTS_PER_MOVE = {
    # counter-based generator: a move takes three of a block's four words, so
    # 3/4 of a block per move.  Of Philox4x32-10's ten rounds, rounds 3-10
    # depend on the block counter in every word (two 32x32->64 multiplies and
    # two three-input XORs each); rounds 1-2 leave two counter-dependent XORs,
    # the rest is fixed per chain and level
    "philox": 0.75 * (16 * SLOT_WEIGHT["mad_u64"] + 16 * 1 + 2 * 1),
    "coordinate_pick": SLOT_WEIGHT["mul_hi"],                 # high word of r0 * n
    "uniforms": 2 * 3,                                        # (r >> 8), convert, scale; twice
    "neighbour": 3,                                           # 2u - 1, fma, clamp (med3)
    "increment": 2 * (2 * SLOT_WEIGHT["trans"] + 2) + 2,      # per term sqrt, sin, two muls; difference, 1/n
    "metropolis": 1 + SLOT_WEIGHT["trans"] + 1,               # scale, exp2, compare
    "commit": 3,                                              # state select, cost select-add, accept count
    "lds_address": 1,
}
SLOTS = sum(SLOTS_PER_MOVE.values())
PEAK_SLOTS_PER_S = 157.3e12 / 2.0

# HBM traffic of one level launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# (KiB per dispatch), each scaled by the counter's reading for a plain 1 GiB
# device copy (FETCH_SIZE reads 0.5x the bytes moved, WRITE_SIZE 1.0x); see
# profiles/level_kernel_schwefel_n100_fp32.md.  Valid only for the kernel
# sources it was measured on (hash below); otherwise reported as null.
TRAFFIC_MEASURED = {"sources_sha256_16": "514386df92a4c560", "fetch_kib": 174.960, "fetch_scale": 2.0,
                    "write_kib": 120.592, "write_scale": 1.0}
# Instruction counters of one level launch (rocprofv3 --pmc SQ_INSTS_VALU
# SQ_INSTS_VALU_TRANS_F32, wave-instructions per dispatch, same sources):
# with the live launch time they give the lane-operation issue rate, set
# against the probe's full-grid FP32 FMA rate and v_sin_f32 rate.
COUNTERS_MEASURED = {"sources_sha256_16": "514386df92a4c560", "insts_valu": 6.379e6, "insts_trans": 5.12e5,
                     "fma_rate": 5.625e13, "trans_rate": 1.824e13}
KERNEL_SOURCES = ["paper_2408_00018_amd/csrc/sa_kernels.hip", "paper_2408_00018_amd/csrc/sa_level_kernel.hpp",
                  "paper_2408_00018_amd/csrc/sa_device.hpp", "paper_2408_00018_amd/csrc/sa_internal.hpp",
                  "paper_2408_00018_amd/csrc/sa_step.hpp", "paper_2408_00018_amd/csrc/sa_level_common.hpp",
                  "paper_2408_00018_amd/csrc/sa_mlp_net.hpp", "paper_2408_00018_amd/build.py"]


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic_bytes():
    t = TRAFFIC_MEASURED
    if kernel_sources_hash() != t["sources_sha256_16"]:
        return None
    return round((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0)


def counter_issue_fractions(avg_launch_s):
    """Measured VALU and transcendental lane-op issue rates of the level
    kernel over the probe's rates, or None once the sources have changed."""
    c = COUNTERS_MEASURED
    if kernel_sources_hash() != c["sources_sha256_16"]:
        return None
    valu = c["insts_valu"] * 64 / avg_launch_s
    trans = c["insts_trans"] * 64 / avg_launch_s
    return {"valu_lane_ops_per_s": float(f"{valu:.4g}"), "valu_issue_frac": round(valu / c["fma_rate"], 4),
            "trans_lane_ops_per_s": float(f"{trans:.4g}"), "trans_issue_frac": round(trans / c["trans_rate"], 4)}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--cpu-levels", type=int, default=10, help="levels of the workload the CPU oracle times")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--probe", action="store_true", help="also measure VALU issue rates")
    p.add_argument("--no-ttt", action="store_true", help="skip the time-to-target comparison")
    p.add_argument("--no-extra", action="store_true", help="skip the large-n and batched throughput figures")
    p.add_argument("--only-extra", action="store_true",
                   help="run only the other workloads' throughput figures (no bench line; for counter passes)")
    p.add_argument("--learned-levels", type=int, default=0,
                   help="only run this many learned-mixture levels of the bench workload (untrained network; "
                        "for counter passes)")
    p.add_argument("--train-steps", type=int, default=0,
                   help="only collect the time-to-target records and run this many training steps (for profiles)")
    p.add_argument("--gauss", action="store_true",
                   help="with --learned-levels: the GELU/Gaussian network kind instead of relu/Cauchy")
    p.add_argument("--ttt-seeds", type=int, default=10, help="seeds per arm of the time-to-target comparison")
    p.add_argument("--exchange-sweep", action="store_true",
                   help="bench workload with the winner broadcast every level, every 10 levels and never")
    p.add_argument("--no-paper-tables", action="store_true",
                   help="skip the paper's V2/V1 setting (Schwefel n=8..512, 16384 chains, T0=1000, rho=0.99, "
                        "1146 levels) and the V0 sample")
    p.add_argument("--wave-sweep", action="store_true",
                   help="cost of a wave's move at 1, 2 and 3 waves per SIMD (Schwefel n=40)")
    p.add_argument("--level-sweep", action="store_true",
                   help="also time the bench workload's level at 1-100 steps and fit fixed + per-step cost")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device copy (torch) three times, to scale HBM byte counters")
    return p.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, levels):
    """The FP64 oracle on the host's cores: the first `levels` levels of the
    workload single-threaded, then the first 4 x `levels` levels with one
    thread per usable core (chains of a level split over threads; the results
    are identical for every thread count).  `value` is the all-core rate."""
    import oracle
    oracle.build(force=False)
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    # at most the 16 cores a one-GPU share of the host has
    threads = max(1, min(usable, 16))

    def timed(nthreads, nlev):
        oracle.set_threads(nthreads)
        t0 = time.perf_counter()
        oracle.sa_run(wl.func, wl.lower, wl.upper, wl.shift, seed=wl.seed, chains=wl.chains, steps=wl.steps,
                      T0=wl.T0, alpha=wl.alpha, levels=nlev, radius_frac=wl.radius_frac, keep_x_best=False)
        return time.perf_counter() - t0

    v0 = v0_sample(oracle)
    dt1 = timed(1, levels)
    all_levels = 4 * levels
    dtn = timed(threads, all_levels)
    oracle.set_threads(1)
    per_level = wl.chains * wl.steps
    single = {"value": per_level * levels / dt1, "unit": "moves/s", "cores": 1,
              "sample": f"first {levels} of {wl.levels} levels, all {wl.chains} chains x {wl.steps} steps, "
                        f"FP64, one thread, {dt1:.1f} s"}
    return {"value": per_level * all_levels / dtn, "unit": "moves/s", "cores": threads, "kind": "oracle",
            "sample": f"first {all_levels} of {wl.levels} levels, all {wl.chains} chains x {wl.steps} steps, FP64, "
                      f"{threads} threads over the chains of each level, {dtn:.1f} s",
            "single_thread": single, "usable_cpus": usable, "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "v0": v0}


PAPER_LEVELS = math.ceil(math.log(0.01 / 1000.0) / math.log(0.99))  # T_k > T_min = 0.01 for k < 1146
PAPER_CHAINS, PAPER_STEPS = 16384, 100
PAPER_NS = (8, 16, 32, 64, 128, 256, 512)


def v0_sample(oracle):
    """The paper's sequential version V0 (Sec. 4.1) at its comparison setting:
    one chain performing the same number of moves as the parallel versions
    (16384 chains x 1146 levels x 100 steps = 1.8776e9), here the FP64 oracle
    on one thread.  Timed on a sample -- one level of 16384 x 100 moves of the
    single chain at T0 = 1000 (whole-interval resampling moves, normalized
    Schwefel on +-500) for each n -- and scaled to the full move count."""
    total = PAPER_CHAINS * PAPER_LEVELS * PAPER_STEPS
    oracle.set_threads(1)
    rows = []
    for n in PAPER_NS:
        lo, hi = np.full(n, -500.0), np.full(n, 500.0)
        t0 = time.perf_counter()
        oracle.sa_run(W.SCHWEFEL, lo, hi, None, seed=1, chains=1, steps=PAPER_CHAINS * PAPER_STEPS, T0=1000.0,
                      alpha=0.99, levels=1, move_rule=oracle.MOVE_RESAMPLE, keep_x_best=False)
        dt = time.perf_counter() - t0
        rate = PAPER_CHAINS * PAPER_STEPS / dt
        rows.append({"n": n, "moves_per_s": float(f"{rate:.4g}"), "seconds_for_all_moves": round(total / rate, 2)})
    return {"moves": total, "sample": f"one level of {PAPER_CHAINS * PAPER_STEPS} moves per n, FP64, one thread",
            "rows": rows}


def probe_rates():
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2408_00018_amd", "libsa_peak.so"))
    lib.sa_peak_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
    names = ["fma_f32", "mad_u64_u32", "mul_hi_u32", "xor", "sin_f32", "sqrt_f32", "exp2_f32", "fma_f64"]
    out = {}
    blocks, iters = 8192, 2048
    for k, name in enumerate(names):
        ms = ctypes.c_float()
        rc = lib.sa_peak_probe(k, blocks, iters, ctypes.byref(ms))
        if rc != 0:
            raise RuntimeError(f"probe {name} failed: {rc}")
        ops = blocks * 256 * iters * 16
        out[name] = ops / (ms.value * 1e-3)
    rates = {k: float(f"{v:.4g}") for k, v in out.items()}
    lib.sa_peak_probe_occupancy.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
    occ = {}
    for k, name in ((0, "fma_f32"), (1, "mad_u64_u32"), (4, "sin_f32")):
        for w in (1, 2, 4, 8):
            ms = ctypes.c_float()
            rc = lib.sa_peak_probe_occupancy(k, w, 4096, ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError(f"occupancy probe {name}/{w} failed: {rc}")
            occ[f"{name}@{w}w"] = float(f"{256 * 4 * w * 64 * 4096 * 16 / (ms.value * 1e-3):.4g}")
    return {"rates_many_waves": rates, "by_waves_per_simd": occ}


WRITTEN_CAP = 1000  # levels the written-configuration arms may run past their first learned level


def time_to_target_report(wl, seeds):
    """Learned vs plain proposal: time until the record is within 1e-4 of f*.

    Collection: plain runs (4096 chains, 100 steps, T0 10, alpha 0.995, 4000
    levels, seed 1001) capture accepted moves at every 8th level, 20000 per
    level (repeated where fewer were accepted): 10^7 records.  Training: 6000 Adam steps,
    minibatch 4096, lr 1e-3.  Arms, on 65536 chains x 100 steps,
    T_k = 10 * 0.995^k up to k = 7999: 'full' starts at level 0 from random
    points; 'final_approach' starts at level 3000 (T = 2.9e-6, where the thermal
    gap n T / 2 = 1.5e-4 is at the target's scale) with every chain at
    x* + U(-2, 2) per coordinate.  Arms: plain radius moves, plain
    whole-interval resampling moves, the learned mixture from the first
    level, and (full regime) 'learned_late': plain moves until the first level
    whose thermal gap n T / 2 is at most the target, the learned mixture from
    there on.  Each arm runs `seeds` seeds; the summary gives hit fractions,
    median times and the learned / plain ratios of median times.

    The learned-proposal configuration as written (GELU/Gaussian network,
    ln T and raw history features, trained on every accepted move of n = 4
    Schwefel runs in FP64 -- 256 chains, T0 10, alpha 0.99, 200 levels x 50
    steps -- seed after seed until 10^7 records; 6000 Adam steps, minibatch
    4096) runs as two more arms, 'written' in the final-approach regime and
    'written_late' (from the same switch level as 'learned_late') in the full
    one, each capped at WRITTEN_CAP levels past its first learned level (its
    step costs ~3x the relu network's).
    """
    import torch
    from paper_2408_00018_amd import learned as Lp
    from paper_2408_00018_amd import sa
    levels = 8000
    out = {"target": 1e-4, "f_star": W.SCHWEFEL_F_STAR, "levels_cap": levels}
    t0 = time.perf_counter()
    col = sa.Schedule(chains=4096, levels=4000, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=1001,
                      precision=sa.FP32)
    rec = Lp.collect(wl.func, wl.lower, wl.upper, wl.shift, col, every=8, per_level=20000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    params, trace = Lp.train(rec, steps=6000, batch=4096, lr=1e-3, seed=0)
    t2 = time.perf_counter()
    out["collect"] = {"records": int(rec.shape[0]), "seconds": round(t1 - t0, 3)}
    out["train"] = {"steps": 6000, "batch": 4096, "loss_first": float(trace[:20].mean()),
                    "loss_last": float(trace[-50:].mean()), "seconds": round(t2 - t1, 3)}
    del rec
    t3 = time.perf_counter()
    cfg1 = W.schwefel_n4_fp64()
    col1 = sa.Schedule(chains=cfg1.chains, levels=cfg1.levels, steps=cfg1.steps, T0=cfg1.T0, alpha=cfg1.alpha,
                       seed=cfg1.seed, precision=sa.FP64)
    rec1, runs1 = Lp.collect_runs(cfg1.func, cfg1.lower, cfg1.upper, cfg1.shift, col1, records=10_000_000,
                                  kind=sa.NET_GELU_GAUSS)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    params_w, trace_w = Lp.train(rec1, steps=6000, batch=4096, lr=1e-3, seed=0, kind=sa.NET_GELU_GAUSS)
    t5 = time.perf_counter()
    out["written"] = {"records": int(rec1.shape[0]), "runs": runs1, "collect_seconds": round(t4 - t3, 3),
                      "loss_first": float(trace_w[:20].mean()), "loss_last": float(trace_w[-50:].mean()),
                      "train_seconds": round(t5 - t4, 3), "cap_levels": WRITTEN_CAP}
    del rec1
    rng = np.random.default_rng(7)
    x0 = W.SCHWEFEL_X_STAR + rng.uniform(-2, 2, wl.n)
    # 'learned_late': plain moves until the thermal gap n T / 2 has fallen to the
    # target, the learned mixture from there on
    k_late = int(math.ceil(math.log(2.0 * 1e-4 / (wl.n * wl.T0)) / math.log(wl.alpha)))
    out["learned_late_from_level"] = k_late
    for regime, start in (("full", 0), ("final_approach", 3000)):
        res = {}
        relu, gauss = sa.NET_RELU_CAUCHY, sa.NET_GELU_GAUSS
        arms = [("plain", None, 0, sa.MOVE_RADIUS, relu, levels),
                ("plain_resample", None, 0, sa.MOVE_RESAMPLE, relu, levels),
                ("learned", params, 0, sa.MOVE_RADIUS, relu, levels)]
        if start == 0:
            arms.append(("learned_late", params, k_late, sa.MOVE_RADIUS, relu, levels))
            arms.append(("written_late", params_w, k_late, sa.MOVE_RADIUS, gauss, k_late + WRITTEN_CAP))
        else:
            arms.append(("written", params_w, 0, sa.MOVE_RADIUS, gauss, start + WRITTEN_CAP))
        for arm, p, learn_from, move, kind, cap in arms:
            runs = []
            for seed in range(1, seeds + 1):
                sched = sa.Schedule(chains=wl.chains, levels=cap, steps=wl.steps, T0=wl.T0, alpha=wl.alpha,
                                    seed=seed, precision=sa.FP32, move=move)
                r = Lp.time_to_target(wl.func, wl.lower, wl.upper, wl.shift, sched, W.SCHWEFEL_F_STAR, 1e-4,
                                      params=p, eps=0.1, start_level=start, x_start=x0 if start else None,
                                      learn_from=learn_from, kind=kind)
                runs.append({"seed": seed, "hit": r.hit, "level": r.level, "seconds": r.seconds,
                             "levels_run": r.levels_run, "ms_per_level": round(r.ms_per_level, 4),
                             "final_gap": r.final_gap})
                print(f"[ttt] {regime} {arm} seed {seed}: {runs[-1]}", file=sys.stderr, flush=True)
            res[arm] = runs
        summary = {}
        for a in [arm[0] for arm in arms]:
            secs = [r["seconds"] for r in res[a] if r["hit"]]
            summary[a] = {"hit_fraction": len(secs) / len(res[a]),
                          "median_seconds": float(np.median(secs)) if secs else None,
                          "median_final_gap": float(np.median([r["final_gap"] for r in res[a]]))}
        # learned / plain speedups: median seconds to the target of each plain
        # arm that hits it, over that of each learned arm
        for pa in ("plain", "plain_resample"):
            for la in ("learned", "learned_late", "written", "written_late"):
                if la in summary and summary[pa]["median_seconds"] and summary[la]["median_seconds"]:
                    summary[f"speedup_{la}_vs_{pa}"] = summary[pa]["median_seconds"] / summary[la]["median_seconds"]
        if "learned_late" in summary and summary["learned"]["median_seconds"] and \
                summary["learned_late"]["median_seconds"]:
            summary["late_vs_learned_median"] = (summary["learned"]["median_seconds"] /
                                                 summary["learned_late"]["median_seconds"])
        res["summary"] = summary
        out[regime] = res
    return out


def extra_workloads():
    """Throughput of the other workloads, one timed run each after a warm-up
    run (graph-replayed levels, HIP events on the library's stream): the
    n = 512 Rastrigin and n = 1024 Ackley runs (131072 chains, 1000 levels x
    64 steps, shifted), the n = 100 Griewank run (65536 chains, 200 levels x
    100 steps; non-separable: every move re-evaluates f in full), the n = 100
    Schwefel run with a full evaluation of f per move as the paper's kernel
    does (SA_FLAG_FULL_EVAL) instead of the increment, the Shekel (m = 10,
    n = 4) and foxholes (n = 5) runs (65536 chains, 200 levels x 100 steps;
    centre families, evaluated in full per move), and 1024
    batched problems (n ~ U{2..256}, 500 levels
    x 64 steps, chains per problem and waves per workgroup from the
    autotuner)."""
    import torch
    from paper_2408_00018_amd import sa
    out = {}
    full_eval = W.schwefel_n100_fp32().with_(name="schwefel_n100_fp32_full_eval")
    for wl in (W.rastrigin_n512_fp32(), W.ackley_n1024_fp32(), W.griewank_n100_fp32(), full_eval,
               W.shekel10_n4_fp32(), W.foxholes_n5_fp32()):
        sched = sa.Schedule(chains=wl.chains, levels=wl.levels, steps=wl.steps, T0=wl.T0, alpha=wl.alpha,
                            seed=wl.seed, precision=sa.FP32, graph=True, full_eval=wl is full_eval)
        with sa.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
            ann.run()
            ann.reset(wl.seed)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(ann.stream)
            ann.run()
            e1.record(ann.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            _, f_rec, _ = ann.best()
            wg, slots, tiles = ann.layout()
        out[wl.name] = {"moves_per_s": float(f"{wl.moves / (ms * 1e-3):.4g}"), "ms_per_run": round(ms, 3),
                        "workgroup": wg, "overlay_slots": slots, "gap_to_f_star": f_rec - wl.f_star}
        print(f"[extra] {wl.name}: {out[wl.name]}", file=sys.stderr, flush=True)
    probs = W.batch_problems()
    bs = sa.BatchSchedule(levels=500, steps=64, T0=10.0, alpha=0.99, seed=4, precision=sa.FP32, graph=True)
    t0 = time.perf_counter()
    chains, wpg, rate = sa.batch_autotune(probs, bs, trial_levels=4)
    tune_s = time.perf_counter() - t0
    bs.waves_per_group = wpg
    with sa.BatchAnnealer(probs, chains, schedule=bs) as b:
        b.run()
        b.reset(4)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(b._stream)
        b.run()
        e1.record(b._stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        # per-family hit rates of the timed run's records (f* = Schwefel's
        # minimum, 0 for Rastrigin and Ackley; every shift keeps the minimiser
        # inside its box)
        names = {W.SCHWEFEL: "schwefel", W.RASTRIGIN: "rastrigin", W.ACKLEY: "ackley"}
        gaps = {}
        for p_i, (func, _, _, _) in enumerate(probs):
            _, f_rec, _ = b.best(p_i)
            gaps.setdefault(names[func], []).append(f_rec - (W.SCHWEFEL_F_STAR if func == W.SCHWEFEL else 0.0))
        families = {k: {"problems": len(v), "hit_1e-4": round(float(np.mean(np.array(v) < 1e-4)), 4),
                        "hit_1e-2": round(float(np.mean(np.array(v) < 1e-2)), 4),
                        "median_gap": float(f"{np.median(v):.4g}")} for k, v in sorted(gaps.items())}
        idle = batch_idle(b, chains, first=100, levels=50)
    moves = float(np.sum(chains.astype(np.float64))) * bs.steps * bs.levels
    out["batched_1024"] = {"moves_per_s": float(f"{moves / (ms * 1e-3):.4g}"), "ms_per_run": round(ms, 3),
                           "problems": len(probs), "total_chains": int(np.sum(chains)),
                           "chains_per_problem": sorted({int(c) for c in chains}), "waves_per_group": wpg,
                           "autotune_s": round(tune_s, 2), "families": families, "idle": idle}
    print(f"[extra] batched: {out['batched_1024']}", file=sys.stderr, flush=True)
    return out


def train_only(wl, steps, kind=0):
    """The time-to-target comparison's collection (relu kind) and `steps`
    Adam steps at minibatch 4096 on it, timed (for the training kernels'
    profiles)."""
    import torch
    from paper_2408_00018_amd import learned as Lp
    from paper_2408_00018_amd import sa
    col = sa.Schedule(chains=4096, levels=4000, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=1001,
                      precision=sa.FP32)
    rec = Lp.collect(wl.func, wl.lower, wl.upper, wl.shift, col, every=8, per_level=20000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    params, trace = Lp.train(rec, steps=steps, batch=4096, lr=1e-3, seed=0, kind=kind)
    dt = time.perf_counter() - t0
    return {"records": int(rec.shape[0]), "steps": steps, "seconds": round(dt, 4),
            "us_per_step": round(1e6 * dt / steps, 2), "loss_first": float(trace[:20].mean()),
            "loss_last": float(trace[-20:].mean())}


def batch_idle(b, chains, first, levels):
    """Where a batched level's time goes, from the device wall clock of every
    64-chain tile (sa_batch_clock) over levels [first, first + levels) of one
    more run.  Per level: `idle_fraction` = 1 - (sum of the tiles' busy times)
    / (peak number of tiles running at once x level span): the share of the
    level's wave slots left empty while the level waits for its last tiles
    (what a launch that let problems run ahead could fill); `problem_wait` =
    1 - mean over problems of (end of its last tile - level start) / level
    span: the share of the level a problem's results wait for the slowest
    problem; `peak_tiles` and `tile_us` = concurrency and mean busy time of a
    tile; `gap_us` = mean time from the last tile end of a level to the first
    tile start of the next (launch and hand-off).  Means over the levels."""
    import torch
    tiles = b.layout()["tiles"]
    ticks = torch.zeros((levels, tiles, 2), dtype=torch.int64, device="cuda")
    rate = b.clock(ticks, first, levels)
    b.reset(4)
    b.run()
    torch.cuda.synchronize()
    b.clock(None)
    t = ticks.cpu().numpy().astype(np.float64) / rate
    owner = np.repeat(np.arange(len(chains)), np.asarray(chains) // 64)
    idle, wait, peak, tile_s, spans, gaps = [], [], [], [], [], []
    for k in range(levels):
        start, end = t[k, :, 0].min(), t[k, :, 1].max()
        span = end - start
        busy = t[k, :, 1] - t[k, :, 0]
        ev = np.concatenate([np.stack([t[k, :, 0], np.ones(tiles)], 1), np.stack([t[k, :, 1], -np.ones(tiles)], 1)])
        ev = ev[np.lexsort((ev[:, 1], ev[:, 0]))]  # ends before starts at equal times
        pk = float(np.max(np.cumsum(ev[:, 1])))
        idle.append(1.0 - busy.sum() / (pk * span))
        p_end = np.zeros(len(chains))
        np.maximum.at(p_end, owner, t[k, :, 1])
        wait.append(1.0 - np.mean(p_end - start) / span)
        peak.append(pk)
        tile_s.append(busy.mean())
        spans.append(span)
        if k + 1 < levels:
            gaps.append(t[k + 1, :, 0].min() - end)
    return {"levels": [first, first + levels], "idle_fraction": round(float(np.mean(idle)), 4),
            "problem_wait": round(float(np.mean(wait)), 4), "peak_tiles": int(round(np.mean(peak))),
            "tile_us": round(1e6 * float(np.mean(tile_s)), 2), "level_span_us": round(1e6 * float(np.mean(spans)), 2),
            "gap_us": round(1e6 * float(np.mean(gaps)), 2)}


def learned_levels(wl, levels, kind=0):
    """`levels` learned-mixture levels (eps = 0.1, untrained network from
    learned.init_params, network kind `kind`) of the bench workload,
    graph-replayed: device ms per level (used to take counters of the learned
    level kernel)."""
    import torch
    from paper_2408_00018_amd import learned as Lp
    from paper_2408_00018_amd import sa
    sched = sa.Schedule(chains=wl.chains, levels=levels, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=wl.seed,
                        precision=sa.FP32, graph=True, learned=True)
    with sa.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
        ann.set_network_kind(kind)
        ann.set_proposal(Lp.init_params(0), 0.1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ann.stream)
        ann.run()
        e1.record(ann.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
    return {"levels": levels, "kind": "gelu_gauss" if kind else "relu_cauchy", "ms_per_level": round(ms / levels, 4),
            "moves_per_s": float(f"{wl.chains * wl.steps * levels / (ms * 1e-3):.4g}")}


def us_per_level(wl, chains, steps, levels=100):
    """Best of three graph-replayed runs of `levels` plain FP32 levels of
    workload `wl` with the given chain and step counts: microseconds per level."""
    import torch
    from paper_2408_00018_amd import sa
    sched = sa.Schedule(chains=chains, levels=levels, steps=steps, T0=wl.T0, alpha=wl.alpha, seed=wl.seed,
                        precision=sa.FP32, graph=True)
    with sa.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
        ann.reset(wl.seed)
        ann.run()
        torch.cuda.synchronize()
        best = math.inf
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(ann.stream)
            ann.reset(wl.seed)
            ann.run()
            e1.record(ann.stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e3 / levels)
    return best


def level_sweep(wl):
    """Per-level time of the bench workload's shape at several step counts
    (graph-replayed runs of 100 levels), and the least-squares line through
    them: its intercept is the fixed cost of a level launch (hand-off, tile
    start, level end, launch gap), its slope the cost of one step of all
    chains."""
    pts = [(steps, us_per_level(wl, wl.chains, steps)) for steps in (1, 25, 50, 75, 100)]
    x = np.array([p[0] for p in pts], dtype=np.float64)
    y = np.array([p[1] for p in pts], dtype=np.float64)
    slope, icpt = np.polyfit(x, y, 1)
    return {"us_per_level": {str(int(a)): round(b, 3) for a, b in pts}, "fixed_us_per_level": round(float(icpt), 3),
            "us_per_step": round(float(slope), 4)}


def exchange_sweep(wl, reps=3):
    """The bench workload with the winner broadcast every level (the
    synchronous scheme), every 10 levels (periodic exchange) and never (the
    asynchronous scheme, Sec. 2.2.1): device time per 500-level run (best of
    `reps` graph replays), moves/s and the final gap to f*."""
    import torch
    from paper_2408_00018_amd import sa
    out = {}
    for name, k in (("every_level", 1), ("every_10_levels", 10), ("never", 0)):
        sched = sa.Schedule(chains=wl.chains, levels=wl.levels, steps=wl.steps, T0=wl.T0, alpha=wl.alpha,
                            seed=wl.seed, precision=sa.FP32, graph=True, exchange=k)
        with sa.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
            ann.reset(wl.seed)
            ann.run()
            torch.cuda.synchronize()
            best = math.inf
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(ann.stream)
                ann.reset(wl.seed)
                ann.run()
                e1.record(ann.stream)
                e1.synchronize()
                best = min(best, e0.elapsed_time(e1))
            _, f_rec, lvl = ann.best()
        out[name] = {"exchange": k, "ms_per_run": round(best, 3),
                     "moves_per_s": float(f"{wl.moves / (best * 1e-3):.4g}"), "f_rec": f_rec,
                     "gap_to_f_star": f_rec - W.SCHWEFEL_F_STAR, "rec_level": lvl}
    return out


def paper_tables(seed=1):
    """The paper's own comparison setting (Sec. 4: T0 = 1000, T_min = 0.01,
    rho = 0.99, i.e. 1146 levels, N = 100 steps, 16384 chains, normalized
    Schwefel n = 8 ... 512, FP32): the synchronous scheme (V2, a broadcast at
    every level) and the asynchronous one (V1, no exchange), each with the
    radius move and with the whole-interval resample move (the two readings
    of the paper's neighbour), each one run after a warm-up; device time,
    moves/s, |f_a - f*| and the relative error ||x_a - x*|| / ||x*|| of the
    record."""
    import torch
    from paper_2408_00018_amd import sa
    levels = PAPER_LEVELS
    out = {"levels": levels, "steps": PAPER_STEPS, "chains": PAPER_CHAINS, "T0": 1000.0, "alpha": 0.99, "rows": []}
    for n in PAPER_NS:
        lo, hi = np.full(n, -500.0), np.full(n, 500.0)
        x_star = np.full(n, W.SCHWEFEL_X_STAR)
        for name, k, move in (("V2", 1, sa.MOVE_RADIUS), ("V1", 0, sa.MOVE_RADIUS), ("V2", 1, sa.MOVE_RESAMPLE),
                              ("V1", 0, sa.MOVE_RESAMPLE)):
            sched = sa.Schedule(chains=16384, levels=levels, steps=100, T0=1000.0, alpha=0.99, seed=seed,
                                precision=sa.FP32, graph=True, exchange=k, move=move)
            with sa.Annealer(W.SCHWEFEL, lo, hi, None, schedule=sched) as ann:
                ann.reset(seed)
                ann.run()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(ann.stream)
                ann.reset(seed)
                ann.run()
                e1.record(ann.stream)
                e1.synchronize()
                ms = e0.elapsed_time(e1)
                x, f, _ = ann.best()
                wg, ov, _ = ann.layout()
            moves = 16384 * levels * 100
            out["rows"].append({"n": n, "scheme": name, "move": "radius" if move == sa.MOVE_RADIUS else "resample",
                                "seconds": round(ms * 1e-3, 5),
                                "moves_per_s": float(f"{moves / (ms * 1e-3):.4g}"),
                                "abs_err_f": float(f"{abs(f - W.SCHWEFEL_F_STAR):.4g}"),
                                "rel_err_x": float(f"{np.linalg.norm(x - x_star) / np.linalg.norm(x_star):.4g}"),
                                "layout": "overlay" if ov else f"dense, {wg} chains per workgroup"})
            print(f"[paper tables] n={n} {name}: {out['rows'][-1]}", flush=True)
    return out


def wave_sweep():
    """Cost of a move of one wave with 1, 2 and 3 waves per SIMD: Schwefel at
    n = 40 (three 256-chain workgroups fit one CU's LDS) with 65536, 131072 and
    196608 chains; the per-step time is the difference between 100-step and
    1-step levels.  Shows how much of the SIMD one wave leaves unused."""
    lo, hi = np.full(40, -500.0), np.full(40, 500.0)
    wl = W.Workload("schwefel_n40_fp32", W.SCHWEFEL, 40, lo, hi, None, chains=65536, levels=100, steps=100,
                    T0=10.0, alpha=0.995, seed=1, precision=W.FP32)
    out = {}
    for waves in (1, 2, 3):
        chains = 65536 * waves
        t1, t100 = us_per_level(wl, chains, 1), us_per_level(wl, chains, 100)
        per_step = (t100 - t1) / 99.0
        out[str(waves)] = {"chains": chains, "us_per_level_1_step": round(t1, 3),
                           "us_per_level_100_steps": round(t100, 3), "us_per_step": round(per_step, 4),
                           "cycles_per_wave_move": round(per_step * 1e-6 * CLOCK_HZ / waves, 1)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the annealer runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2408_00018_amd import sa

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "copies": 3}), flush=True)
        return
    wl = W.schwefel_n100_fp32()
    if args.only_extra:
        print(json.dumps({"other_workloads": extra_workloads()}), flush=True)
        return
    if args.train_steps:
        print(json.dumps({"train": train_only(wl, args.train_steps, 1 if args.gauss else 0)}), flush=True)
        return
    if args.learned_levels:
        print(json.dumps({"learned_levels": learned_levels(wl, args.learned_levels, 1 if args.gauss else 0)}),
              flush=True)
        return
    sched = sa.Schedule(chains=wl.chains, levels=wl.levels, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=wl.seed,
                        precision=sa.FP32, graph=True)
    ann = sa.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched)
    stream = ann.stream
    for _ in range(args.warmup):
        ann.reset(wl.seed)
        ann.run()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        ann.reset(wl.seed)
        ann.run()
    stop.record(stream)
    stop.synchronize()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    ms_per_step = ms / args.steps
    moves = wl.moves
    value = moves / (ms_per_step * 1e-3)
    x_rec, f_rec, lvl = ann.best()
    rec = ann.trace()
    ann.close()

    launches = args.steps * wl.levels
    avg_launch_s = ms * 1e-3 / launches
    per_launch = SLOTS * wl.chains * wl.steps
    achieved = per_launch / avg_launch_s
    roofline = {"bound": "alu", "achieved": round(achieved / 1e12, 3), "peak": round(PEAK_SLOTS_PER_S / 1e12, 3),
                "unit": "Tslot/s", "frac": round(achieved / PEAK_SLOTS_PER_S, 4), "traffic": measured_traffic_bytes(),
                "kernel": "level_kernel<float,Schwefel,uniform box,radius>", "slots_per_move": round(SLOTS, 2),
                "avg_launch_us": round(avg_launch_s * 1e6, 3), "counters": counter_issue_fractions(avg_launch_s)}
    out = {
        "metric": "SA moves/s (Schwefel n=100)",
        "value": float(f"{value:.6g}"),
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "func": "normalized_schwefel", "n": wl.n, "chains": wl.chains,
                   "levels": wl.levels, "steps": wl.steps, "T0": wl.T0, "alpha": wl.alpha, "seed": wl.seed,
                   "moves_per_step": moves},
        "roofline": roofline,
        "result": {"f_rec": f_rec, "gap_to_f_star": f_rec - W.SCHWEFEL_F_STAR, "rec_level": lvl,
                   "accept_rate": float(rec["accepts"].sum()) / moves},
    }
    if args.probe:
        out["valu_rates_per_s"] = probe_rates()
    if args.level_sweep:
        out["level_sweep"] = level_sweep(wl)
    if args.wave_sweep:
        out["wave_sweep"] = wave_sweep()
    if args.exchange_sweep:
        out["exchange_sweep"] = exchange_sweep(wl)
    if not args.no_paper_tables:
        out["paper_tables"] = paper_tables()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_levels)
        if "paper_tables" in out:
            # speedups over V0 as the paper's Table 2 gives them (its V0: one CPU core)
            v0 = {r["n"]: r["seconds_for_all_moves"] for r in out["cpu_baseline"]["v0"]["rows"]}
            for r in out["paper_tables"]["rows"]:
                r["speedup_vs_v0"] = round(v0[r["n"]] / r["seconds"], 1)
    if not args.no_extra:
        try:
            out["other_workloads"] = extra_workloads()
        except Exception as e:  # the throughput line is printed regardless
            out["other_workloads"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_ttt:
        try:
            out["time_to_target"] = time_to_target_report(wl, args.ttt_seeds)
        except Exception as e:  # the throughput line is printed regardless
            out["time_to_target"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
