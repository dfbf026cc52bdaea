"""Learned-proposal workflow on the device (an extension of the method; the
paper's moves are the plain radius/resample neighbours).

1. ``collect``: plain FP32 runs with capture switched on at every k-th level
   record accepted moves (features at the old state, accepted scaled
   displacement) across the whole temperature range, the same number from
   every captured level (acceptance falls by orders of magnitude as T drops,
   so levels with fewer accepted moves are repeated to the quota).
2. ``train``: Adam on the negative log-likelihood of those records (Cauchy
   for the relu network, Gaussian for the GELU one), on the GPU
   (``MLPTrainer``).  ``collect_runs`` captures every accepted move of whole
   runs over successive seeds instead (the learned-proposal configuration
   that trains the GELU/Gaussian network on small-problem runs).
3. ``time_to_target``: run a schedule with plain or learned moves and report
   the first level whose record is within ``target`` of f*, with its device
   time.

Every step runs in the library's kernels; this module only sequences calls.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import sa

MLP_INPUTS, MLP_HIDDEN = 6, 128


def init_params(seed: int = 0, sigma0: float = 0.01) -> np.ndarray:
    """He-normal hidden weights, small output weights, zero biases except the
    output log-scale, which starts at ln(sigma0)."""
    rng = np.random.default_rng(seed)
    H, I = MLP_HIDDEN, MLP_INPUTS
    W1 = rng.normal(0.0, math.sqrt(2.0 / I), (I, H))
    W2 = rng.normal(0.0, math.sqrt(2.0 / H), (H, H))
    W3 = rng.normal(0.0, 0.01 * math.sqrt(1.0 / H), (H, 2))
    b3 = np.array([0.0, math.log(sigma0)])
    p = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), b3])
    assert p.size == sa.MLP_PARAMS
    return p.astype(np.float32)


def collect(func, lower, upper, shift, schedule: sa.Schedule, every: int = 4, per_level: int = 2000,
            kind: int = sa.NET_RELU_CAUCHY):
    """Run `schedule` (plain moves) and capture the accepted moves of every
    `every`-th level: the first `per_level` of each, or all of them repeated
    up to `per_level` when there are fewer; features of network kind `kind`.
    Returns a float32 CUDA tensor [N, 7]."""
    import torch
    nlev = (schedule.levels + every - 1) // every
    rec = torch.empty((nlev * per_level, 7), dtype=torch.float32, device="cuda")
    off = 0
    sched = sa.Schedule(**{**schedule.__dict__, "graph": False, "learned": False, "log_chains": 0})
    with sa.Annealer(func, lower, upper, shift, schedule=sched) as ann:
        ann.set_network_kind(kind)
        level = 0
        while level < sched.levels:
            ann.capture(rec[off:off + per_level])
            ann.run(1)
            got = min(ann.capture_count(), per_level)
            ann.capture(None)
            if got:
                if got < per_level:
                    rep = off + torch.arange(per_level - got, device=rec.device) % got
                    rec[off + got:off + per_level] = rec[rep]
                off += per_level
            level += 1
            rest = min(every - 1, sched.levels - level)
            if rest:
                ann.run(rest)
                level += rest
    return rec[:off]


def collect_runs(func, lower, upper, shift, schedule: sa.Schedule, records: int, kind: int = sa.NET_RELU_CAUCHY,
                 first_seed: Optional[int] = None, max_runs: int = 1000):
    """Capture every accepted move of whole plain runs of `schedule`, seed
    after seed (from `first_seed`, default the schedule's), until `records`
    are stored (the last run's surplus is dropped).  Returns (float32 CUDA
    tensor [records, 7], runs used)."""
    import torch
    rec = torch.empty((records, 7), dtype=torch.float32, device="cuda")
    off, runs = 0, 0
    seed = schedule.seed if first_seed is None else first_seed
    while off < records and runs < max_runs:
        sched = sa.Schedule(**{**schedule.__dict__, "graph": False, "learned": False, "log_chains": 0, "seed": seed})
        with sa.Annealer(func, lower, upper, shift, schedule=sched) as ann:
            ann.set_network_kind(kind)
            ann.capture(rec[off:])
            ann.run()
            off += min(ann.capture_count(), records - off)
            ann.capture(None)
        seed += 1
        runs += 1
    return rec[:off], runs


def train(records, steps: int = 6000, batch: int = 1024, lr: float = 1e-3, seed: int = 0,
          params: Optional[np.ndarray] = None, kind: int = sa.NET_RELU_CAUCHY):
    """Train the proposal network of kind `kind` on `records`; returns
    (params, loss trace)."""
    tr = sa.MLPTrainer(max_batch=batch)
    try:
        tr.set_kind(kind)
        tr.set_params(init_params(seed) if params is None else params)
        trace = tr.train(records, batch=batch, steps=steps, lr=lr, seed=seed)
        return tr.params(), trace
    finally:
        tr.close()


@dataclass
class TargetResult:
    hit: bool
    level: Optional[int]       # first level whose record is within target
    levels_run: int
    seconds: Optional[float]   # device time from the first level to the hit
    ms_per_level: float
    final_gap: float           # record - f* after the last level run


def time_to_target(func, lower, upper, shift, schedule: sa.Schedule, f_star: float, target: float = 1e-4, *,
                   params=None, eps: float = 0.1, start_level: int = 0, x_start=None, chunk: int = 100,
                   learn_from: int = 0, kind: int = sa.NET_RELU_CAUCHY):
    """Run levels in chunks until the record is within `target` of f_star or
    the schedule ends.  With `params`, levels from `learn_from` on use the
    learned mixture and earlier ones the plain moves.  The time to the hit is
    the chunks' device time (HIP events on the annealer's stream), pro rata
    within the last chunk."""
    import torch
    sched = sa.Schedule(**{**schedule.__dict__, "trace_x": False, "graph": False, "learned": params is not None,
                           "log_chains": 0})
    with sa.Annealer(func, lower, upper, shift, schedule=sched) as ann:
        if params is not None:
            ann.set_network_kind(kind)
        if start_level:
            ann.set_start(start_level, x_start)
        learning = False
        first = ann.levels_done()
        elapsed = 0.0
        hit_level, hit_time = None, None
        gap = math.inf
        with torch.cuda.stream(ann.stream):
            while ann.levels_done() < sched.levels:
                k0 = ann.levels_done()
                if params is not None and not learning and k0 >= learn_from:
                    ann.set_proposal(params, eps)
                    learning = True
                count = min(chunk, sched.levels - k0)
                if params is not None and not learning:
                    count = min(count, learn_from - k0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(ann.stream)
                ann.run(count)
                e1.record(ann.stream)
                e1.synchronize()
                dt = e0.elapsed_time(e1) / 1e3
                rec = ann.trace(k0, count)
                gaps = rec["f_rec"] - f_star
                gap = float(gaps[-1])
                idx = np.flatnonzero(gaps < target)
                if idx.size:
                    hit_level = k0 + int(idx[0])
                    hit_time = elapsed + dt * (idx[0] + 1) / count
                    elapsed += dt
                    break
                elapsed += dt
        done = ann.levels_done() - first
    return TargetResult(hit=hit_level is not None, level=hit_level, levels_run=done, seconds=hit_time,
                        ms_per_level=1e3 * elapsed / max(done, 1), final_gap=gap)
