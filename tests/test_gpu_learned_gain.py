"""What the trained proposal gains over the method without it.

Schwefel n=16 in FP32: accepted moves are captured from plain runs over the
whole temperature range (seed 101), the network is trained on them on the
GPU, and then three arms run the same final-approach schedule (every chain
starts at one point within +-20 of x* per coordinate, at a level where T is
already low) from the same seeds: plain radius moves, the trained proposal,
and the untrained network.  The trained arm must reach |f - f*| < 1e-4 in
fewer levels than the plain arm, and end with a smaller gap than both other
arms.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_trained_proposal_beats_plain_and_untrained():
    import torch
    assert torch.cuda.is_available()
    from paper_2408_00018_amd import learned as Lp
    from paper_2408_00018_amd import sa
    n = 16
    lo, hi = np.full(n, -500.0), np.full(n, 500.0)
    base = sa.Schedule(chains=1024, levels=1200, steps=50, T0=10.0, alpha=0.99, seed=101, precision=sa.FP32)
    say("[gain] collecting")
    rec = Lp.collect(W.SCHWEFEL, lo, hi, None, base, every=4, per_level=20000)
    say(f"[gain] {rec.shape[0]} records; training")
    params, trace = Lp.train(rec, steps=1500, batch=1024, lr=1e-3, seed=0)
    say(f"[gain] loss {trace[:20].mean():.3f} -> {trace[-50:].mean():.3f}")
    assert trace[-50:].mean() < trace[:20].mean()
    untrained = Lp.init_params(0)
    rng = np.random.default_rng(7)
    x0 = np.clip(W.SCHWEFEL_X_STAR + rng.uniform(-20, 20, n), -500, 500)
    results = {}
    for arm, p in (("plain", None), ("trained", params), ("untrained", untrained)):
        results[arm] = []
        for seed in (1, 2):
            sched = sa.Schedule(**{**base.__dict__, "seed": seed})
            r = Lp.time_to_target(W.SCHWEFEL, lo, hi, None, sched, W.SCHWEFEL_F_STAR, 1e-4, params=p, eps=0.1,
                                  start_level=500, x_start=x0, chunk=50)
            say(f"[gain] {arm} seed {seed}: {r}")
            results[arm].append(r)

    def levels(arm):
        return [r.level if r.hit else np.inf for r in results[arm]]

    def gaps(arm):
        return [r.final_gap if not r.hit else 0.0 for r in results[arm]]

    assert all(r.hit for r in results["trained"])
    assert np.all(np.array(levels("trained")) < np.array(levels("plain")))
    assert np.median(levels("trained")) <= np.median(levels("untrained"))
    assert max(gaps("trained")) <= min(min(gaps("plain")), min(gaps("untrained"))) + 1e-12
