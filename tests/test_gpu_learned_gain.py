"""What the trained proposal gains over the method without it.

Schwefel n=16 in FP32.  Accepted moves are captured from a plain run over
1800 levels (T0 = 10, alpha = 0.99, 1024 chains x 50 steps, seed 101), the
same number from every second level, and the network is trained on them on
the GPU.  Three arms then run the greedy end of the same schedule from the
same seeds: every chain starts at level 1400 (T = 7.7e-6, where the thermal
gap n T / 2 is already below the target) at one point within +-0.2 of x* per
coordinate: plain radius moves, the trained proposal, and the untrained
network (a fixed Cauchy scale of 0.01 of the box).  The trained arm must
reach |f - f*| < 1e-4 in fewer levels than both.
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
    base = sa.Schedule(chains=1024, levels=1800, steps=50, T0=10.0, alpha=0.99, seed=101, precision=sa.FP32)
    say("[gain] collecting")
    rec = Lp.collect(W.SCHWEFEL, lo, hi, None, base, every=2, per_level=2000)
    say(f"[gain] {rec.shape[0]} records; training")
    params, trace = Lp.train(rec, steps=6000, batch=1024, lr=1e-3, seed=0)
    say(f"[gain] loss {trace[:20].mean():.3f} -> {trace[-50:].mean():.3f}")
    assert trace[-50:].mean() < trace[:20].mean()
    untrained = Lp.init_params(0)
    rng = np.random.default_rng(7)
    x0 = W.SCHWEFEL_X_STAR + rng.uniform(-0.2, 0.2, n)
    results = {}
    for arm, p in (("plain", None), ("trained", params), ("untrained", untrained)):
        results[arm] = []
        for seed in (1, 2):
            sched = sa.Schedule(**{**base.__dict__, "seed": seed})
            r = Lp.time_to_target(W.SCHWEFEL, lo, hi, None, sched, W.SCHWEFEL_F_STAR, 1e-4, params=p, eps=0.1,
                                  start_level=1400, x_start=x0, chunk=10)
            say(f"[gain] {arm} seed {seed}: {r}")
            results[arm].append(r)

    def levels(arm):
        return np.array([r.level - 1400 + 1 if r.hit else np.inf for r in results[arm]])

    say(f"[gain] levels to target: plain {levels('plain')} trained {levels('trained')} "
        f"untrained {levels('untrained')}")
    assert all(r.hit for r in results["trained"])
    assert np.all(levels("trained") < levels("plain"))
    assert np.all(levels("trained") < levels("untrained"))
