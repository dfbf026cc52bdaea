"""The allocation-free entry point (sa_run_static) against the allocating one
(sa_create + sa_run + sa_best) on the same problems: two calls in a row, the
second on a smaller problem (the static scratch keeps the first call's
contents), both bit-identical to the allocating path's record; a run whose
workspace exceeds the static scratch is refused with SA_ERR_UNSUPPORTED."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2408_00018_amd import sa
    sa.load_library()
    return sa


def allocating(S, wl, sched):
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as a:
        a.run()
        return a.best()


def sched_of(S, wl, levels):
    return S.Schedule(chains=wl.chains, levels=levels, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=wl.seed,
                      precision=wl.precision, radius_frac=wl.radius_frac)


def test_static_equals_allocating_on_two_calls(S):
    big = W.schwefel_n100_fp32()
    rng = np.random.default_rng(3)
    lo, hi = W.uneven_box(9, 4)
    small = W.Workload("rastrigin_n9_fp64_table", W.RASTRIGIN, 9, lo, hi, W.inner_shift(lo, hi, rng), chains=512,
                       levels=0, steps=32, T0=5.0, alpha=0.9, seed=11, precision=W.FP64)
    for wl, levels in ((big, 40), (small, 30)):
        sched = sched_of(S, wl, levels)
        say(f"[no-alloc] {wl.name} n={wl.n} chains={wl.chains} levels={levels} prec={wl.precision}")
        xs, fs, ls = S.run_static(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched)
        xa, fa, la = allocating(S, wl, sched)
        say(f"[no-alloc] static f={fs!r} level {ls}; allocating f={fa!r} level {la}")
        assert ls == la and fs == fa
        assert np.array_equal(xs, xa)


def test_static_refuses_a_workspace_beyond_its_scratch(S):
    wl = W.schwefel_n100_fp32()
    sched = sched_of(S, wl, 4)
    sched.exchange = 0  # every chain keeps its own state: 26 MB of workspace
    with pytest.raises(S.SAError) as e:
        S.run_static(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched)
    assert e.value.status == -5 and "static scratch" in str(e.value)  # SA_ERR_UNSUPPORTED
