"""The SA_FAULT injection hook on a GPU: an injected launch fault leaves the
context exactly as it was (a later run equals an undisturbed one bit for
bit), and an injected allocation fault refuses only the calls that would
allocate (a caller-provided workspace still works)."""
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


def test_launch_fault_leaves_the_context_usable(S, monkeypatch):
    wl = W.random_problem(W.SCHWEFEL, 8, seed=3)
    sched = S.Schedule(chains=256, levels=6, steps=16, T0=5.0, alpha=0.8, seed=4, precision=S.FP32, trace_x=True)
    say("[gpu faults] launch fault")
    cols = ["win_chain", "accepts", "f_win", "f_best", "f_rec"]
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as a, \
            S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as b:
        a.run(2)
        b.run(2)
        monkeypatch.setenv("SA_FAULT", "launch")
        for call in (lambda: a.run(2), lambda: a.reset(9)):
            with pytest.raises(S.SAError) as e:
                call()
            assert e.value.status == -3 and "SA_FAULT=launch" in str(e.value)
        monkeypatch.delenv("SA_FAULT")
        assert a.levels_done() == 2
        a.run(0)
        b.run(0)
        ra, xa = a.trace(with_x=True)
        rb, xb = b.trace(with_x=True)
    assert np.array_equal(ra[cols], rb[cols]) and np.array_equal(xa, xb)


def test_alloc_fault_spares_caller_workspaces(S, monkeypatch):
    wl = W.random_problem(W.RASTRIGIN, 6, seed=5)
    sched = S.Schedule(chains=128, levels=3, steps=8, T0=5.0, alpha=0.8, seed=1, precision=S.FP32)
    say("[gpu faults] alloc fault")
    monkeypatch.setenv("SA_FAULT", "alloc")
    with pytest.raises(S.SAError) as e:
        S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched, torch_workspace=False)
    assert e.value.status == -2
    with pytest.raises(S.SAError) as e:
        S.MLPTrainer(max_batch=64)
    assert e.value.status == -2
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as a:  # torch-allocated workspace
        a.run(0)
        _, f_rec, _ = a.best()
    monkeypatch.delenv("SA_FAULT")
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched, torch_workspace=False) as a:
        a.run(0)
        _, f_ref, _ = a.best()
    assert f_rec == f_ref
