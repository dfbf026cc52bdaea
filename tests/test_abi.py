"""C ABI checks that need no GPU: the library loads, exports every function
include/sa.h declares, and rejects invalid problems before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sa.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:sa_status|void|const char\s*\*)\s*(sa_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def S():
    from paper_2408_00018_amd import sa
    sa.load_library()
    return sa


def test_library_exports_every_declared_function(S):
    names = declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(S.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(S.EXPORTED) == names


def test_structs_match_header_sizes(S):
    # sa_problem: 2 x u32 + 3 pointers; sa_config: u64 + 6 x u32 + 3 doubles + 4 x u32
    assert ctypes.sizeof(S.Problem) == 8 + 3 * 8
    assert ctypes.sizeof(S.Config) == 8 + 6 * 4 + 3 * 8 + 4 * 4
    assert S.LEVEL_DTYPE.itemsize == 48
    assert S.MOVE_DTYPE.itemsize == 32


def _ws(S, wl, **kw):
    d = dict(chains=wl.chains, levels=wl.levels, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=wl.seed,
             precision=wl.precision)
    d.update(kw)
    return S.workspace_bytes(wl.func, wl.lower, wl.upper, wl.shift, S.Schedule(**d))


def test_workspace_sizes(S):
    wl = W.schwefel_n100_fp32()
    b = _ws(S, wl)
    # state slots per 256-chain workgroup + traces: a few hundred KB at most
    assert 100_000 < b < 1_000_000
    assert _ws(S, wl, trace_x=True) >= b + wl.levels * wl.n * 4 - 256
    log = _ws(S, wl, log_chains=64, log_level=0, log_levels=2)
    assert log >= b + 2 * 64 * wl.steps * 32 + 2 * wl.chains * 8 - 512


@pytest.mark.parametrize("bad,status", [
    (dict(chains=96), -1),
    (dict(chains=0), -1),
    (dict(levels=0), -1),
    (dict(steps=0), -1),
    (dict(T0=0.0), -1),
    (dict(T0=float("nan")), -1),
    (dict(alpha=1.5), -1),
    (dict(alpha=0.0), -1),
    (dict(radius_frac=0.0), -1),
    (dict(precision=7), -1),
    (dict(move=3), -1),
    (dict(log_chains=64, log_level=500, log_levels=1), -1),
    (dict(log_chains=65537 * 64, log_level=0, log_levels=1), -1),
])
def test_invalid_configs_are_rejected(S, bad, status):
    wl = W.schwefel_n100_fp32()
    with pytest.raises(S.SAError) as e:
        _ws(S, wl, **bad)
    assert e.value.status == status
    assert S.load_library().sa_last_error().decode()


def test_invalid_problems_are_rejected(S):
    wl = W.schwefel_n4_fp64()
    sched = S.Schedule(chains=64, levels=2, steps=2, T0=1.0, alpha=0.9)
    with pytest.raises(S.SAError):
        S.workspace_bytes(9, wl.lower, wl.upper, None, sched)
    with pytest.raises(S.SAError):
        S.workspace_bytes(0, wl.upper, wl.lower, None, sched)
    with pytest.raises(S.SAError):
        S.workspace_bytes(0, np.array([0.0, np.inf]), np.array([1.0, 2.0]), None, sched)
    with pytest.raises(S.SAError):
        S.workspace_bytes(0, wl.lower, wl.upper, np.array([0.0, np.nan, 0.0, 0.0]), sched)
    with pytest.raises(S.SAError):
        S.workspace_bytes(0, np.zeros(0), np.zeros(0), None, sched)


def test_state_too_large_for_lds_is_unsupported(S):
    # n = 5000 fits only as a shared start state plus per-chain tables
    lo, hi = np.full(5000, -1.0), np.full(5000, 1.0)
    assert S.workspace_bytes(0, lo, hi, None, S.Schedule(chains=64, levels=2, steps=2, T0=1.0, alpha=0.9)) > 0
    # two copies of n = 25000 FP32 coordinates exceed the 160 KiB of LDS in either layout
    lo, hi = np.full(25000, -1.0), np.full(25000, 1.0)
    with pytest.raises(S.SAError) as e:
        S.workspace_bytes(0, lo, hi, None, S.Schedule(chains=64, levels=2, steps=2, T0=1.0, alpha=0.9))
    assert e.value.status == -5
    # the learned proposal needs the dense layout
    lo, hi = np.full(16, -1.0), np.full(16, 1.0)
    with pytest.raises(S.SAError) as e:
        S.workspace_bytes(0, lo, hi, None, S.Schedule(chains=64, levels=2, steps=2, T0=1.0, alpha=0.9, learned=True,
                                                      overlay=True))
    assert e.value.status == -5


def test_exchange_period_options(S):
    """Chains that keep their own state between broadcasts get a per-chain
    state buffer (n + 6 reals per chain) in the workspace; the period needs
    the dense layout and plain or logged moves."""
    wl = W.schwefel_n100_fp32()
    b1 = _ws(S, wl)
    for k in (0, 3):
        bk = _ws(S, wl, exchange=k)
        assert bk >= b1 + wl.chains * (wl.n + 6) * 4 - 512  # the empty buffers' alignment slots
    assert _ws(S, wl, exchange=1) == b1
    lo, hi = np.full(16, -1.0), np.full(16, 1.0)
    for kw in (dict(learned=True), dict(overlay=True)):
        with pytest.raises(S.SAError) as e:
            S.workspace_bytes(0, lo, hi, None, S.Schedule(chains=64, levels=2, steps=2, T0=1.0, alpha=0.9,
                                                          exchange=0, **kw))
        assert e.value.status == -5
    # n = 5000 fits only the overlay layout: no own-state runs
    lo, hi = np.full(5000, -1.0), np.full(5000, 1.0)
    with pytest.raises(S.SAError) as e:
        S.workspace_bytes(0, lo, hi, None, S.Schedule(chains=64, levels=2, steps=2, T0=1.0, alpha=0.9, exchange=4))
    assert e.value.status == -5


def test_null_arguments(S):
    L = S.load_library()
    assert L.sa_workspace_bytes(None, None, None) == -1
    assert L.sa_run(None, 0) == -1
    assert L.sa_best(None, None, None, None) == -1
    L.sa_destroy(None)


def test_bench_refuses_more_than_one_gpu():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_non_separable_families(S):
    """Griewank, Levy-Montalvo and Rosenbrock are valid problems (Griewank's
    FP32 runs keep n cosine-argument factors in the workspace); they run on the
    dense layout with plain or logged moves only, and not in batches."""
    sched = S.Schedule(chains=64, levels=2, steps=2, T0=1.0, alpha=0.9)
    lo, hi = np.full(300, -2.0), np.full(300, 2.0)
    ros = S.workspace_bytes(W.ROSENBROCK, lo, hi, None, sched)
    assert S.workspace_bytes(W.LEVY_MONTALVO, lo, hi, None, sched) == ros
    assert S.workspace_bytes(W.GRIEWANK, lo, hi, None, sched) >= ros + 300 * 4 - 256  # the empty entry's slot
    for kw in (dict(overlay=True), dict(learned=True)):
        with pytest.raises(S.SAError) as e:
            S.workspace_bytes(W.GRIEWANK, lo, hi, None, S.Schedule(chains=64, levels=2, steps=2, T0=1.0,
                                                                   alpha=0.9, **kw))
        assert e.value.status == -5
    # n = 5000 would only fit the overlay layout, which these families do not use
    lo, hi = np.full(5000, -1.0), np.full(5000, 1.0)
    with pytest.raises(S.SAError) as e:
        S.workspace_bytes(W.ROSENBROCK, lo, hi, None, sched)
    assert e.value.status == -5
    with pytest.raises(S.SAError) as e:
        S.workspace_bytes(6, lo[:4], hi[:4], None, sched)
    assert e.value.status == -1
    bs = S.BatchSchedule(levels=2, steps=2, T0=1.0, alpha=0.9)
    with pytest.raises(S.SAError) as e:
        S.batch_workspace_bytes([(W.GRIEWANK, lo[:4], hi[:4], None)], [64], bs)
    assert e.value.status == -5


def test_exchange_variant_flags(S):
    """Stochastic exchange and best-seen reduction: accepted on the dense
    layout of the separable families (the stochastic exchange keeps every
    chain's state in the workspace), refused with the overlay layout, the
    learned proposal and the non-separable families."""
    lo, hi = np.full(100, -500.0), np.full(100, 500.0)
    base = S.Schedule(chains=65536, levels=10, steps=100, T0=10.0, alpha=0.99)
    plain = S.workspace_bytes(S.SCHWEFEL, lo, hi, None, base)
    sos = S.workspace_bytes(S.SCHWEFEL, lo, hi, None, S.Schedule(**{**base.__dict__, "sos": True}))
    assert sos - plain >= 65536 * 101 * 4
    best = S.workspace_bytes(S.SCHWEFEL, lo, hi, None, S.Schedule(**{**base.__dict__, "best_seen": True}))
    assert best == plain
    for kw in (dict(sos=True, overlay=True), dict(best_seen=True, learned=True)):
        with pytest.raises(S.SAError) as e:
            S.workspace_bytes(S.SCHWEFEL, lo, hi, None, S.Schedule(**{**base.__dict__, **kw}))
        assert e.value.status == -5
    with pytest.raises(S.SAError) as e:
        S.workspace_bytes(S.GRIEWANK, np.full(8, -600.0), np.full(8, 600.0), None,
                          S.Schedule(**{**base.__dict__, "best_seen": True}))
    assert e.value.status == -5
