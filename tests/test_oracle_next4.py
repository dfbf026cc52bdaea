"""Pins of the oracle's exchange variants (Sec. 2.2: the minimum operator as a
deterministic crossover, a stochastic crossover as the alternative; the
reduction over each chain's best-seen state instead of its final state).

Stochastic exchange (SOS reading): at a level that starts with an exchange a
chain keeps its own state with probability exp(-(f_own - f_win)/T_prev),
else starts from the winner.
- At a temperature so high that every probability is 1 the run is the
  asynchronous scheme bit for bit.
- The number of chains that keep their state matches the sum of the
  probabilities computed here from the previous level's costs (4 standard
  deviations; a sign error, the wrong level's temperature or the fresh
  instead of the carried cost moves it by far more).
- Each chain's next level replays (orc_replay_level, one chain at a time)
  from its own previous state if it kept it and from the winner otherwise,
  to its logged final cost.
Elitist exchange (the record broadcast instead of the level winner):
- Each level equals one plain level whose broadcast state is the record
  after the level before, the record tracked from the plain levels.
- Without exchanges it is the asynchronous run.
Best-seen reduction:
- Near zero temperature (only downhill moves) it equals the final-state run.
- The level winner's state is one of the states its chain visited (replayed
  move by move), and no visited state of any chain evaluates lower than the
  winner's re-evaluation (beyond carried-cost rounding).
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def base(n=4, chains=256):
    lo, hi = np.full(n, -500.0), np.full(n, 500.0)
    return dict(lower=lo, upper=hi, chains=chains, steps=40, seed=7)


def test_sos_at_very_high_temperature_is_the_asynchronous_scheme():
    b = base()
    kw = dict(seed=b["seed"], chains=b["chains"], steps=b["steps"], T0=1e300, alpha=1.0, levels=6)
    a = O.sa_run(O.SCHWEFEL, b["lower"], b["upper"], exchange=1, sos=True, **kw)
    z = O.sa_run(O.SCHWEFEL, b["lower"], b["upper"], exchange=0, **kw)
    for key in ("win_chain", "f_win", "f_best", "accepts"):
        assert np.array_equal(a[key], z[key]), key
    assert np.array_equal(a["x_best"], z["x_best"])


def _two_stage(chains, T0, alpha, levels, sos=True):
    """Levels [0, levels-1) then level levels-1 alone, carrying everything."""
    n = 4
    lo, hi = np.full(n, -500.0), np.full(n, 500.0)
    kw = dict(seed=11, chains=chains, steps=30, T0=T0, alpha=alpha)
    first = O.sa_run(O.SCHWEFEL, lo, hi, levels=levels - 1, exchange=1, sos=sos, final_f=True, **kw)
    second = O.sa_run(O.SCHWEFEL, lo, hi, levels=1, level_begin=levels - 1, exchange=1, sos=sos,
                      x_start=first["x_last"], chain_x=first["chain_x"], chain_cost=first["chain_cost"],
                      f_win_prev=first["f_win_last"], record=(first["x_rec"], first["f_rec_final"],
                                                              first["rec_level"]),
                      final_f=True, kept=True, **kw)
    return lo, hi, kw, first, second


def test_sos_keep_count_follows_the_metropolis_probability():
    chains, T0, alpha, levels = 65536, 0.4, 0.9, 4
    lo, hi, kw, first, second = _two_stage(chains, T0, alpha, levels)
    T_prev = T0 * alpha ** (levels - 2)
    f_own = first["final_f"]  # each chain's carried final cost at the level that ended
    d = f_own - first["f_win"][-1]
    assert np.all(d >= 0.0)
    p = np.exp(-d / T_prev)
    kept = second["kept"]
    mean, sd = p.sum(), math.sqrt(np.sum(p * (1 - p)))
    assert 0.05 * chains < mean < 0.95 * chains  # the probabilities are not all 0 or 1
    assert abs(kept.sum() - mean) <= 4 * sd, (kept.sum(), mean, sd)
    # the same count under the level's own temperature would be far off
    p_wrong = np.exp(-d / (T_prev * alpha))
    assert abs(kept.sum() - p_wrong.sum()) > 8 * sd
    # the winner chain always keeps its state
    assert kept[first["win_chain"][-1]]


def test_sos_chains_continue_from_the_state_they_chose():
    chains, T0, alpha, levels = 512, 0.4, 0.9, 4
    lo, hi, kw, first, second = _two_stage(chains, T0, alpha, levels)
    level = levels - 1
    T = T0 * alpha ** level
    kept = second["kept"]
    assert 0 < kept.sum() < chains
    for c in list(range(0, chains, 23)) + [int(first["win_chain"][-1])]:
        start = first["chain_x"][c] if kept[c] else first["x_last"]
        r = O.replay_level(O.SCHWEFEL, lo, hi, seed=kw["seed"], steps=kw["steps"], T=T, level=level, x_start=start,
                           chain0=c, nchains=1)
        if kept[c]:
            # the replay starts from a full evaluation; the chain carried its own cost in
            f0 = O.f(O.SCHWEFEL, start)
            assert abs(r["f_final"][0] - f0 - (second["final_f"][c] - first["chain_cost"][c, 0])) <= 1e-9
        else:
            assert abs(r["f_final"][0] - second["final_f"][c]) <= 1e-12 * max(1.0, abs(r["f_final"][0]))


def test_best_seen_near_zero_temperature_is_the_final_state_run():
    b = base()
    kw = dict(seed=b["seed"], chains=b["chains"], steps=b["steps"], T0=1e-300, alpha=1.0, levels=5)
    bs = O.sa_run(O.RASTRIGIN, np.full(4, -5.12), np.full(4, 5.12), best_seen=True, **kw)
    fs = O.sa_run(O.RASTRIGIN, np.full(4, -5.12), np.full(4, 5.12), **kw)
    for key in ("win_chain", "f_win", "f_best", "accepts"):
        assert np.array_equal(bs[key], fs[key]), key
    assert np.array_equal(bs["x_best"], fs["x_best"])


def test_best_seen_winner_is_the_lowest_visited_state():
    n, chains, steps = 3, 128, 60
    lo, hi = np.full(n, -500.0), np.full(n, 500.0)
    x0 = np.array([300.0, -200.0, 410.0])
    T = 2.0
    # level 1 from a given start (record carried empty): one level with best-seen
    o = O.sa_run(O.SCHWEFEL, lo, hi, seed=3, chains=chains, steps=steps, T0=T, alpha=1.0, levels=1, level_begin=1,
                 x_start=x0, best_seen=True, final_f=True)
    fs = O.sa_run(O.SCHWEFEL, lo, hi, seed=3, chains=chains, steps=steps, T0=T, alpha=1.0, levels=1, level_begin=1,
                  x_start=x0, final_f=True)
    r = O.replay_level(O.SCHWEFEL, lo, hi, seed=3, steps=steps, T=T, level=1, x_start=x0, chain0=0, nchains=chains)
    best_visit = math.inf
    visited = {}
    for c in range(chains):
        x = x0.copy()
        states = [x.copy()]
        for s in range(steps):
            if r["acc"][c, s]:
                x[r["d"][c, s]] = r["x_new"][c, s]
                states.append(x.copy())
        visited[c] = states
        vals = [O.f(O.SCHWEFEL, v) for v in states]
        best_visit = min(best_visit, min(vals))
        # the chain's reduced value is its lowest carried cost: never above its final cost
        assert o["final_f"][c] <= fs["final_f"][c] + 1e-12
        assert abs(o["final_f"][c] - min(vals)) <= 1e-9
    w = int(o["win_chain"][0])
    assert any(np.array_equal(o["x_best"][0], v) for v in visited[w])
    assert o["f_best"][0] <= best_visit + 1e-9
    assert o["f_best"][0] <= fs["f_best"][0] + 1e-9


def _elitist_cases():
    # T0 at which level winners often come out worse than the record
    return [(W.SCHWEFEL, 6, "canonical", 1, 200.0), (W.RASTRIGIN, 5, "shifted", 1, 40.0),
            (W.ACKLEY, 4, "canonical", 2, 40.0)]


@pytest.mark.parametrize("func,n,box,exchange,T0", _elitist_cases())
def test_elitist_is_the_plain_run_restarted_from_the_record(func, n, box, exchange, T0):
    """The elitist exchange composed from plain runs: level k of an elitist
    run equals one plain level k whose broadcast state is the record after
    level k - 1 (the lowest re-evaluated winner so far, the first of equal
    ones), with every chain's own state carried between exchanges.  The
    record is tracked here from the plain levels' f_best, so broadcasting the
    winner instead, or moving the record on a tie, fails at the levels whose
    winner does not improve it (the test requires some)."""
    wl = W.random_problem(func, n, seed=600 + n, shifted=(box == "shifted"))
    kw = dict(seed=7, chains=64, steps=12, T0=T0, alpha=0.9, radius_frac=wl.radius_frac)
    levels = 14
    el = O.sa_run(wl.func, wl.lower, wl.upper, wl.shift, levels=levels, exchange=exchange, elitist=True, **kw)
    x_rec, f_rec, rec_level = np.zeros(n), math.inf, 0
    x_start = None
    cx = cc = None
    not_improving = 0
    for k in range(levels):
        r = O.sa_run(wl.func, wl.lower, wl.upper, wl.shift, levels=1, level_begin=k, exchange=exchange,
                     x_start=x_start, chain_x=cx, chain_cost=cc, record=(x_rec, f_rec, rec_level), **kw)
        for key in ("win_chain", "f_win", "f_best", "f_rec", "accepts"):
            assert np.array_equal(r[key], el[key][k:k + 1]), (k, key)
        assert np.array_equal(r["x_best"], el["x_best"][k:k + 1])
        fb = float(r["f_best"][0])
        if fb < f_rec:
            x_rec, f_rec, rec_level = r["x_best"][0].copy(), fb, k
        else:
            not_improving += 1
        x_start = x_rec.copy()
        cx, cc = r.get("chain_x"), r.get("chain_cost")
    assert not_improving >= 3, not_improving
    assert np.array_equal(el["x_rec"], x_rec) and el["f_rec_final"] == f_rec


def test_elitist_without_exchange_is_the_asynchronous_run():
    wl = W.random_problem(W.RASTRIGIN, 5, seed=77)
    kw = dict(seed=3, chains=64, steps=10, T0=5.0, alpha=0.9, levels=8, exchange=0, radius_frac=wl.radius_frac)
    a = O.sa_run(wl.func, wl.lower, wl.upper, wl.shift, **kw)
    b = O.sa_run(wl.func, wl.lower, wl.upper, wl.shift, elitist=True, **kw)
    for key in ("win_chain", "f_win", "f_best", "f_rec", "accepts"):
        assert np.array_equal(a[key], b[key])
