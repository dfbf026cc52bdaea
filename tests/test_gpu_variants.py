"""GPU parity of the exchange variants (Sec. 2.2: the minimum operator read as
a deterministic crossover; a stochastic crossover beside it; the best-seen
state in place of the final state; the record broadcast in place of the
winner) against the FP64 oracle.

- FP64 runs follow the oracle's trajectory exactly (winners, accepted-move
  counts, broadcast states, costs to 1e-12), with the stochastic exchange,
  the best-seen reduction and both, at exchange periods 0-3, split over
  several sa_run calls.
- FP32 runs are replayed move by move from the start state each chain
  chose: at a stochastic exchange the oracle's decision on the GPU's carried
  costs (both starts tried where rounding could flip it); under the
  best-seen reduction each chain's logged reduced value matches the lowest
  FP64 cost of the states it visited, and the broadcast state is one of the
  winner's visited states, bit for bit.
- Whole, chunked and graph-captured FP32 runs agree bit for bit; the bench
  shape (n = 100, 65536 chains) is replayed on sampled chains.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_util import U32, box32, check_fp32_level, check_record, f32, fp32_init_state, lexi_argmin

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


def run(S, wl, chunks=None, **kw):
    d = dict(chains=wl.chains, levels=wl.levels, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=wl.seed,
             precision=wl.precision, radius_frac=wl.radius_frac, trace_x=True)
    d.update(kw)
    sched = S.Schedule(**d)
    say(f"[gpu variants] {wl.name} n={wl.n} chains={sched.chains} levels={sched.levels} steps={sched.steps} "
        f"prec={sched.precision} exchange={sched.exchange} sos={sched.sos} best_seen={sched.best_seen} "
        f"elitist={sched.elitist} move={sched.move} chunks={chunks} graph={sched.graph} log={sched.log_chains}")
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as a:
        for c in (chunks or [0]):
            a.run(c)
        rec, xb = a.trace(with_x=True)
        x_rec, f_rec, lvl = a.best()
        out = dict(rec=rec, xb=xb, x_rec=x_rec, f_rec=f_rec, rec_level=lvl)
        if sched.log_chains:
            out["moves"], out["final_f"] = a.move_log()
    return out


def problem(func, n, box, seed, **kw):
    wl = W.random_problem(func, n, seed=seed, shifted=(box == "shifted"))
    if box == "uneven":
        lo, hi = W.uneven_box(n, seed + 1)
        wl = wl.with_(lower=lo, upper=hi, shift=None)
    return wl.with_(**kw)


FP64_CASES = [
    # func, n, chains, levels, steps, box, exchange, sos, best, move, chunks
    (W.SCHWEFEL, 4, 256, 12, 30, "canonical", 1, True, False, O.MOVE_RADIUS, None),
    (W.RASTRIGIN, 6, 512, 10, 20, "shifted", 3, True, False, O.MOVE_RADIUS, [4, 0]),
    (W.ACKLEY, 5, 256, 9, 25, "uneven", 1, False, True, O.MOVE_RADIUS, None),
    (W.SCHWEFEL, 7, 192, 8, 33, "canonical", 1, True, True, O.MOVE_RESAMPLE, [3, 0]),
    (W.RASTRIGIN, 9, 128, 7, 40, "uneven", 0, False, True, O.MOVE_RADIUS, None),
    (W.ACKLEY, 3, 320, 8, 17, "shifted", 2, True, True, O.MOVE_RADIUS, [1, 2, 0]),
]


@pytest.mark.parametrize("func,n,chains,levels,steps,box,exchange,sos,best,move,chunks", FP64_CASES)
def test_fp64_variant_trajectory_equals_oracle(S, func, n, chains, levels, steps, box, exchange, sos, best, move,
                                               chunks):
    wl = problem(func, n, box, 3000 + 10 * func + n, chains=chains, levels=levels, steps=steps, precision=W.FP64,
                 T0=5.0, alpha=0.8)
    g = run(S, wl, chunks=chunks, exchange=exchange, sos=sos, best_seen=best, move=move)
    o = O.sa_run(wl.func, wl.lower, wl.upper, wl.shift, seed=wl.seed, chains=chains, steps=steps, T0=wl.T0,
                 alpha=wl.alpha, levels=levels, radius_frac=wl.radius_frac, move_rule=move, exchange=exchange,
                 sos=sos, best_seen=best, kept=True)
    if sos and exchange == 1:
        # the decisions of the last level went both ways
        assert 0 < o["kept"].sum() < chains, o["kept"].sum()
    assert np.array_equal(g["rec"]["win_chain"], o["win_chain"])
    assert np.array_equal(g["rec"]["accepts"], o["accepts"])
    np.testing.assert_allclose(g["xb"], o["x_best"], rtol=1e-12, atol=1e-12)
    for k in ("f_win", "f_best", "f_rec"):
        np.testing.assert_allclose(g["rec"][k], o[k], rtol=1e-12, atol=1e-12)
    assert g["rec_level"] == o["rec_level"]


def sos_keeps(d, u, T_prev):
    """The oracle's stochastic-exchange decision on a cost difference d, and
    whether FP32 rounding of d, 1/T and the hardware exp2 could flip it."""
    if d <= 0.0:
        return True, False
    p = math.exp(-d / T_prev)
    margin = p * (d / T_prev) * 2.0 ** -20 + 2.0 ** -18 * p + 2.0 ** -24
    return u < p, abs(u - p) <= margin


def elite_state(g, level):
    """The record after `level` as an elitist run broadcasts it: the first
    level winner of lowest full re-evaluation up to that level."""
    fb = g["rec"]["f_best"][:level + 1]
    return g["xb"][int(np.argmin(fb))]


def replay(wl, g, exchange, sos, best, chains, elitist=False):
    """Per-move replay of a logged FP32 variant run from level 0; each chain
    from the start it chose.  Returns (moves replayed, ambiguous decisions)."""
    lo32, hi32 = box32(wl.lower, wl.upper)
    sh32 = None if wl.shift is None else f32(wl.shift)
    moves, final_f, rec, xb = g["moves"], g["final_f"], g["rec"], g["xb"]
    state, err, flast, total, ambiguous = {}, {}, {}, 0, 0
    for level in range(moves.shape[0]):
        T = O.temperature(wl.T0, wl.alpha, level)
        win = lexi_argmin(final_f[level])
        assert rec["win_chain"][level] == win
        assert rec["f_win"][level] == final_f[level][win]
        fb = O.f(wl.func, xb[level], sh32)
        assert abs(rec["f_best"][level] - fb) <= 1e-11 * max(1.0, abs(fb))
        exch = level > 0 and exchange > 0 and level % exchange == 0
        for c in chains:
            if level == 0:
                starts = [(fp32_init_state(wl, c), None, False)]
            elif not exch:
                starts = [(state[c], err[c], True)]
            elif not sos:
                starts = [(elite_state(g, level - 1) if elitist else xb[level - 1], None, False)]
            else:
                T_prev = O.temperature(wl.T0, wl.alpha, level - 1)
                u = O.sos_uniform(wl.seed, 0, level, c)
                f_win = rec["f_win"][level - 1]
                if best:
                    # the GPU decides on the chain's final carried cost, within err of its FP64 value
                    keep_hi, amb_hi = sos_keeps(max(flast[c] + err[c] - f_win, 0.0), u, T_prev)
                    keep_lo, amb_lo = sos_keeps(max(flast[c] - err[c] - f_win, 0.0), u, T_prev)
                    keep, amb = keep_hi, amb_hi or amb_lo or keep_hi != keep_lo
                else:
                    keep, amb = sos_keeps(float(np.float32(final_f[level - 1][c] - f_win)), u, T_prev)
                own = (state[c], err[c], True)
                bcast = (xb[level - 1], None, False)
                if amb:
                    ambiguous += 1
                    starts = [own, bcast]
                else:
                    starts = [own] if keep else [bcast]
            last_exc = None
            for x0, se, is_own in starts:
                try:
                    st = check_fp32_level(wl.func, wl.n, lo32, hi32, sh32, wl.seed, level, T, O.MOVE_RADIUS,
                                          wl.radius_frac, x0, moves[level, c:c + 1], final_f[level], [c],
                                          start_err=se, best_seen=best)
                    break
                except AssertionError as e:  # the other start of an ambiguous decision
                    last_exc = e
            else:
                raise last_exc
            if best and c == win:
                assert any(np.array_equal(xb[level], v) for v in st["visited"][c]), (level, c)
            state[c], err[c], flast[c] = st["x_final"][c], st["f_err"][c], st["f_last"][c]
            total += st["moves"]
    return total, ambiguous


@pytest.mark.parametrize("func,n,exchange,sos,best", [(W.SCHWEFEL, 12, 1, False, True),
                                                      (W.RASTRIGIN, 8, 1, True, False),
                                                      (W.ACKLEY, 6, 2, True, True),
                                                      (W.SCHWEFEL, 10, 0, False, True)])
def test_fp32_variant_levels_replay_against_oracle(S, func, n, exchange, sos, best):
    wl = W.random_problem(func, n, seed=70 + n).with_(chains=256, levels=6, steps=24, T0=5.0, alpha=0.8)
    g = run(S, wl, exchange=exchange, sos=sos, best_seen=best, log_chains=256, log_level=0, log_levels=6)
    moves, amb = replay(wl, g, exchange, sos, best, range(256))
    check_record(wl, g)
    say(f"[fp32 variant parity] {wl.name} exchange={exchange} sos={sos} best={best}: {moves} moves, "
        f"{amb} ambiguous exchange decisions")
    assert amb <= 0.02 * 256 * 6


def test_fp32_variant_runs_agree_bitwise(S):
    """Whole, chunked and graph-captured variant runs: identical bits."""
    wl = W.random_problem(W.RASTRIGIN, 24, seed=43).with_(chains=1024, levels=9, steps=37, T0=5.0, alpha=0.8)
    keys = ["win_chain", "accepts", "f_win", "f_best", "f_rec"]
    for kw in (dict(sos=True), dict(best_seen=True), dict(sos=True, best_seen=True, exchange=2)):
        whole = run(S, wl, **kw)
        for other in (run(S, wl, chunks=[1, 4, 2, 0], **kw), run(S, wl, graph=True, chunks=[4, 0], **kw)):
            assert np.array_equal(other["rec"][keys], whole["rec"][keys])
            assert np.array_equal(other["xb"], whole["xb"])
        check_record(wl, whole)


def test_fp32_variants_bench_shape(S):
    """The bench workload's shape (Schwefel n = 100, 65536 chains, 100 steps)
    with the stochastic exchange and the best-seen reduction: three levels
    logged, sampled chains replayed from the starts they chose."""
    wl = W.schwefel_n100_fp32().with_(levels=3, T0=1.0)
    for kw in (dict(sos=True), dict(best_seen=True)):
        g = run(S, wl, log_chains=512, log_level=0, log_levels=3, **kw)
        moves, amb = replay(wl, g, 1, kw.get("sos", False), kw.get("best_seen", False), range(0, 512, 31))
        check_record(wl, g)
        say(f"[fp32 variant parity] bench shape {kw}: {moves} moves, {amb} ambiguous")


def test_variants_rejected_where_unsupported(S):
    wl = W.random_problem(W.SCHWEFEL, 8, seed=1)
    for kw in (dict(sos=True, overlay=True), dict(best_seen=True, learned=True)):
        with pytest.raises(S.SAError) as e:
            run(S, wl, **kw)
        assert e.value.status == -5
    g = W.griewank_n100_fp32().with_(chains=256, levels=2, steps=4)
    with pytest.raises(S.SAError) as e:
        run(S, g, best_seen=True)
    assert e.value.status == -5


ELITIST_CASES = [
    # func, n, chains, levels, steps, box, exchange, best, move, chunks, T0
    (W.SCHWEFEL, 4, 256, 12, 30, "canonical", 1, False, O.MOVE_RADIUS, None, 200.0),
    (W.RASTRIGIN, 6, 512, 10, 20, "shifted", 3, False, O.MOVE_RADIUS, [4, 0], 40.0),
    (W.ACKLEY, 5, 256, 9, 25, "uneven", 1, True, O.MOVE_RESAMPLE, [2, 0], 40.0),
    (W.GRIEWANK, 7, 256, 9, 20, "shifted", 1, False, O.MOVE_RADIUS, None, 20.0),
]


@pytest.mark.parametrize("func,n,chains,levels,steps,box,exchange,best,move,chunks,T0", ELITIST_CASES)
def test_fp64_elitist_trajectory_equals_oracle(S, func, n, chains, levels, steps, box, exchange, best, move, chunks,
                                               T0):
    """SA_FLAG_ELITIST in FP64: the trajectory equals the oracle's elitist run
    (winners, accepted moves, winner states, costs to 1e-12) -- dense layout,
    a periodic exchange, the best-seen reduction, a non-separable family --
    with levels whose winner does not improve the record (where broadcasting
    the winner would differ)."""
    wl = problem(func, n, box, 3100 + 10 * func + n, chains=chains, levels=levels, steps=steps, precision=W.FP64,
                 T0=T0, alpha=0.9)
    g = run(S, wl, chunks=chunks, exchange=exchange, best_seen=best, move=move, elitist=True)
    o = O.sa_run(wl.func, wl.lower, wl.upper, wl.shift, seed=wl.seed, chains=chains, steps=steps, T0=wl.T0,
                 alpha=wl.alpha, levels=levels, radius_frac=wl.radius_frac, move_rule=move, exchange=exchange,
                 best_seen=best, elitist=True)
    fb = o["f_best"]
    if not best:  # (a best-seen winner never trails the record it started from)
        assert np.sum(fb[1:] >= np.minimum.accumulate(fb)[:-1]) >= 2  # some winners leave the record alone
    assert np.array_equal(g["rec"]["win_chain"], o["win_chain"])
    assert np.array_equal(g["rec"]["accepts"], o["accepts"])
    np.testing.assert_allclose(g["xb"], o["x_best"], rtol=1e-12, atol=1e-12)
    for k in ("f_win", "f_best", "f_rec"):
        np.testing.assert_allclose(g["rec"][k], o[k], rtol=1e-12, atol=1e-12)
    assert g["rec_level"] == o["rec_level"]


def test_fp32_elitist_levels_replay_against_oracle(S):
    """FP32 elitist run: every logged move replayed against the oracle from
    the record state each level broadcasts; whole, chunked and graph-captured
    runs agree bit for bit."""
    wl = W.random_problem(W.RASTRIGIN, 8, seed=91).with_(chains=256, levels=6, steps=24, T0=40.0, alpha=0.9)
    g = run(S, wl, elitist=True, log_chains=256, log_level=0, log_levels=6)
    moves, amb = replay(wl, g, 1, False, False, range(256), elitist=True)
    check_record(wl, g)
    fb = g["rec"]["f_best"]
    kept = int(np.sum(fb[1:-1] >= np.minimum.accumulate(fb)[:-2]))
    say(f"[fp32 elitist parity] {moves} moves, {amb} ambiguous; {kept} broadcasts kept the record")
    assert kept >= 1
    keys = ["win_chain", "accepts", "f_win", "f_best", "f_rec"]
    whole = run(S, wl, elitist=True)
    for other in (run(S, wl, chunks=[2, 1, 0], elitist=True), run(S, wl, graph=True, chunks=[3, 0], elitist=True)):
        assert np.array_equal(other["rec"][keys], whole["rec"][keys])
        assert np.array_equal(other["xb"], whole["xb"])
