"""Pins of the FP64 CPU oracle against things other than itself.

Each test ties one part of the oracle to the paper's printed values, a
closed form, a library routine, brute force, or an invariant the method must
satisfy, so that a plausible slip (dropped term, wrong sign, transposed
operand, inverted test) fails at least one of them.
"""
import math
import os
import shutil
import subprocess
import textwrap

import numpy as np
import pytest

import oracle as O
import workloads as W
from conftest import read_golden

# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------


def test_philox_known_answers():
    rows = read_golden("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for row in rows:
        v = [int(t, 16) for t in row]
        out = O.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


ROCRAND_SRC = textwrap.dedent(r"""
    #include <rocrand/rocrand_kernel.h>
    #include <cstdio>
    int main() {
      unsigned long long seed, sub, off;
      while (scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, off, &st);
        uint4 r = rocrand4(&st);
        printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
      }
      return 0;
    }
""")


@pytest.fixture(scope="session")
def rocrand_philox(tmp_path_factory):
    """rocRAND's host-callable Philox4x32-10, used as a black-box comparator:
    rocrand_init(seed, subsequence, 4 m) yields the block at counter
    (m_lo, m_hi, sub_lo, sub_hi) under key (seed_lo, seed_hi)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tmp_path_factory.mktemp("rocrand")
    src = d / "rr.cpp"
    src.write_text(ROCRAND_SRC)
    exe = d / "rr"
    subprocess.check_call([hipcc, "-x", "hip", "--cuda-host-only", "-O1", str(src), "-o", str(exe)])

    def gen(cases):
        inp = "\n".join(f"{s} {sub} {off}" for s, sub, off in cases) + "\n"
        out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split()
        return np.array([int(t) for t in out], dtype=np.uint64).reshape(-1, 4)

    return gen


def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(7)
    cases, ctrs, keys = [], [], []
    for _ in range(200):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        c = [int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        m = c[0] | (c[1] << 32)
        sub = c[2] | (c[3] << 32)
        if 4 * m >= 2**64:
            m &= (1 << 61) - 1
            c[0], c[1] = m & 0xFFFFFFFF, m >> 32
        cases.append((seed, sub, 4 * m))
        ctrs.append(c)
        keys.append([seed & 0xFFFFFFFF, seed >> 32])
    ref = rocrand_philox(cases)
    for c, k, r in zip(ctrs, keys, ref):
        assert [int(v) for v in O.philox4x32_10(c, k)] == [int(v) for v in r]


def test_uniform_and_pick():
    assert O.uniform(0) == 0.0
    assert O.uniform(0xFFFFFFFF) == (2**24 - 1) / 2**24
    assert O.uniform(0x80000000) == 0.5
    # the low 8 bits are ignored
    assert O.uniform(0x12345678) == O.uniform(0x12345600)
    for n in (1, 2, 3, 100, 1024):
        assert O.pick(0, n) == 0
        assert O.pick(0xFFFFFFFF, n) == n - 1
        # equal-width bins: r in [k 2^32/n, (k+1) 2^32/n) -> k
        for k in range(min(n, 50)):
            lo = -(-(k << 32) // n)
            assert O.pick(lo, n) == k
            if lo > 0:
                assert O.pick(lo - 1, n) == k - 1


def test_move_draw_uses_documented_counter():
    """Move s takes words 3s, 3s+1, 3s+2 of the stream of blocks
    (b, level, chain, 0 | problem << 8), b = 0, 1, ...: four moves take three
    blocks, in order, with no word skipped or repeated."""
    seed, problem, level, chain, n = 0x0123456789ABCDEF, 3, 17, 999, 100
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for g in (0, 1, 10, 333):
        words = []
        for b in range(3 * g, 3 * g + 3):
            words += [int(w) for w in O.philox4x32_10([b, level, chain, 0 | (problem << 8)], key)]
        for r in range(4):
            d, u1, u2 = O.move_draw(seed, problem, level, chain, 4 * g + r, n)
            assert d == O.pick(words[3 * r], n)
            assert u1 == O.uniform(words[3 * r + 1])
            assert u2 == O.uniform(words[3 * r + 2])


def test_learned_block_words():
    """The learned block (step, level, chain, 3 | problem << 8): word 0 is the
    Cauchy draw by inversion, word 1 the mixture choice."""
    seed, problem, level, chain, step = 77, 2, 5, 123, 41
    r = O.philox4x32_10([step, level, chain, 3 | (problem << 8)], [seed & 0xFFFFFFFF, seed >> 32])
    assert O.learn_mix(seed, problem, level, chain, step) == O.uniform(int(r[1]))
    t = O.learn_draw(seed, problem, level, chain, step)
    assert abs(t - math.tan(math.pi * (O.uniform(int(r[0])) - 0.5))) <= 1e-12 * max(1.0, abs(t))


def test_init_point_uniform_in_box():
    lo, hi = W.uneven_box(37, 5)
    xs = np.array([O.init_point(11, 0, c, lo, hi) for c in range(400)])
    assert np.all(xs >= lo) and np.all(xs <= hi)
    # every coordinate is uniform in its own box: mean of (x-l)/(u-l) near 1/2
    z = (xs - lo) / (hi - lo)
    assert abs(z.mean() - 0.5) < 0.02
    assert abs(z.var() - 1 / 12) < 0.01
    # start counter layout: coordinate i uses word i%4 of block i/4
    r = O.philox4x32_10([1, 0xFFFFFFFF, 5, 1], [11, 0])
    x = O.init_point(11, 0, 5, lo, hi)
    assert x[6] == lo[6] + (hi[6] - lo[6]) * O.uniform(int(r[2]))


# --------------------------------------------------------------------------
# Test functions: closed forms and the paper's printed minima
# --------------------------------------------------------------------------


def test_schwefel_minimum_matches_paper(paper_values):
    xs, fs = paper_values["schwefel_x_star"], paper_values["schwefel_f_star"]
    for n in (1, 3, 100):
        assert abs(O.f(W.SCHWEFEL, np.full(n, xs)) - fs) < 1e-6
    # the paper's x* is the minimiser of one term over the box: brute force
    grid = np.linspace(-500.0, 500.0, 200001)
    vals = np.array([-O.schwefel_term(g) for g in grid])
    gmin = grid[np.argmin(vals)]
    assert abs(gmin - xs) < 0.01
    # a library root finder on the oracle's central-difference slope lands on
    # it to the printed precision (the minimum is too flat to locate by value)
    from scipy.optimize import brentq

    def slope(y, h=1e-3):
        return (O.schwefel_term(y + h) - O.schwefel_term(y - h)) / (2 * h)

    root = brentq(slope, 400.0, 440.0, xtol=1e-12)
    assert abs(root - xs) < 1e-6
    assert abs(root - W.SCHWEFEL_X_STAR) < 1e-7
    assert abs(-O.schwefel_term(W.SCHWEFEL_X_STAR) - W.SCHWEFEL_F_STAR) < 1e-12
    assert abs(W.SCHWEFEL_F_STAR - fs) < 1e-6


def test_schwefel_closed_forms():
    # y = ((2k + 1/2) pi)^2 -> sin(sqrt y) = 1, term = y; y = (k pi)^2 -> term = 0
    for k in range(0, 3):
        y = ((2 * k + 0.5) * math.pi) ** 2
        assert abs(O.f(W.SCHWEFEL, [y, y]) + y) < 1e-9 * y
        # the term is odd in y: at -y it is -y, so f = +y
        assert abs(O.f(W.SCHWEFEL, [-y]) - y) < 1e-9 * y
        z = ((k + 1) * math.pi) ** 2
        assert abs(O.f(W.SCHWEFEL, [z])) < 1e-9 * z
    # normalisation: mean of the terms, negated
    x = np.array([1.0, 4.0, 9.0])
    expect = -(1.0 * math.sin(1.0) + 4.0 * math.sin(2.0) + 9.0 * math.sin(3.0)) / 3.0
    assert abs(O.f(W.SCHWEFEL, x) - expect) < 1e-12


def test_rastrigin_closed_forms(paper_values):
    n = 7
    s = np.linspace(-2.0, 2.0, n)
    assert abs(O.f(W.RASTRIGIN, s, s) - paper_values["rastrigin_f_star"]) < 1e-12
    # integer coordinates: cos(2 pi k) = 1 -> f = sum k^2
    k = np.array([1.0, -2.0, 3.0, 0.0])
    assert abs(O.f(W.RASTRIGIN, k) - np.sum(k * k)) < 1e-10
    # half-integers: cos = -1 -> each coordinate contributes y^2 + 20
    h = np.array([0.5, -1.5, 2.5])
    assert abs(O.f(W.RASTRIGIN, h) - (np.sum(h * h) + 20 * 3)) < 1e-10
    # shift enters as y = x - s
    assert abs(O.f(W.RASTRIGIN, k + s[:4], s[:4]) - np.sum(k * k)) < 1e-10


def test_ackley_closed_forms(paper_values):
    n = 9
    s = np.linspace(-3.0, 3.0, n)
    assert abs(O.f(W.ACKLEY, s, s) - paper_values["ackley_f_star"]) < 1e-12
    # y_i = +-1: S1/n = 1, S2/n = 1 -> f = 20 (1 - e^-0.2)
    y = np.array([1.0, -1.0, 1.0, 1.0])
    assert abs(O.f(W.ACKLEY, y) - 20.0 * (1.0 - math.exp(-0.2))) < 1e-12
    # y_i = 1/2: S1/n = 1/4, S2/n = -1 -> f = -20 e^{-0.1} - e^{-1} + 20 + e
    y = np.full(5, 0.5)
    expect = -20.0 * math.exp(-0.1) - math.exp(-1.0) + 20.0 + math.e
    assert abs(O.f(W.ACKLEY, y) - expect) < 1e-12


@pytest.mark.parametrize("func", [W.SCHWEFEL, W.RASTRIGIN, W.ACKLEY])
def test_brute_force_n2(func):
    """Grid search over a shifted 2-D box: the grid minimum sits next to the
    known minimiser and is within the grid's Lipschitz bound of f*."""
    wl = W.random_problem(func, 2, seed=101 + func)
    lo, hi, s = wl.lower, wl.upper, wl.shift
    if func == W.SCHWEFEL:
        # Schwefel's minimiser is a corner region of the canonical box; shift the box with it.
        s = np.array([-37.5, 12.25])
        lo, hi = lo + s, hi + s
        x_star = W.SCHWEFEL_X_STAR + s
        f_star = W.SCHWEFEL_F_STAR
    else:
        x_star = s
        f_star = 0.0
    m = 401
    g0 = np.linspace(lo[0], hi[0], m)
    g1 = np.linspace(lo[1], hi[1], m)
    best, arg = np.inf, None
    for a in g0:
        for b in g1:
            v = O.f(func, [a, b], s)
            if v < best:
                best, arg = v, (a, b)
    h = (hi - lo) / (m - 1)
    assert best >= f_star - 1e-9
    assert np.all(np.abs(np.array(arg) - x_star) <= h + 1e-9)
    # Lipschitz bound from a fine local grid around the minimiser
    lg = [x_star + np.array([dx, dy]) for dx in np.linspace(-h[0], h[0], 21) for dy in np.linspace(-h[1], h[1], 21)]
    local = max(O.f(func, p, s) for p in lg)
    assert best <= local + 1e-12


# --------------------------------------------------------------------------
# Move, acceptance, cooling
# --------------------------------------------------------------------------


def test_metropolis_rule():
    # downhill and flat moves are always taken
    for u in (0.0, 0.5, 1.0 - 2**-24):
        assert O.accept(-1.0, 1.0, u)
        assert O.accept(0.0, 1e-300, u)
    # uphill at T -> 0 never
    assert not O.accept(1e-6, 1e-300, 0.0)
    # uphill: acceptance probability exp(-dE/T) over a uniform u grid (eq. (5))
    us = (np.arange(2**14) + 0.5) / 2**14
    for dE, T in ((1.0, 1.0), (0.3, 2.0), (5.0, 1.0)):
        frac = np.mean([O.accept(dE, T, u) for u in us])
        assert abs(frac - math.exp(-dE / T)) < 2.0 / 2**14


def test_neighbour_radius_and_clamp():
    lo, hi, rf = -500.0, 500.0, 0.1
    rho = rf * (hi - lo)
    assert O.neighbour(O.MOVE_RADIUS, 10.0, lo, hi, rf, 0.5) == 10.0
    assert O.neighbour(O.MOVE_RADIUS, 10.0, lo, hi, rf, 0.0) == 10.0 - rho
    assert O.neighbour(O.MOVE_RADIUS, 495.0, lo, hi, rf, 0.99) == hi
    assert O.neighbour(O.MOVE_RADIUS, -495.0, lo, hi, rf, 0.01) == lo
    assert O.neighbour(O.MOVE_RESAMPLE, 123.0, lo, hi, rf, 0.25) == -250.0
    us = np.linspace(0, 1 - 2**-24, 1001)
    ys = np.array([O.neighbour(O.MOVE_RADIUS, 0.0, lo, hi, rf, u) for u in us])
    assert np.all(np.abs(ys) <= rho)
    assert abs(ys.mean()) < 0.2


def _levels_until(T0, alpha, T_min):
    """Levels run by the paper's do { level(T); T *= rho } while (T > T_min)."""
    k = 0
    while True:
        k += 1
        if not O.temperature(T0, alpha, k) > T_min:
            return k


def test_cooling_schedule_and_evaluation_counts(paper_values):
    assert O.temperature(10.0, 0.99, 0) == 10.0
    assert abs(O.temperature(10.0, 0.99, 200) - 10.0 * 0.99**200) < 1e-12
    # Sec. 4.1 setting: 1146 levels, chains * (L N + 1) evaluations
    L = _levels_until(1000.0, 0.99, 0.01)
    assert L == 1146
    assert float(f"{16384 * (L * 100 + 1):.4e}") == paper_values["evals_schwefel_setting"]
    for chains in (8192, 65536, 131072):
        assert float(f"{chains * (L * 100 + 1):.4e}") == paper_values[f"evals_table4_{chains}"]
    # Table 3 setting: T0=5, Tmin=0.5, rho=0.7, N=5
    L3 = _levels_until(5.0, 0.7, 0.5)
    assert L3 == 7
    for thr in (768, 76800, 7680000):
        assert float(f"{thr * (L3 * 5 + 1):.4e}") == paper_values[f"evals_table3_{thr}"]


# --------------------------------------------------------------------------
# The synchronous scheme
# --------------------------------------------------------------------------

SMALL = dict(seed=5, chains=64, steps=20, T0=10.0, alpha=0.9)


@pytest.mark.parametrize("func", [W.SCHWEFEL, W.RASTRIGIN, W.ACKLEY])
def test_incremental_equals_direct_difference(func):
    wl = W.random_problem(func, 13, seed=3)
    lo, hi = W.uneven_box(13, 4) if func == W.SCHWEFEL else (wl.lower, wl.upper)
    rep = O.replay_level(func, lo, hi, wl.shift, seed=9, steps=200, T=5.0, level=2,
                         x_start=O.init_point(9, 0, 0, lo, hi), chain0=0, nchains=3)
    for c in range(3):
        x = O.init_point(9, 0, 0, lo, hi)
        for s in range(200):
            d = rep["d"][c, s]
            assert rep["x_old"][c, s] == x[d]
            xn = x.copy()
            xn[d] = rep["x_new"][c, s]
            direct = O.f(func, xn, wl.shift) - O.f(func, x, wl.shift)
            scale = max(abs(O.f(func, xn, wl.shift)), abs(O.f(func, x, wl.shift)), 1.0)
            assert abs(rep["df"][c, s] - direct) <= 1e-12 * scale
            if rep["acc"][c, s]:
                x = xn
        assert np.array_equal(rep["x_final"][c], x)


def test_single_chain_is_sequential_sa():
    """With one chain the synchronous scheme is the sequential algorithm of
    Sec. 2.1 (its pseudo-code): a pure-Python loop over the same draws."""
    lo, hi = np.full(3, -500.0), np.full(3, 500.0)
    seed, steps, T0, alpha, levels = 21, 15, 50.0, 0.8, 6
    r = O.sa_run(W.SCHWEFEL, lo, hi, seed=seed, chains=1, steps=steps, T0=T0, alpha=alpha, levels=levels)
    x = O.init_point(seed, 0, 0, lo, hi)
    T = T0
    for level in range(levels):
        for j in range(steps):
            d, u1, u2 = O.move_draw(seed, 0, level, 0, j, 3)
            xn = x.copy()
            xn[d] = min(max(x[d] + 0.1 * (hi[d] - lo[d]) * (2 * u1 - 1), lo[d]), hi[d])
            dE = O.f(W.SCHWEFEL, xn) - O.f(W.SCHWEFEL, x)
            if dE <= 0 or u2 < math.exp(-dE / T):
                x = xn
        T *= alpha
        assert np.allclose(r["x_best"][level], x, rtol=0, atol=1e-12)


def test_level_winner_is_argmin_and_broadcast():
    lo, hi = W.uneven_box(6, 8)
    kw = dict(seed=4, chains=128, steps=25, T0=20.0, alpha=0.9)
    r = O.sa_run(W.SCHWEFEL, lo, hi, levels=5, final_f=True, **kw)
    ff = r["final_f"]
    assert r["win_chain"][-1] == int(np.argmin(ff))
    assert r["f_win"][-1] == ff.min()
    # level 4 starts every chain from level 3's winner: replaying it from there
    # reproduces every chain's final cost and the winner's state.
    rep = O.replay_level(W.SCHWEFEL, lo, hi, None, seed=4, steps=25, T=O.temperature(20.0, 0.9, 4), level=4,
                         x_start=r["x_best"][3], chain0=0, nchains=128)
    assert np.allclose(rep["f_final"], ff, rtol=1e-13, atol=1e-13)
    assert np.array_equal(rep["x_final"][r["win_chain"][-1]], r["x_best"][-1])


def test_ties_go_to_lowest_chain():
    # at T -> 0 with a radius move most chains reject everything and tie
    lo, hi = np.full(2, -500.0), np.full(2, 500.0)
    r = O.sa_run(W.SCHWEFEL, lo, hi, seed=1, chains=64, steps=1, T0=1e-300, alpha=1.0, levels=3, final_f=True)
    ff = r["final_f"]
    m = ff.min()
    assert r["win_chain"][-1] == int(np.flatnonzero(ff == m)[0])


def test_invariants_box_and_monotone_record():
    lo, hi = W.uneven_box(5, 2)
    r = O.sa_run(W.RASTRIGIN, lo, hi, W.random_problem(1, 5, 2).shift * 0.0, seed=2, chains=64, steps=30, T0=30.0,
                 alpha=0.9, levels=20)
    xb = r["x_best"]
    assert np.all(xb >= lo) and np.all(xb <= hi)
    assert np.all(np.diff(r["f_rec"]) <= 0)
    assert np.allclose(r["f_rec"], np.minimum.accumulate(r["f_best"]))
    for k in range(20):
        assert abs(r["f_best"][k] - O.f(W.RASTRIGIN, xb[k], np.zeros(5))) < 1e-12 * max(1, abs(r["f_best"][k]))


def test_infinite_temperature_is_clipped_random_walk():
    lo, hi = np.full(3, -5.0), np.full(3, 5.0)
    seed, steps = 13, 40
    rep = O.replay_level(W.ACKLEY, lo, hi, None, seed=seed, steps=steps, T=1e300, level=0,
                         x_start=np.zeros(3), chain0=7, nchains=1)
    assert rep["acc"].all()
    x = np.zeros(3)
    for j in range(steps):
        d, u1, _ = O.move_draw(seed, 0, 0, 7, j, 3)
        x[d] = min(max(x[d] + 1.0 * (2 * u1 - 1), -5.0), 5.0)
    assert np.array_equal(rep["x_final"][0], x)


def test_zero_temperature_only_downhill():
    lo, hi = np.full(4, -500.0), np.full(4, 500.0)
    rep = O.replay_level(W.SCHWEFEL, lo, hi, None, seed=3, steps=300, T=1e-300, level=1,
                         x_start=np.full(4, 100.0), chain0=0, nchains=8)
    assert np.all(rep["df"][rep["acc"]] <= 0)
    assert np.all(rep["acc"][rep["df"] <= 0])


def test_resume_is_bit_identical():
    lo, hi = W.uneven_box(4, 3)
    kw = dict(seed=8, chains=64, steps=10, T0=10.0, alpha=0.95)
    full = O.sa_run(W.ACKLEY, lo, hi, levels=9, **kw)
    a = O.sa_run(W.ACKLEY, lo, hi, levels=4, **kw)
    b = O.sa_run(W.ACKLEY, lo, hi, levels=5, level_begin=4, x_start=a["x_last"],
                 record=(a["x_rec"], a["f_rec_final"], a["rec_level"]), **kw)
    assert np.array_equal(np.concatenate([a["x_best"], b["x_best"]]), full["x_best"])
    assert np.array_equal(np.concatenate([a["f_rec"], b["f_rec"]]), full["f_rec"])
    assert np.array_equal(b["x_rec"], full["x_rec"])


def test_async_variant_keeps_chains_apart():
    """Without exchange (Sec. 2.2.1) each chain continues from its own state:
    chain c of a multi-chain run equals a one-chain run of chain c's stream."""
    lo, hi = np.full(3, -500.0), np.full(3, 500.0)
    kw = dict(seed=6, steps=12, T0=10.0, alpha=0.9, levels=4, exchange=False)
    r = O.sa_run(W.SCHWEFEL, lo, hi, chains=64, **kw)
    # a one-chain run starting from chain 5's start, replayed with chain index 5 via replay_level
    x = O.init_point(6, 0, 5, lo, hi)
    for level in range(4):
        rep = O.replay_level(W.SCHWEFEL, lo, hi, None, seed=6, steps=12, T=O.temperature(10.0, 0.9, level),
                             level=level, x_start=x, chain0=5, nchains=1)
        x = rep["x_final"][0]
    assert np.array_equal(r["chain_x"][5], x)


KEYS = ("win_chain", "f_win", "f_best", "accepts")


def _levels(r, a, b):
    return {k: r[k][a:b] for k in KEYS} | {"x_best": r["x_best"][a:b]}


def _same(x, y):
    for k in x:
        assert np.array_equal(x[k], y[k]), k


def test_exchange_period_one_is_the_synchronous_run():
    lo, hi = np.full(3, -5.12), np.full(3, 5.12)
    kw = dict(seed=8, chains=64, steps=10, T0=10.0, alpha=0.9, levels=5)
    a = O.sa_run(W.RASTRIGIN, lo, hi, exchange=True, **kw)
    b = O.sa_run(W.RASTRIGIN, lo, hi, exchange=1, **kw)
    _same(_levels(a, 0, 5), _levels(b, 0, 5))


@pytest.mark.parametrize("func", [W.SCHWEFEL, W.ACKLEY])
def test_periodic_exchange_every_third_level(func):
    """Periodic exchange (Sec. 2.2) every 3 levels, pinned level by level
    against the two schemes it interleaves: before the first exchange it is
    the asynchronous run; at level 3 every chain restarts from level 2's
    winner with its cost evaluated in full, exactly as one synchronous level
    started from that state; at levels 4-5 the chains carry their own states
    and costs again (an asynchronous continuation of the level-3 chains)."""
    half = 500.0 if func == W.SCHWEFEL else 32.768
    lo, hi = np.full(4, -half), np.full(4, half)
    kw = dict(seed=9, chains=64, steps=11, T0=10.0, alpha=0.9)
    per = O.sa_run(func, lo, hi, levels=6, exchange=3, **kw)
    asy = O.sa_run(func, lo, hi, levels=3, exchange=False, **kw)
    _same(_levels(per, 0, 3), _levels(asy, 0, 3))
    rec = (asy["x_rec"], asy["f_rec_final"], asy["rec_level"])
    sync3 = O.sa_run(func, lo, hi, levels=1, level_begin=3, x_start=per["x_best"][2], record=rec,
                     exchange=True, final_f=True, **kw)
    _same(_levels(per, 3, 4), _levels(sync3, 0, 1))
    # the chains after level 3, then levels 4-5 without exchange
    upto3 = O.sa_run(func, lo, hi, levels=4, exchange=3, **kw)
    _same(_levels(upto3, 0, 4), _levels(per, 0, 4))
    rec3 = (upto3["x_rec"], upto3["f_rec_final"], upto3["rec_level"])
    cont = O.sa_run(func, lo, hi, levels=2, level_begin=4, exchange=False, chain_x=upto3["chain_x"],
                    chain_cost=upto3["chain_cost"], record=rec3, **kw)
    _same(_levels(per, 4, 6), _levels(cont, 0, 2))
    assert np.array_equal(per["f_rec"][4:], cont["f_rec"])


def test_asynchronous_chains_carry_their_cost():
    """Without exchange a chain's cost is carried through every level, never
    re-evaluated: after 6 levels each chain's carried Ackley cost (through its
    two sums) still equals the definition evaluated at its state, to the
    rounding of ~6 x 20 increments."""
    lo, hi = np.full(5, -32.768), np.full(5, 32.768)
    r = O.sa_run(W.ACKLEY, lo, hi, seed=10, chains=64, steps=20, T0=5.0, alpha=0.9, levels=6, exchange=0)
    for ch in range(64):
        fx = O.f(W.ACKLEY, r["chain_x"][ch])
        assert abs(r["chain_cost"][ch][0] - fx) <= 1e-11 * max(1.0, abs(fx))
        assert abs(r["chain_cost"][ch][1] - float(np.sum(r["chain_x"][ch] ** 2))) <= 1e-9


def test_reaches_schwefel_minimum():
    """The method reaches the closed-form minimum (Sec. 4.1) within 1e-4: at
    n=2 with either move rule, and at n=4 under the 256-chain, 200x50 FP64
    schedule on a seed whose chains do not freeze in a side basin (seed 15;
    seed 0 freezes one coordinate in the -302.5 basin, gap 29.6: whether a
    run freezes is decided mostly by the random starts of level 0)."""
    lo, hi = np.full(2, -500.0), np.full(2, 500.0)
    for rule in (O.MOVE_RADIUS, O.MOVE_RESAMPLE):
        r = O.sa_run(W.SCHWEFEL, lo, hi, seed=0, chains=256, steps=50, T0=10.0, alpha=0.99, levels=200,
                     move_rule=rule)
        assert 0.0 <= r["f_rec_final"] - W.SCHWEFEL_F_STAR < 1e-4
    wl = W.schwefel_n4_fp64()
    r = O.sa_run(wl.func, wl.lower, wl.upper, seed=15, chains=wl.chains, steps=wl.steps, T0=wl.T0, alpha=wl.alpha,
                 levels=wl.levels)
    assert 0.0 <= r["f_rec_final"] - W.SCHWEFEL_F_STAR < 1e-4
    # the minimiser: |x - x*| within the quadratic bound sqrt(2 n gap / h''), h'' = 0.2524
    gap = r["f_rec_final"] - W.SCHWEFEL_F_STAR
    assert np.max(np.abs(r["x_rec"] - W.SCHWEFEL_X_STAR)) <= math.sqrt(2 * 4 * max(gap, 1e-12) / 0.25) + 1e-6


@pytest.mark.parametrize("func,exchange", [(O.SCHWEFEL, 1), (O.ACKLEY, 1), (O.RASTRIGIN, 3), (O.SCHWEFEL, 0),
                                           (O.GRIEWANK, 1), (O.ROSENBROCK, 2)])
def test_chain_threads_are_bit_identical(func, exchange):
    """The oracle's chain-threaded mode (threads over a level's chains, winner
    reduced in chain order afterwards) gives the single-thread bits for every
    thread count, including counts that do not divide the chains."""
    wl = W.random_problem(func, 6, seed=71 + func)
    outs = []
    for t in (1, 3, 8):
        O.set_threads(t)
        try:
            outs.append(O.sa_run(wl.func, wl.lower, wl.upper, wl.shift, seed=7, chains=200, steps=40, T0=3.0,
                                 alpha=0.8, levels=7, exchange=exchange, final_f=True))
        finally:
            O.set_threads(1)
    for o in outs[1:]:
        for k in ("win_chain", "accepts", "f_win", "f_best", "f_rec", "x_best", "x_rec", "final_f"):
            assert np.array_equal(np.asarray(o[k]), np.asarray(outs[0][k])), k
