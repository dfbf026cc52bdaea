"""Pins of the oracle's full-evaluation variant (every move's cost increment
taken as f(x') - f(x) with f evaluated in full, Sec. 2.1's plain definition)
against things other than the variant itself."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _plain_levels(func, lo, hi, shift, seed, chains, steps, T0, alpha, levels):
    """The synchronous scheme written out in Python from Sec. 2.1-2.2: every
    chain runs `steps` Metropolis moves with dE = f(x') - f(x), then the
    lowest final cost (ties to the lowest chain) is broadcast."""
    n = lo.size
    radius = 0.1 * (hi - lo)
    start = None
    out = []
    for level in range(levels):
        T = T0 * alpha ** level
        finals = []
        for c in range(chains):
            x = O.init_point(seed, 0, c, lo, hi) if start is None else start.copy()
            fx = O.f(func, x, shift)
            for j in range(steps):
                d, u1, u2 = O.move_draw(seed, 0, level, c, j, n)
                xn = x.copy()
                xn[d] = min(max(x[d] + radius[d] * (2 * u1 - 1), lo[d]), hi[d])
                fn = O.f(func, xn, shift)
                dE = fn - fx
                if dE <= 0 or u2 < math.exp(-dE / T):
                    x, fx = xn, fn
            finals.append((fx, c, x))
        fw, cw, xw = min(finals, key=lambda t: (t[0], t[1]))
        out.append((cw, fw, xw))
        start = xw
    return out


@pytest.mark.parametrize("func", [W.SCHWEFEL, W.RASTRIGIN, W.ACKLEY, W.GRIEWANK])
def test_full_eval_run_is_the_plain_definition(func):
    wl = W.random_problem(func, 5, seed=4)
    lo, hi = W.uneven_box(5, 2) if func == W.SCHWEFEL else (wl.lower, wl.upper)
    T0 = 200.0 if func == W.SCHWEFEL else 5.0
    args = dict(seed=17, chains=6, steps=12, T0=T0, alpha=0.7, levels=4)
    r = O.sa_run(func, lo, hi, wl.shift, full_eval=True, **args)
    ref = _plain_levels(func, lo, hi, wl.shift, **args)
    for level, (cw, fw, xw) in enumerate(ref):
        assert r["win_chain"][level] == cw
        assert r["f_win"][level] == fw
        assert np.array_equal(r["x_best"][level], xw)


@pytest.mark.parametrize("func", [W.SCHWEFEL, W.RASTRIGIN, W.ACKLEY])
def test_full_eval_agrees_with_increment_up_to_rounding(func):
    """For the separable families the two evaluations give the same
    increment up to rounding, so the runs share their winners while no
    acceptance sits on a rounding-sized margin."""
    wl = W.random_problem(func, 24, seed=2)
    args = dict(seed=3, chains=128, steps=40, T0=10.0, alpha=0.9, levels=6)
    a = O.sa_run(func, wl.lower, wl.upper, wl.shift, **args)
    b = O.sa_run(func, wl.lower, wl.upper, wl.shift, full_eval=True, **args)
    assert np.array_equal(a["win_chain"], b["win_chain"])
    np.testing.assert_allclose(b["f_win"], a["f_win"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b["x_best"], a["x_best"], rtol=0, atol=1e-12)
    assert np.array_equal(a["accepts"], b["accepts"])


def test_full_eval_leaves_coupled_families_unchanged():
    """The non-separable families always evaluate in full, so the flag does
    not change their runs."""
    wl = W.random_problem(W.GRIEWANK, 9, seed=1)
    args = dict(seed=8, chains=32, steps=25, T0=2.0, alpha=0.8, levels=5)
    a = O.sa_run(W.GRIEWANK, wl.lower, wl.upper, wl.shift, **args)
    b = O.sa_run(W.GRIEWANK, wl.lower, wl.upper, wl.shift, full_eval=True, **args)
    for k in ("win_chain", "f_win", "x_best", "accepts"):
        assert np.array_equal(a[k], b[k])
