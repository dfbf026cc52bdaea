"""Pins of the oracle's non-separable families (a move changes terms that
other coordinates enter, so the increment is not one coordinate's term):
Griewank (Appendix, Test 8), Levy and Montalvo (Appendix, Test 10) and the
generalized Rosenbrock function (Appendix, Test 14).

Closed forms at points where every sine or cosine is 0 or +-1 fix each
function's structure (the product kept apart from the sum, the sqrt(i)
scaling counted from i = 1, which neighbour carries the sine factor);
scipy's own Rosenbrock is a library reference; n = 2 grids over the paper's
boxes find nothing below the stated minima; short annealing runs reach them.
"""
import math

import numpy as np
import pytest
from scipy.optimize import rosen

import oracle as O


def f(func, x, shift=None):
    return O.f(func, np.asarray(x, dtype=np.float64), None if shift is None else np.asarray(shift, dtype=np.float64))


# ---------------------------------------------------------------- Griewank
def test_griewank_minimum_and_cosines_one():
    assert f(O.GRIEWANK, np.zeros(7)) == 0.0
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 30):
        k = rng.integers(-20, 21, n)
        y = 2.0 * math.pi * k * np.sqrt(np.arange(1, n + 1))   # cos(y_i / sqrt(i)) = 1
        assert abs(f(O.GRIEWANK, y) - np.sum(y * y) / 4000.0) <= 1e-12 * (1.0 + np.sum(y * y) / 4000.0)


def test_griewank_cosines_minus_one_and_zero():
    rng = np.random.default_rng(2)
    for n in (1, 2, 3, 8):
        k = rng.integers(-10, 11, n)
        y = math.pi * (2 * k + 1) * np.sqrt(np.arange(1, n + 1))  # every cosine -1
        want = 1.0 + np.sum(y * y) / 4000.0 - (-1.0) ** n
        assert abs(f(O.GRIEWANK, y) - want) <= 1e-12 * abs(want)
        z = rng.uniform(-600, 600, n)
        j = int(rng.integers(0, n))
        z[j] = 0.5 * math.pi * math.sqrt(j + 1)                   # one cosine 0: the product vanishes
        want = 1.0 + np.sum(z * z) / 4000.0
        assert abs(f(O.GRIEWANK, z) - want) <= 1e-12 * want


def test_griewank_shifted():
    s = np.array([10.0, -250.0, 3.5])
    assert f(O.GRIEWANK, s, s) == 0.0


# ------------------------------------------------------- Levy and Montalvo
def levy_x(w):
    """x with w_i = 1 + (x_i + 1) / 4 equal to w."""
    return 4.0 * (np.asarray(w, dtype=np.float64) - 1.0) - 1.0


def test_levy_minimum():
    for n in (1, 2, 5, 10):
        assert abs(f(O.LEVY_MONTALVO, np.full(n, -1.0))) < 1e-30


def test_levy_integer_points():
    rng = np.random.default_rng(3)
    for n in (1, 2, 5, 10):
        w = rng.integers(-1, 4, n).astype(np.float64)             # every sine 0
        want = math.pi / n * np.sum((w - 1.0) ** 2)
        assert abs(f(O.LEVY_MONTALVO, levy_x(w)) - want) <= 1e-12 * max(1.0, want)


def test_levy_which_neighbour_carries_the_sine():
    # w = (integer, half-integer, integer): sin^2(pi w_2) = 1 multiplies the
    # term of w_1 (the preceding coordinate), not that of w_2 itself
    w = np.array([3.0, 2.5, -1.0])
    want = math.pi / 3 * ((w[0] - 1) ** 2 * 11.0 + (w[1] - 1) ** 2 * 1.0 + (w[2] - 1) ** 2)
    assert abs(f(O.LEVY_MONTALVO, levy_x(w)) - want) <= 1e-12 * want
    # a half-integer first coordinate adds the leading 10 sin^2(pi w_1)
    w = np.array([1.5, 2.0])
    want = math.pi / 2 * (10.0 + (w[0] - 1) ** 2 * 1.0 + (w[1] - 1) ** 2)
    assert abs(f(O.LEVY_MONTALVO, levy_x(w)) - want) <= 1e-12 * want


# ------------------------------------------------------ generalized Rosenbrock
def test_rosenbrock_against_scipy():
    rng = np.random.default_rng(4)
    for n in (2, 3, 4, 17, 100):
        for _ in range(20):
            x = rng.uniform(-2.048, 2.048, n)
            want = rosen(x)
            assert abs(f(O.ROSENBROCK, x) - want) <= 1e-12 * max(1.0, abs(want))
    assert f(O.ROSENBROCK, np.ones(4)) == 0.0
    s = rng.uniform(-1, 1, 4)
    assert f(O.ROSENBROCK, np.ones(4) + s, s) == pytest.approx(0.0, abs=1e-24)


# ------------------------------------------------------------ n = 2 grids
@pytest.mark.parametrize("func,half,x_star", [(O.GRIEWANK, 600.0, 0.0), (O.LEVY_MONTALVO, 10.0, -1.0),
                                              (O.ROSENBROCK, 2.048, 1.0)])
def test_n2_grid_finds_nothing_below_the_minimum(func, half, x_star):
    m = 801
    g = np.linspace(-half, half, m)
    best, arg = math.inf, None
    for a in g:
        for b in g[::2]:
            v = f(func, [a, b])
            if v < best:
                best, arg = v, (a, b)
    assert best >= -1e-12
    fs = f(func, [x_star, x_star])
    assert abs(fs) < 1e-12
    # the grid's best point lies in the minimum's basin: a local descent from
    # it (scipy) reaches f* = 0
    from scipy.optimize import minimize
    r = minimize(lambda v: f(func, v), np.array(arg), method="Nelder-Mead",
                 options=dict(xatol=1e-10, fatol=1e-14, maxiter=4000))
    assert r.fun < 1e-8


@pytest.mark.parametrize("func,half,tol", [(O.LEVY_MONTALVO, 10.0, 1e-4), (O.ROSENBROCK, 2.048, 1e-3),
                                           (O.GRIEWANK, 600.0, 1e-2)])
def test_annealing_reaches_the_minimum_at_n2(func, half, tol):
    lo, hi = np.full(2, -half), np.full(2, half)
    r = O.sa_run(func, lo, hi, seed=5, chains=256, steps=100, T0=1.0, alpha=0.95, levels=250,
                 move_rule=O.MOVE_RESAMPLE if func == O.GRIEWANK else O.MOVE_RADIUS)
    assert r["f_rec_final"] < tol, r["f_rec_final"]
    assert np.all(np.diff(r["f_rec"]) <= 0.0)
