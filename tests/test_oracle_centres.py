"""Pins of the oracle's centre families (Appendix: Test 18 Shekel with m = 5,
7, 10; Test 19 modified Shekel foxholes; Test 11 modified Langerman): each
is a sum over table centres a_i of a function of the squared distance
|y - a_i|^2.

The paper prints each family's minimiser and minimum (tests/golden/
centre_families.txt): a local minimisation (scipy) from the printed point
must land within the printed point's rounding and reach the printed value to
its printed digits -- a mistyped centre, a transposed table, a weight taken
from the wrong row or a sign slip moves one of them.  n = 2 grids over the
paper's boxes find nothing below the printed minima, more centres only lower
Shekel's value, and a shift translates the function.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from conftest import read_golden

IDS = {"shekel5": O.SHEKEL5, "shekel7": O.SHEKEL7, "shekel10": O.SHEKEL10, "foxholes": O.FOXHOLES,
       "langerman": O.LANGERMAN}
BOX = {O.SHEKEL5: (0.0, 10.0), O.SHEKEL7: (0.0, 10.0), O.SHEKEL10: (0.0, 10.0), O.FOXHOLES: (-5.0, 15.0),
       O.LANGERMAN: (0.0, 10.0)}


def f(func, x, shift=None):
    return O.f(func, np.asarray(x, dtype=np.float64), None if shift is None else np.asarray(shift, dtype=np.float64))


def printed_rows():
    rows = []
    for key, n, fstar, *xs in read_golden("centre_families.txt"):
        digits = len(fstar.split(".")[1])
        rows.append((key, IDS[key], int(n), float(fstar), digits, np.array([float(v) for v in xs])))
    return rows


@pytest.mark.parametrize("key,func,n,fstar,digits,xstar", printed_rows(),
                         ids=[f"{r[0]}_n{r[2]}" for r in printed_rows()])
def test_printed_minimum(key, func, n, fstar, digits, xstar):
    assert xstar.size == n
    r = minimize(lambda x: f(func, x), xstar, method="Nelder-Mead",
                 options=dict(xatol=1e-11, fatol=1e-14, maxiter=20000, maxfev=40000))
    # the minimiser sits within the printed point's last digits
    assert np.max(np.abs(r.x - xstar)) < 1e-3
    # its value is the printed one to the printed digits (rounded or cut)
    assert abs(r.fun - fstar) <= 10.0 ** -digits
    # and the printed point itself is close to it
    assert abs(f(func, xstar) - fstar) <= 2e-4


@pytest.mark.parametrize("func,fstar", [(O.FOXHOLES, -12.1190), (O.LANGERMAN, -1.080938)])
def test_n2_grid_finds_nothing_below_the_printed_minimum(func, fstar):
    lo, hi = BOX[func]
    g = np.linspace(lo, hi, 401)
    best = min(f(func, [a, b]) for a in g for b in g)
    assert best >= fstar - 10.0 ** -6


def test_more_shekel_centres_only_lower_the_value():
    rng = np.random.default_rng(3)
    for _ in range(200):
        x = rng.uniform(0.0, 10.0, 4)
        f5, f7, f10 = f(O.SHEKEL5, x), f(O.SHEKEL7, x), f(O.SHEKEL10, x)
        assert f10 < f7 < f5 < 0.0


@pytest.mark.parametrize("func,n", [(O.SHEKEL10, 4), (O.FOXHOLES, 7), (O.LANGERMAN, 3)])
def test_shift_translates(func, n):
    rng = np.random.default_rng(n)
    lo, hi = BOX[func]
    for _ in range(20):
        x = rng.uniform(lo, hi, n)
        s = rng.uniform(-1.0, 1.0, n)
        assert f(func, x + s, s) == pytest.approx(f(func, x), rel=1e-13, abs=1e-13)


def test_dimensions_outside_the_tables_are_nan():
    assert np.isnan(f(O.SHEKEL5, np.full(3, 4.0)))
    assert np.isnan(f(O.SHEKEL7, np.full(5, 4.0)))
    assert np.isnan(f(O.FOXHOLES, np.zeros(11)))
    assert np.isnan(f(O.LANGERMAN, np.zeros(11)))
    assert np.isfinite(f(O.FOXHOLES, np.zeros(10))) and np.isfinite(f(O.LANGERMAN, np.zeros(1)))
