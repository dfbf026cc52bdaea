"""Pins of the oracle's Nelder-Mead polish (the paper's hybrid strategy: a
local minimizer from the point where the annealing stopped).

scipy's Nelder-Mead (same coefficients 1, 2, 1/2, 1/2, same start simplex
x0_i / 20 or 0.00025, same termination test, bounds by clipping) is the
library reference: from the same start both reach the same minimum with
about the same work.  Plus: a start at a minimiser stays there, the result
never leaves the box and never rises above the start.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
import workloads as W


CASES = [(O.ROSENBROCK, 2), (O.ROSENBROCK, 4), (O.SCHWEFEL, 3), (O.ACKLEY, 5), (O.RASTRIGIN, 4),
         (O.GRIEWANK, 3), (O.LEVY_MONTALVO, 3)]


@pytest.mark.parametrize("func,n", CASES)
def test_matches_scipy_nelder_mead(func, n):
    half = W.HALF_BOX[func]
    lo, hi = np.full(n, -half), np.full(n, half)
    rng = np.random.default_rng(10 * func + n)
    x0 = rng.uniform(-0.5 * half, 0.5 * half, n)
    r = O.nelder_mead(func, lo, hi, x0=x0, maxiter=40000, ftol=1e-12, xtol=1e-10)
    sp = minimize(lambda v: O.f(func, v), x0, method="Nelder-Mead", bounds=list(zip(lo, hi)),
                  options=dict(xatol=1e-10, fatol=1e-12, maxiter=40000, maxfev=10 ** 7))
    assert abs(r["f"] - sp.fun) <= 1e-9 * max(1.0, abs(sp.fun)), (r["f"], sp.fun)
    assert np.max(np.abs(r["x"] - sp.x)) <= 1e-5 * max(1.0, half)
    assert abs(r["evals"] - sp.nfev) <= 0.1 * sp.nfev + 5
    assert r["f"] <= O.f(func, x0)
    assert set(np.unique(r["steps"])) <= {0, 1, 2, 3, 4}


def test_start_at_a_minimiser_stays():
    n = 4
    lo, hi = np.full(n, -2.048), np.full(n, 2.048)
    r = O.nelder_mead(O.ROSENBROCK, lo, hi, x0=np.ones(n), ftol=1e-14, xtol=1e-12)
    assert r["f"] == 0.0 and np.array_equal(r["x"], np.ones(n))


def test_projection_keeps_the_box():
    # Rosenbrock's minimiser (1, 1, 1) lies outside [-2, 0.5]^3: the result is
    # on the box and no worse than any clipped trial the method could reach
    n = 3
    lo, hi = np.full(n, -2.0), np.full(n, 0.5)
    r = O.nelder_mead(O.ROSENBROCK, lo, hi, x0=np.full(n, -1.5), maxiter=20000)
    assert np.all(r["x"] >= lo) and np.all(r["x"] <= hi)
    assert r["f"] < O.f(O.ROSENBROCK, np.full(n, -1.5))
    sp = minimize(lambda v: O.f(O.ROSENBROCK, v), np.full(n, -1.5), method="Nelder-Mead", bounds=list(zip(lo, hi)),
                  options=dict(xatol=1e-10, fatol=1e-12, maxiter=20000))
    assert abs(r["f"] - sp.fun) <= 1e-8 * max(1.0, sp.fun)
