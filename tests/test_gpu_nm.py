"""GPU parity of the Nelder-Mead polish (the paper's hybrid strategy: a local
minimizer started where the annealing stopped, Sec. 4.2, hybrid results
table) against the oracle's Nelder-Mead.

Both evaluate costs in FP64 in coordinate order and build trial points
elementwise, so the GPU follows the oracle's step sequence.  The vertex
coordinates depend only on the steps taken, so where the step logs agree to
the end the results are bit-identical.  The two libm implementations (host
and device) may differ in a last bit of a sine or cosine; that can flip a
comparison only between costs equal to ~1e-13, so a step log may part from
the oracle's only once the simplex's cost gap f_w - f_b has closed to that
scale, and both must then end at the same minimum within the termination
tolerances.  Also: the candidates the polish starts from (one per workgroup,
lowest carried cost first) against the oracle's final chain costs, and the
hybrid run (anneal, then polish) on the two-dimensional and 4-D problems.
"""
import sys

import numpy as np
import pytest

import oracle as O
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


CASES = [(O.SCHWEFEL, 4, False), (O.RASTRIGIN, 5, True), (O.ACKLEY, 6, True), (O.GRIEWANK, 3, False),
         (O.LEVY_MONTALVO, 7, True), (O.ROSENBROCK, 5, False), (O.ROSENBROCK, 70, False), (O.GRIEWANK, 130, True)]


def problem(func, n, shifted, seed):
    half = W.HALF_BOX[func]
    lo, hi = np.full(n, -half), np.full(n, half)
    rng = np.random.default_rng(seed)
    sh = W.inner_shift(lo, hi, rng) if shifted else None
    return lo, hi, sh, rng


def compare(func, lo, hi, sh, x0, g, j, o, maxiter):
    """Start j of the GPU polish g against the oracle's run o from the same start."""
    it_g, it_o = int(g["iters"][j]), o["iters"]
    steps_g = g["steps"][j, :it_g]
    common = min(it_g, it_o)
    diff = np.flatnonzero(steps_g[:common] != o["steps"][:common])
    scale = max(1.0, abs(o["f"]))
    x_g, f_g = g["x"][j], float(g["f"][j])
    # the GPU result is a point of the box whose FP64 cost it reports
    assert np.all(x_g >= lo) and np.all(x_g <= hi)
    assert abs(f_g - O.f(func, x_g, sh)) <= 1e-14 * max(1.0, abs(f_g))
    assert f_g <= O.f(func, x0, sh)
    if diff.size == 0 and it_g == it_o:
        # same steps to the end: the same vertices
        assert np.array_equal(x_g, o["x"]), (j, np.max(np.abs(x_g - o["x"])))
        assert abs(f_g - o["f"]) <= 1e-14 * scale
        assert int(g["evals"][j]) == o["evals"]
        return "identical", it_g
    first = int(diff[0]) if diff.size else common
    # parted only once the simplex's costs agreed to the last bits
    assert o["gaps"][first] <= 1e-11 * scale, (j, first, o["gaps"][first], it_g, it_o)
    if it_g < maxiter and it_o < maxiter:
        assert abs(f_g - o["f"]) <= 1e-9 * scale, (j, f_g, o["f"])
        assert np.max(np.abs(x_g - o["x"])) <= 1e-6 * max(1.0, hi[0] - lo[0]), (j, x_g, o["x"])
    return f"parted at {first} of {it_o}", it_g


@pytest.mark.parametrize("func,n,shifted", CASES)
def test_polish_follows_the_oracle(S, func, n, shifted):
    lo, hi, sh, rng = problem(func, n, shifted, 100 * func + n)
    starts = rng.uniform(lo + 0.05 * (hi - lo), hi - 0.05 * (hi - lo), (5, n))
    starts[0, 0] = 0.0  # a zero coordinate takes the fixed start step
    maxiter = 30000 if n < 64 else 4000
    say(f"[gpu nm] func={func} n={n} shifted={shifted} starts={len(starts)} maxiter={maxiter}")
    g = S.nm_polish(func, lo, hi, sh, x0=starts, maxiter=maxiter, ftol=1e-12, xtol=1e-10, log_steps=True)
    for j in range(len(starts)):
        o = O.nelder_mead(func, lo, hi, sh, x0=starts[j], maxiter=maxiter, ftol=1e-12, xtol=1e-10)
        how, it = compare(func, lo, hi, sh, starts[j], g, j, o, maxiter)
        say(f"[gpu nm]   start {j}: {how}, {it} iterations, f = {g['f'][j]:.15g} (oracle {o['f']:.15g})")


def test_polish_iteration_cap(S):
    lo, hi, sh, rng = problem(O.ROSENBROCK, 6, False, 3)
    starts = rng.uniform(lo, hi, (3, 6))
    g = S.nm_polish(O.ROSENBROCK, lo, hi, sh, x0=starts, maxiter=57, log_steps=True)
    assert np.all(g["iters"] == 57)
    for j in range(3):
        o = O.nelder_mead(O.ROSENBROCK, lo, hi, sh, x0=starts[j], maxiter=57)
        assert o["iters"] == 57 and np.array_equal(g["steps"][j], o["steps"])
        assert np.array_equal(g["x"][j], o["x"])


def test_polish_one_dimension_and_errors(S):
    lo, hi = np.array([-500.0]), np.array([500.0])
    g = S.nm_polish(O.SCHWEFEL, lo, hi, None, x0=[[300.0]], log_steps=True)
    o = O.nelder_mead(O.SCHWEFEL, lo, hi, None, x0=[300.0])
    assert np.array_equal(g["steps"][0, :g["iters"][0]], o["steps"]) and np.array_equal(g["x"][0], o["x"])
    with pytest.raises(S.SAError) as e:
        S.nm_polish(O.SCHWEFEL, lo, hi, None, x0=[[600.0]])
    assert e.value.status == -1


def test_candidates_are_the_workgroup_bests(S):
    """Candidates of an FP64 run (trajectory-equal to the oracle): one per
    workgroup -- the lowest final cost over its tiles, ties to the lower chain --
    lowest first, each with the full re-evaluation of its state."""
    wl = W.schwefel_n4_fp64().with_(levels=30)
    sched = S.Schedule(chains=wl.chains, levels=wl.levels, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=wl.seed,
                       precision=S.FP64)
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as a:
        a.run()
        wg, _, tiles = a.layout()
        cx, cf, cc = a.candidates(0)
    o = O.sa_run(wl.func, wl.lower, wl.upper, seed=wl.seed, chains=wl.chains, steps=wl.steps, T0=wl.T0,
                 alpha=wl.alpha, levels=wl.levels, final_f=True)
    G = len(cc)
    ff = o["final_f"]
    exp = []
    for gi in range(G):
        chains = [t * wg + l for t in range(gi, tiles, G) for l in range(wg)]
        best = min(chains, key=lambda c: (ff[c], c))
        exp.append((ff[best], best))
    exp.sort()
    assert [c for _, c in exp] == list(cc)
    for r in range(G):
        assert abs(cf[r] - O.f(wl.func, cx[r])) <= 1e-12 * abs(cf[r])
    assert cc[0] == o["win_chain"][-1]


def test_hybrid_polish_from_the_record(S):
    """Anneal (n = 4 FP64 Schwefel, trajectory-equal to the oracle), then polish
    from the record and the best candidates: no worse than the oracle's
    Nelder-Mead from the same record, and no worse than the record."""
    wl = W.schwefel_n4_fp64().with_(levels=120)
    sched = S.Schedule(chains=wl.chains, levels=wl.levels, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=wl.seed,
                       precision=S.FP64)
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as a:
        a.run()
        _, f_rec, _ = a.best()
        x, f, j = a.polish(4)
    o = O.sa_run(wl.func, wl.lower, wl.upper, seed=wl.seed, chains=wl.chains, steps=wl.steps, T0=wl.T0,
                 alpha=wl.alpha, levels=wl.levels)
    on = O.nelder_mead(wl.func, wl.lower, wl.upper, x0=o["x_rec"])
    say(f"[gpu nm] hybrid: record {f_rec:.12f}, polished {f:.12f} (start {j}); oracle polish {on['f']:.12f}; "
        f"f* {W.SCHWEFEL_F_STAR}")
    assert f <= f_rec and f <= on["f"] + 1e-12 * abs(on["f"])
    assert abs(O.f(wl.func, x) - f) <= 1e-13 * abs(f)
