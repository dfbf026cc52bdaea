"""CPU checks of the FP32 error bounds the GPU parity tests use for the full
evaluation per move: the non-separable families, and the separable ones
under SA_FLAG_FULL_EVAL (parity_util.eval_err32).

The FP32 evaluation is emulated in numpy float32 in the kernels' operation
order, with the hardware sine/cosine replaced by the FP64 value of the same
FP32 revolution argument rounded to FP32 (an error below E_TRIG), and the
hardware square root and 2^x by the correctly rounded FP32 values.  The bound
must cover the emulation's error against the FP64 definition on random
states, and must not be vacuous (a small fraction of the cost's scale).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_util import eval_err32

F32 = np.float32


def emulate32(func, x, shift):
    x = np.asarray(x, dtype=np.float32)
    n = x.size
    sh = np.zeros(n, dtype=np.float32) if shift is None else np.asarray(shift, dtype=np.float32)
    y = (x - sh).astype(np.float32)

    def fma(a, b, c):  # one rounding
        return F32(np.float64(a) * np.float64(b) + np.float64(c))

    def hw_cos_rev(t):
        return F32(np.cos(2 * np.pi * (np.float64(t) - np.round(np.float64(t)))))

    def hw_sin_rev(t):
        return F32(np.sin(2 * np.pi * (np.float64(t) - np.round(np.float64(t)))))

    def hw_sqrt(t):
        return F32(np.sqrt(np.float64(t)))

    def expm1_32(t):  # the kernels' FP32 e^t - 1
        if abs(t) <= 0.5:
            p = F32(1.0 / 362880.0)
            for k in (40320.0, 5040.0, 720.0, 120.0, 24.0, 6.0, 2.0, 1.0):
                p = fma(t, p, F32(1.0 / k))
            return F32(t * p)
        return F32(F32(np.exp2(np.float64(F32(t * F32(1.4426950408889634))))) - F32(1))

    if func in (O.SHEKEL5, O.SHEKEL7, O.SHEKEL10, O.FOXHOLES, O.LANGERMAN):
        A, C = O.centres(func)
        A32, C32 = A.astype(np.float32), C.astype(np.float32)
        acc = F32(0)
        for i in range(C.size):
            d = F32(0)
            for j in range(n):
                t = F32(y[j] - A32[i, j])
                d = fma(t, t, d)
            if func == O.LANGERMAN:
                h = F32(F32(0.5) * d)
                r = F32(h - F32(np.rint(h)))
                e = F32(np.exp2(np.float64(F32(d * F32(-np.log2(np.e) / np.pi)))))
                term = F32(F32(C32[i] * e) * hw_cos_rev(r))
            else:
                term = F32(1.0 / np.float64(F32(d + C32[i])))
            acc = F32(acc + term)
        return float(-acc)
    if func == O.SCHWEFEL:
        acc = F32(0)
        k = F32(1.0 / (4 * np.pi ** 2))
        for i in range(n):
            acc = fma(y[i], hw_sin_rev(hw_sqrt(F32(abs(y[i]) * k))), acc)
        return float(F32(acc * F32(-1.0 / n)))
    if func == O.RASTRIGIN:
        acc = F32(0)
        for i in range(n):
            sp = hw_sin_rev(F32(0.5) * y[i])
            acc = fma(y[i], y[i], fma(F32(F32(20) * sp), sp, acc))
        return float(acc)
    if func == O.ACKLEY:
        s1, dd = F32(0), F32(0)
        for i in range(n):
            sp = hw_sin_rev(F32(0.5) * y[i])
            s1 = fma(y[i], y[i], s1)
            dd = fma(sp, sp, dd)
        inv_n = F32(1.0 / n)
        ea = expm1_32(F32(F32(-0.2) * hw_sqrt(F32(s1 * inv_n))))
        eb = expm1_32(F32(F32(-2) * F32(dd * inv_n)))
        return float(fma(F32(-20), ea, F32(-F32(np.e) * eb)))
    if func == O.GRIEWANK:
        c = (1.0 / (2 * np.pi * np.sqrt(np.arange(1, n + 1, dtype=np.float64)))).astype(np.float32)
        s, p = F32(0), F32(1)
        for i in range(n):
            s = fma(y[i], y[i], s)
            p = F32(p * hw_cos_rev(F32(y[i] * c[i])))
        return float(F32(fma(s, F32(2.5e-4), F32(1)) - p))
    if func == O.LEVY_MONTALVO:
        h0 = fma(y[0], F32(0.125), F32(0.125))
        s0 = hw_sin_rev(h0)
        acc = F32(F32(F32(10) * s0) * s0)
        vp = F32(2 * h0)
        for i in range(1, n):
            h = fma(y[i], F32(0.125), F32(0.125))
            si = hw_sin_rev(h)
            acc = fma(F32(vp * vp), fma(F32(F32(10) * si), si, F32(1)), acc)
            vp = F32(2 * h)
        acc = fma(vp, vp, acc)
        return float(F32(acc * F32(np.pi / n)))
    acc = F32(0)
    a = y[0]
    for i in range(1, n):
        b = y[i]
        t = fma(-a, a, b)
        u = F32(F32(1) - a)
        acc = fma(F32(F32(100) * t), t, acc)
        acc = fma(u, u, acc)
        a = b
    return float(acc)


@pytest.mark.parametrize("func,n,shifted", [(O.SHEKEL5, 4, False), (O.SHEKEL7, 4, True), (O.SHEKEL10, 4, False),
                                            (O.FOXHOLES, 2, False), (O.FOXHOLES, 5, True), (O.FOXHOLES, 10, False),
                                            (O.LANGERMAN, 2, False), (O.LANGERMAN, 5, True),
                                            (O.LANGERMAN, 10, False)])
def test_fp32_centre_evaluation_within_bound(func, n, shifted):
    """The centre families on their boxes, near their table centres (where
    the terms peak) and across the box."""
    lo, hi = W.CENTRE_BOX[func]
    A, _ = O.centres(func)
    rng = np.random.default_rng(100 * func + n)
    worst = 0.0
    for trial in range(24):
        shift = rng.uniform(-0.5, 0.5, n).astype(np.float32).astype(np.float64) if shifted else None
        if trial % 2:
            x = A[rng.integers(A.shape[0]), :n] + rng.uniform(-0.05, 0.05, n) + (0.0 if shift is None else shift)
        else:
            x = rng.uniform(lo, hi, n)
        x = np.clip(x, lo, hi).astype(np.float32).astype(np.float64)
        exact = O.f(func, x, shift)
        err = abs(emulate32(func, x, shift) - exact)
        bound = eval_err32(func, x, shift)
        assert err <= bound, (trial, err, bound)
        worst = max(worst, err / bound if bound > 0 else 0.0)
        assert bound <= 1e-4 * max(1.0, abs(exact))
    print(f"func {func} n {n}: max err/bound {worst:.3f}")


@pytest.mark.parametrize("func", [O.GRIEWANK, O.LEVY_MONTALVO, O.ROSENBROCK, O.SCHWEFEL, O.RASTRIGIN, O.ACKLEY])
@pytest.mark.parametrize("n,shifted", [(1, False), (2, True), (17, False), (100, True), (100, False)])
def test_fp32_evaluation_within_bound(func, n, shifted):
    half = W.HALF_BOX[func]
    rng = np.random.default_rng(1000 * func + n)
    worst = 0.0
    for trial in range(12):
        shift = rng.uniform(-0.8 * half, 0.8 * half, n).astype(np.float32).astype(np.float64) if shifted else None
        # states across the box, and near the minimiser (where the increments are small)
        scale = half if trial % 2 == 0 else half * 1e-3
        centre = (0.0 if shift is None else shift) + (1.0 if func == O.ROSENBROCK else
                                                      -1.0 if func == O.LEVY_MONTALVO else
                                                      420.968746 if func == O.SCHWEFEL else 0.0)
        x = np.clip(centre + rng.uniform(-scale, scale, n), -half, half).astype(np.float32).astype(np.float64)
        exact = O.f(func, x, shift)
        err = abs(emulate32(func, x, shift) - exact)
        bound = eval_err32(func, x, shift)
        assert err <= bound, (trial, err, bound)
        worst = max(worst, err / bound if bound > 0 else 0.0)
        # not vacuous: far below the cost's own scale (Schwefel: that of its
        # terms, -y sin(sqrt|y|)/n, which cancel in the sum)
        size = max(1.0, abs(exact), float(np.mean(np.abs(x - (0.0 if shift is None else shift))))
                   if func == O.SCHWEFEL else 0.0)
        assert bound <= 1e-4 * size + (2e-3 if func == O.GRIEWANK else 0.0)
    print(f"func {func} n {n}: max err/bound {worst:.3f}")


def _oracle_learned_log(func, n, lo, hi, shift, params, eps, T, featT, steps, chains, seed=3, level=1):
    """The oracle's own learned level, logged in the device's move-record layout."""
    from paper_2408_00018_amd.sa import MOVE_DTYPE
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(lo, hi)
    out = O.learned_run(params, O.NET_DEVICE, func, lo, hi, shift, seed=seed, level=level, nchains=chains,
                        steps=steps, T=T, featT=featT, eps=eps, x_start=x0, log=True)
    mv = np.zeros((chains, steps), dtype=MOVE_DTYPE)
    for key in ("d", "accept", "x_old", "x_new", "df"):
        mv[key] = out[key].reshape(chains, steps)
    return x0, mv, out["f_final"]


@pytest.mark.parametrize("func,n,lo,hi", [(O.SCHWEFEL, 8, -500.0, 500.0), (O.ACKLEY, 6, -32.768, 32.768)])
def test_learned_checker_accepts_the_oracle_and_rejects_a_flipped_decision(func, n, lo, hi):
    """check_learned_level, fed the oracle's own learned level (the device's
    record layout), passes; the same log with one firm decision flipped
    fails.  The checker itself holds no Metropolis-Hastings arithmetic: it
    asks the oracle's learned move for every decision."""
    import parity_util as P
    lo_v, hi_v = np.full(n, lo), np.full(n, hi)
    p = P.bf16_matrices(P.learned_params(11, scale=0.05, sigma0=0.02))
    T, eps, steps = 2.0, 0.25, 24
    featT = float(np.float32(np.log(O.feature_tau(func, n) * T)))
    x0, mv, ff = _oracle_learned_log(func, n, lo_v, hi_v, None, p, eps, T, featT, steps, chains=3)
    st = P.check_learned_level(func, n, lo_v, hi_v, None, 3, 1, T, featT, eps, p, 0.1, x0, mv, ff, [0, 1, 2])
    assert st["learned"] > 0 and st["moves"] == 3 * steps
    # flip the decision of chain 0's first move: the checker must object (at
    # that decision, at a later move whose logged old value no longer follows,
    # or at the final cost)
    bad = mv.copy()
    bad[0, 0]["accept"] ^= 1
    with pytest.raises(AssertionError):
        P.check_learned_level(func, n, lo_v, hi_v, None, 3, 1, T, featT, eps, p, 0.1, x0, bad, ff, [0])
