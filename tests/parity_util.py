"""Shared checks of the GPU path against the FP64 oracle.

The GPU side is reached only through the C ABI binding
(``paper_2408_00018_amd.sa``); the expected values come only from ``oracle``.
"""
from __future__ import annotations

import math

import numpy as np

import oracle as O

U32 = 2.0 ** -24  # FP32 unit roundoff
# Error bounds of the FP32 hardware transcendentals, checked against FP64 on
# the GPU by tests/test_gpu_trig.py: absolute for sine/cosine on arguments up
# to 64 revolutions (E_TRIG) and up to 256 (E_TRIG_WIDE, Griewank's
# cos(y/sqrt(i)) at |y| up to 1200), relative for sqrt and 2^t.  The
# sine/cosine bounds are the measured maximum (2.10 x 2^-24 at every range)
# with a margin of 1.9 (E_TRIG) and 3.8 (E_TRIG_WIDE).
E_TRIG = 2.0 ** -21
E_TRIG_WIDE = 2.0 ** -20
E_SQRT = 2.0 ** -22
E_EXP2 = 2.0 ** -21
# Relative error of the FP32 e^x - 1 of the Ackley increment (polynomial for
# |x| <= 1/2, hardware exponential minus one beyond); the Ackley floor below
# allows 36 and 68 of 2^-24 on its two terms.
E_EXPM1 = 2.0 ** -20
# v_log_f32, relative, over (0, 1] (the Box-Muller radius of the Gaussian
# proposal network; tests/test_gpu_trig.py)
E_LOG2 = 2.0 ** -21
# v_rcp_f32, relative (the centre families' 1/(d + c); documented as 1 ulp,
# checked by tests/test_gpu_trig.py)
E_RCP = 2.0 ** -22


def f32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def box32(lower, upper):
    """The FP32 box the library uses: bounds rounded inward."""
    lo = np.asarray(lower, dtype=np.float64)
    hi = np.asarray(upper, dtype=np.float64)
    l32 = lo.astype(np.float32)
    l32 = np.where(l32.astype(np.float64) < lo, np.nextafter(l32, np.float32(np.inf)), l32)
    h32 = hi.astype(np.float32)
    h32 = np.where(h32.astype(np.float64) > hi, np.nextafter(h32, np.float32(-np.inf)), h32)
    return l32.astype(np.float64), h32.astype(np.float64)


CENTRE_FAMILIES = (O.SHEKEL5, O.SHEKEL7, O.SHEKEL10, O.FOXHOLES, O.LANGERMAN)
COUPLED = (O.GRIEWANK, O.LEVY_MONTALVO, O.ROSENBROCK) + CENTRE_FAMILIES


def eval_err32(func, x, shift):
    """First-order bound on the absolute error of the FP32 full evaluation of
    the full-evaluation kernel at state x (FP64 copy of the FP32 state),
    following its operation order: y = x - s rounded, then per coordinate
      Schwefel     acc = fma(y, sin_rev(sqrt(|y| fl(1/(4 pi^2)))), acc); f = acc fl(-1/n)
      Rastrigin    S = sin_rev(y/2); acc = fma(y, y, fma(20 S, S, acc))
      Ackley       S = sin_rev(y/2); s1 = fma(y, y, s1); D = fma(S, S, D);
                   f = fma(-20, expm1(-0.2 sqrt(s1 fl(1/n))), -fl(e) expm1(-2 D fl(1/n)))
      Griewank     s += y^2 (fma); p *= cos_rev(y c_i), c_i = fl(1/(2 pi sqrt(i)));
                   f = fma(s, fl(1/4000), 1) - p
      Levy         h = fma(y, 1/8, 1/8) = v/2; S = sin_rev(h);
                   acc = fma(v_prev^2, fma(10 S, S, 1), acc); f = acc fl(pi/n)
      Rosenbrock   t = fma(-a, a, b); acc = fma(100 t, t, acc); acc = fma(u, u, acc)
      centres      per centre i: t = y - fl(a_ij); d = fma(t, t, d) over j; then
                   Shekel/foxholes  acc += rcp(d + fl(c_i));
                   Langerman        acc += fl(c_i) exp2(d fl(-log2(e)/pi)) cos_rev(d/2 - rint(d/2));
                   f = -acc
    (v_rcp_f32 relative error E_RCP.)  Every rounding contributes U32 times the magnitude of its result, the
    hardware sine/cosine E_TRIG (E_TRIG_WIDE past 64 revolutions) absolutely,
    sqrt E_SQRT and e^x - 1 E_EXPM1 relatively, and errors propagate through
    first derivatives.  Sums of n roundings are bounded by n U32 times the sum
    of the magnitudes."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    y = x - (0.0 if shift is None else np.asarray(shift, dtype=np.float64))
    dy = U32 * np.abs(y) if shift is not None else np.zeros(n)
    ay = np.abs(y)
    if func == O.SCHWEFEL:
        r = np.sqrt(ay / (4 * np.pi ** 2))  # the sine's argument in revolutions
        S = np.sin(2 * np.pi * r)
        rel_r = E_SQRT + 0.5 * (2 * U32 + np.divide(dy, ay, out=np.zeros(n), where=ay > 0))
        dS = E_TRIG + 2 * np.pi * r * np.abs(np.cos(2 * np.pi * r)) * rel_r
        h = np.abs(y * S)
        f = -float(np.sum(y * S)) / n
        return (float(np.sum(np.abs(S) * dy + ay * dS)) + n * U32 * float(np.sum(h))) / n + 2 * U32 * abs(f)
    if func in (O.RASTRIGIN, O.ACKLEY):
        S = np.sin(np.pi * y)
        dS = np.pi * np.abs(np.cos(np.pi * y)) * dy + E_TRIG
        if func == O.RASTRIGIN:
            g = y * y + 20 * S * S
            dg = 2 * ay * dy + 40 * np.abs(S) * dS + 20 * S * S * U32
            return float(np.sum(dg)) + 2 * n * U32 * float(np.sum(g))
        s1, D = float(np.sum(y * y)), float(np.sum(S * S))
        ds1 = float(np.sum(2 * ay * dy)) + n * U32 * s1
        dD = float(np.sum(2 * np.abs(S) * dS)) + n * U32 * D
        u = s1 / n
        du = ds1 / n + 2 * U32 * u
        q = math.sqrt(u)
        dq = (min(du / (2 * q), math.sqrt(du)) if q > 0 else math.sqrt(du)) + E_SQRT * q
        a = -0.2 * q
        da = 0.2 * dq + 2 * U32 * 0.2 * q
        ea = math.expm1(a)
        dea = math.exp(a) * da + E_EXPM1 * abs(ea)
        b = -2 * D / n
        db = 2 * dD / n + 2 * U32 * abs(b)
        eb = math.expm1(b)
        deb = math.exp(b) * db + E_EXPM1 * abs(eb)
        f = -20 * ea - math.e * eb
        return 20 * dea + math.e * deb + 2 * U32 * math.e * abs(eb) + U32 * abs(f)
    if func in CENTRE_FAMILIES:
        A, C = O.centres(func)
        A = A[:, :n]
        T = y[None, :] - A
        dT = dy[None, :] + U32 * np.abs(A) + U32 * np.abs(T)
        D = np.sum(T * T, axis=1)
        dD = np.sum(2 * np.abs(T) * dT, axis=1) + n * U32 * D
        if func == O.LANGERMAN:
            K = math.log2(math.e) / math.pi
            e = np.exp(-D / math.pi)
            cs = np.cos(math.pi * D)
            de = e * (math.log(2) * (K * dD + 2 * U32 * K * D) + E_EXP2)
            dcs = math.pi * dD + E_TRIG
            term = C * e * cs
            dterm = C * (de * np.abs(cs) + e * dcs) + U32 * C * e * np.abs(cs) + 2 * U32 * np.abs(term)
        else:
            u = D + C
            r = 1.0 / u
            du = dD + U32 * C + U32 * u
            term = r
            dterm = r * r * du + E_RCP * r
        m = C.size
        return float(np.sum(dterm)) + m * U32 * float(np.sum(np.abs(term)))
    if func == O.GRIEWANK:
        idx = np.arange(1, n + 1, dtype=np.float64)
        th = y / np.sqrt(idx)
        S = float(np.sum(y * y))
        c = np.cos(th)
        # leave-one-out products of |cos| through prefix/suffix products
        a = np.abs(c)
        pre = np.concatenate([[1.0], np.cumprod(a)[:-1]])
        suf = np.concatenate([np.cumprod(a[::-1])[::-1][1:], [1.0]])
        loo = pre * suf
        rev = np.abs(th) / (2 * np.pi)
        e_trig = np.where(rev <= 64.0, E_TRIG, E_TRIG_WIDE)
        dth = np.abs(th) * 3 * U32 + dy / np.sqrt(idx)
        e_p = float(np.sum(loo * (np.abs(np.sin(th)) * dth + e_trig))) + n * U32 * float(np.prod(a))
        e_s = (n + 2) * U32 * S + float(np.sum(2 * np.abs(y) * dy))
        f = 1.0 + S / 4000.0 - float(np.prod(c))
        return e_p + e_s / 4000.0 + U32 * S / 4000.0 + U32 * (1.0 + S / 4000.0) + U32 * abs(f)
    if func == O.LEVY_MONTALVO:
        v = (y + 1.0) / 4.0
        dh = U32 * (np.abs(y) / 8.0 + np.abs(v) / 2.0) + dy / 8.0
        dv = 2 * dh
        S = np.sin(np.pi * v)
        dS = 2 * np.pi * np.abs(np.cos(np.pi * v)) * dh + E_TRIG
        q = 1.0 + 10.0 * S * S
        dq = 20 * np.abs(S) * dS + U32 * (10 * S * S + q)
        terms = np.concatenate([[10 * S[0] ** 2], v[:-1] ** 2 * q[1:], [v[-1] ** 2]])
        dterms = np.concatenate([[20 * abs(S[0]) * dS[0] + U32 * 10 * S[0] ** 2],
                                 2 * np.abs(v[:-1]) * dv[:-1] * q[1:] + v[:-1] ** 2 * dq[1:]
                                 + 2 * U32 * v[:-1] ** 2 * q[1:],
                                 [2 * abs(v[-1]) * dv[-1]]])
        tot = float(np.sum(terms))
        return (np.pi / n) * (float(np.sum(dterms)) + (n + 3) * U32 * tot)
    # Rosenbrock
    if n < 2:
        return 0.0
    aa, bb = y[:-1], y[1:]
    da, db = dy[:-1], dy[1:]
    t = bb - aa * aa
    u = 1.0 - aa
    dt = 2 * np.abs(aa) * da + db + U32 * (np.abs(t) + aa * aa)
    du = da + U32 * np.abs(u)
    terms = 100 * t * t + u * u
    dterms = 100 * (2 * np.abs(t) * dt + 2 * U32 * t * t) + 2 * np.abs(u) * du
    return float(np.sum(dterms)) + 2 * (n + 1) * U32 * float(np.sum(terms))


def df_floor(func, n, x, xn, d, shift, full=False):
    """Absolute error floor of an FP32 cost increment, from the rounding of its
    inputs and the hardware transcendental error (the relative 1e-5 is added
    on top): twice a first-order bound (the factor 2 covers the second-order
    terms the bound leaves out).  x, xn: FP64 copies of the FP32 states
    before/after the move.
    Non-separable families, and every family with `full` (a run under
    SA_FLAG_FULL_EVAL): the increment is the difference of two full FP32
    evaluations (the carried cost is the last one, or the FP64 start value
    rounded to FP32), so the floor is the sum of their error bounds, doubled
    for the first-order analysis."""
    if func in COUPLED or full:
        return 2.0 * (eval_err32(func, x, shift) + eval_err32(func, xn, shift))
    s = 0.0 if shift is None else shift[d]
    y, yn = x[d] - s, xn[d] - s
    if func == O.SCHWEFEL:
        def t(v):
            a = abs(v)
            return a * (math.sqrt(a) * 4 * U32 + E_TRIG) + a * 2 * U32
        return 2.0 * (t(y) + t(yn)) / n
    if func == O.RASTRIGIN:
        dl, sg = abs(yn - y), abs(yn + y)
        ddl = U32 * (abs(y) + abs(yn) + dl)
        dsg = U32 * (abs(y) + abs(yn) + sg)
        return 2.0 * (sg * ddl + dl * dsg + dl * sg * 2 * U32 + 20 * (math.pi * (ddl + dsg) + 2 * E_TRIG)
                      + 40 * U32)
    # Ackley, increment formed from the two sums (S1 = sum y^2, S2 = sum cos 2 pi y):
    # errors of dS1 = dl sg and dS2 = -2 sin(pi sg) sin(pi dl), plus the FP32
    # rounding/drift of the carried sums (<= 64 roundings per level) acting on
    # e^a = exp(-0.2 sqrt(S1/n)) and e^b = exp(S2/n).
    ys = x - (0.0 if shift is None else shift)
    s1 = float(np.dot(ys, ys))
    s2 = float(np.sum(np.cos(2 * math.pi * ys)))
    q = math.sqrt(s1 / n)
    s1n = s1 + (yn * yn - y * y)
    qn = math.sqrt(max(s1n, 0.0) / n)
    ea, eb = math.exp(-0.2 * q), math.exp(s2 / n)
    dl, sg = abs(yn - y), abs(yn + y)
    ddl = U32 * (abs(y) + abs(yn) + dl)
    dsg = U32 * (abs(y) + abs(yn) + sg)
    ds1 = dl * sg
    e_ds1 = sg * ddl + dl * dsg + U32 * ds1
    ds2 = 2.0 * abs(math.sin(math.pi * sg) * math.sin(math.pi * dl))
    e_ds2 = 2.0 * (math.pi * (ddl + dsg) + 2 * E_TRIG) + 3 * U32 * ds2
    den = max(q + qn, 1e-30)
    da = 0.2 * (ds1 / n) / den
    term_a = 20.0 * ea * da * (6.4 * q * U32 + 36 * U32) + 20.0 * ea * 0.2 * e_ds1 / (n * den)
    term_b = eb * (ds2 / n) * 68 * U32 + eb * e_ds2 / n
    return 2.0 * (term_a + term_b)


def check_fp32_level(func, n, lower32, upper32, shift32, seed, level, T, move_rule, radius_frac, x_start, moves,
                     final_f, chain_ids, rel=1e-5, problem=0, start_err=None, best_seen=False, full=False):
    """Replay the logged moves of `chain_ids` at one level against the oracle.

    x_start: the level's start state (the previous level's broadcast winner,
    or the chain's own state, FP32 values).  start_err: bound on the error of
    the start cost the chain carries in (default: one FP32 rounding of a full
    evaluation, as after a broadcast).  Returns statistics, with each chain's
    error bound on its final cost in stats["f_err"]; raises AssertionError on
    a mismatch.  best_seen: final_f holds each chain's best-seen cost (the
    lowest cost it carried during the level, start included), which must match
    the lowest FP64 cost of the states it visited within the same bound;
    stats["visited"][c] lists those states and stats["f_last"][c] bounds
    the final state's FP64 cost.  full: the increments are differences of full
    FP32 evaluations (SA_FLAG_FULL_EVAL)."""
    stats = dict(moves=0, max_rel_excess=0.0, decision_mismatch=0, ambiguous=0, max_df_err=0.0, f_err={},
                 x_final={}, visited={}, f_last={})
    for j, c in enumerate(chain_ids):
        x = np.array(x_start, dtype=np.float64)
        f_acc_err = 0.0
        visited = [x.copy()]
        vis_f = [O.f(func, x, shift32)] if best_seen else []
        for s in range(moves.shape[-1]):
            m = moves[j, s]
            d_ref, u1, u2 = O.move_draw(seed, problem, level, c, s, n)
            assert int(m["d"]) == d_ref, (level, c, s)
            assert m["x_old"] == x[d_ref], (level, c, s)
            xn_ref = O.neighbour(move_rule, float(m["x_old"]), float(lower32[d_ref]), float(upper32[d_ref]),
                                 radius_frac, u1)
            rho = radius_frac * (upper32[d_ref] - lower32[d_ref])
            tol_x = 2.0 ** -23 * (abs(xn_ref) + rho)
            assert abs(m["x_new"] - xn_ref) <= tol_x, (level, c, s, m["x_new"], xn_ref)
            assert lower32[d_ref] <= m["x_new"] <= upper32[d_ref]
            xn = x.copy()
            xn[d_ref] = m["x_new"]
            df_ref = O.f(func, xn, shift32) - O.f(func, x, shift32)
            floor = df_floor(func, n, x, xn, d_ref, shift32, full)
            err = abs(m["df"] - df_ref)
            tol = rel * abs(df_ref) + floor
            stats["max_df_err"] = max(stats["max_df_err"], err)
            stats["max_rel_excess"] = max(stats["max_rel_excess"], err / tol if tol > 0 else 0.0)
            assert err <= tol, (level, c, s, float(m["df"]), df_ref, floor)
            # Metropolis decision: equal wherever the oracle's decision cannot
            # be flipped by an increment error within tolerance.
            acc_ref = O.accept(df_ref, T, u2)
            # plus the FP32 rounding of 1/T and of the hardware exp2 (a few ulp)
            margin = tol + 2.0 ** -18 * T
            lo_df, hi_df = df_ref - margin, df_ref + margin
            firm = O.accept(lo_df, T, u2) == O.accept(hi_df, T, u2)
            if firm:
                if bool(m["accept"]) != acc_ref:
                    stats["decision_mismatch"] += 1
            else:
                stats["ambiguous"] += 1
            assert not firm or bool(m["accept"]) == acc_ref, (level, c, s, float(m["df"]), df_ref, u2, T)
            if m["accept"]:
                x = xn
                f_acc_err += tol + 2 * U32 * abs(O.f(func, x, shift32))
                if best_seen:
                    visited.append(x.copy())
                    vis_f.append(O.f(func, x, shift32))
            stats["moves"] += 1
        f_ref = O.f(func, x, shift32)
        s_err = 2 * U32 * abs(O.f(func, x_start, shift32)) + 1e-12 if start_err is None else start_err
        bound = f_acc_err + s_err + 2 * U32 * abs(f_ref)
        if best_seen:
            # the carried costs of the visited states are each within this bound
            bound = f_acc_err + s_err + 2 * U32 * max(abs(v) for v in vis_f)
            assert abs(final_f[c] - min(vis_f)) <= bound, (level, c, final_f[c], min(vis_f), bound)
            stats["visited"][c] = visited
        else:
            assert abs(final_f[c] - f_ref) <= bound, (level, c)
        stats["f_err"][c] = bound
        stats["f_last"][c] = f_ref
        stats["x_final"][c] = x
    return stats


def lexi_argmin(values):
    m = np.min(values)
    return int(np.flatnonzero(values == m)[0])


def fp32_init_state(wl, chain, problem=0):
    """Level-0 start of one chain as the FP32 path forms it: l + (u - l) U in
    FP32 arithmetic, from the oracle's Philox draws (start counters)."""
    lo32, hi32 = box32(wl.lower, wl.upper)
    x = np.zeros(wl.n, dtype=np.float32)
    for i in range(wl.n):
        r = O.philox4x32_10([i >> 2, 0xFFFFFFFF, chain, 1 | (problem << 8)], [wl.seed & 0xFFFFFFFF, wl.seed >> 32])
        u = np.float32(O.uniform(int(r[i & 3])))
        v = np.float32(lo32[i]) + (np.float32(hi32[i]) - np.float32(lo32[i])) * u
        x[i] = min(max(v, np.float32(lo32[i])), np.float32(hi32[i]))
    # the FP64 start differs from it by at most one FP32 rounding per operation
    x64 = O.init_point(wl.seed, problem, chain, lo32, hi32)
    assert np.all(np.abs(x.astype(np.float64) - x64) <= 2.0 ** -22 * (np.abs(x64) + (hi32 - lo32)))
    return x.astype(np.float64)


def check_fp32_run(wl, g, log_level, chain_ids=None, problem=0, move_rule=O.MOVE_RADIUS, say=print, full=False):
    """Per-move replay of a logged FP32 run (moves, final costs, per-level
    trace and broadcast states in g) against the oracle, plus the level
    argmin and the full re-evaluation of each broadcast."""
    lo32, hi32 = box32(wl.lower, wl.upper)
    sh32 = None if wl.shift is None else f32(wl.shift)
    moves, final_f = g["moves"], g["final_f"]
    rec, xb = g["rec"], g["xb"]
    nlog = moves.shape[0]
    if chain_ids is None:
        chain_ids = list(range(moves.shape[1]))
    totals = dict(moves=0, ambiguous=0, max_rel_excess=0.0)
    for k in range(nlog):
        level = log_level + k
        T = O.temperature(wl.T0, wl.alpha, level)
        # device-wide argmin of the level: bit-exact on the GPU's own final costs
        win = lexi_argmin(final_f[k])
        assert rec["win_chain"][level] == win
        assert rec["f_win"][level] == final_f[k][win]
        # broadcast state re-evaluated in full (FP64 on the device)
        fb = O.f(wl.func, xb[level], sh32)
        assert abs(rec["f_best"][level] - fb) <= 1e-11 * max(1.0, abs(fb))
        for c in chain_ids:
            x_start = fp32_init_state(wl, c, problem) if level == 0 else xb[level - 1]
            st = check_fp32_level(wl.func, wl.n, lo32, hi32, sh32, wl.seed, level, T, move_rule, wl.radius_frac,
                                  x_start, moves[k, c:c + 1], final_f[k], [c], problem=problem, full=full)
            totals["moves"] += st["moves"]
            totals["ambiguous"] += st["ambiguous"]
            totals["max_rel_excess"] = max(totals["max_rel_excess"], st["max_rel_excess"])
    say(f"[fp32 parity] {wl.name} problem {problem}: {totals}")
    return totals


def check_record(wl, g):
    """Record invariants: states in the box, monotone record equal to the
    running minimum of the re-evaluated winners, x_rec/f_rec consistent."""
    rec, xb = g["rec"], g["xb"]
    lo32, hi32 = box32(wl.lower, wl.upper)
    if wl.precision == 1:
        lo32, hi32 = np.asarray(wl.lower), np.asarray(wl.upper)
    assert np.all(xb >= lo32) and np.all(xb <= hi32)
    assert np.all(np.diff(rec["f_rec"]) <= 0)
    assert np.array_equal(rec["f_rec"], np.minimum.accumulate(rec["f_best"]))
    lvl = g["rec_level"]
    assert np.array_equal(g["x_rec"], xb[lvl])
    assert g["f_rec"] == rec["f_best"][lvl]
    sh = None if wl.shift is None else (f32(wl.shift) if wl.precision == 0 else np.asarray(wl.shift))
    fr = O.f(wl.func, g["x_rec"], sh)
    assert abs(g["f_rec"] - fr) <= 1e-11 * max(1.0, abs(fr))
    assert np.all(np.diff(rec["t_ns"].astype(np.int64)) >= 0)


def learned_params(seed, scale=0.1, mu0=0.0, sigma0=0.05):
    """A proposal network for parity tests: random weights, output biases that
    centre the proposal at mu0 with scale sigma0 (so most proposals land in
    the box and the Metropolis-Hastings branch is exercised)."""
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, scale, O.mlp_nparam())
    p[-2], p[-1] = mu0, math.log(sigma0)
    return p.astype(np.float32)


def bf16_matrices(params):
    """Parameters as the device uses them: the three weight matrices rounded
    to BF16 (ties to even), biases FP32; returned in float64."""
    p = np.asarray(params, dtype=np.float32).copy()
    H, I = O.MLP_HIDDEN, O.MLP_INPUTS
    for a, b in ((0, I * H), (I * H + H, I * H + H + H * H), (I * H + 2 * H + H * H, I * H + 2 * H + H * H + 2 * H)):
        u = p[a:b].view(np.uint32).astype(np.uint64)
        u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
        p[a:b] = u.astype(np.uint32).view(np.float32)
    return p.astype(np.float64)


def gauss_draw_error(seed, problem, level, chain, step):
    """Bound on the FP32 Box-Muller draw's error (the Gaussian network kind):
    t = sqrt(-2 ln(1 - U0)) cos(2 pi U2), with ln from the hardware log2
    (relative E_LOG2, then two roundings), the hardware square root (E_SQRT)
    and cosine (absolute E_TRIG), and the final product's rounding."""
    w = O.philox4x32_10([step, level, chain, 3 | (problem << 8)], [seed & 0xFFFFFFFF, seed >> 32])
    u0, u2 = O.uniform(w[0]), O.uniform(w[2])
    rad = math.sqrt(-2.0 * math.log(1.0 - u0))
    cv = abs(math.cos(2.0 * math.pi * u2))
    drad = rad * (0.5 * (E_LOG2 + 3 * U32) + E_SQRT)
    return rad * E_TRIG + cv * drad + 2 * U32 * rad


def check_learned_level(func, n, lower32, upper32, shift32, seed, level, T, featT, eps32, params64, radius_frac,
                        x_start, moves, final_f, chain_ids, problem=0, kind=O.NET_RELU_CAUCHY):
    """Replay the logged moves of a learned-mixture level against the oracle's
    learned move (oracle.learned_propose / oracle.learned_accept with the
    network under the device's stated precision, NET_DEVICE, and its bounds),
    for network kind `kind` (the relu/Cauchy network or the GELU/Gaussian one).

    Each move: the coordinate and the plain/learned choice are bit-exact; a
    plain move is checked as in check_fp32_level; a learned move's proposal
    must equal the oracle's mu + e^s t within the bounds the oracle gives for
    mu and s, a proposal outside the box must be rejected with df = 0, and an
    in-box decision must equal the oracle's Metropolis-Hastings decision
    wherever those bounds (and the FP32 increment's) cannot flip it.  The
    chain state and history follow the GPU's own accepted moves.  Returns
    statistics."""
    O.set_net_kind(kind)
    try:
        return _check_learned_level(func, n, lower32, upper32, shift32, seed, level, T, featT, eps32, params64,
                                    radius_frac, x_start, moves, final_f, chain_ids, problem, kind)
    finally:
        O.set_net_kind(O.NET_RELU_CAUCHY)


def _check_learned_level(func, n, lower32, upper32, shift32, seed, level, T, featT, eps32, params64, radius_frac,
                         x_start, moves, final_f, chain_ids, problem, kind):
    gauss = kind == O.NET_GELU_GAUSS
    stats = dict(moves=0, learned=0, outside=0, ambiguous=0, max_dl_excess=0.0, max_rel_excess=0.0)
    nd = O.NET_DEVICE
    for j, c in enumerate(chain_ids):
        x = np.array(x_start, dtype=np.float64)
        h = [0.0, 0.0, 0.0, 0.0]
        f_acc_err = 0.0
        for s in range(moves.shape[-1]):
            m = moves[j, s]
            pr = O.learned_propose(params64, nd, seed=seed, problem=problem, level=level, chain=c, step=s, x=x,
                                   lower=lower32, upper=upper32, radius_frac=radius_frac, featT=featT, eps=eps32,
                                   hist=h)
            d = pr["d"]
            assert int(m["d"]) == d, (level, c, s)
            assert m["x_old"] == x[d], (level, c, s)
            lo, hi = float(lower32[d]), float(upper32[d])
            w = hi - lo
            xn = x.copy()
            xn[d] = m["x_new"]
            x_old, x_new = float(m["x_old"]), float(m["x_new"])
            if pr["plain"]:
                assert abs(x_new - pr["x_new"]) <= 2.0 ** -23 * (abs(pr["x_new"]) + radius_frac * w), (level, c, s)
                take, det = O.learned_accept(params64, nd, func, lower=lower32, upper=upper32, shift=shift32, seed=seed,
                                             problem=problem, level=level, chain=c, step=s, T=T, featT=featT,
                                             plain=True, x=x, d=d, x_new=x_new, mu=0.0, s=0.0, hist=h)
                df_ref = det["df"]
                tol = 1e-5 * abs(df_ref) + df_floor(func, n, x, xn, d, shift32)
                assert abs(m["df"] - df_ref) <= tol, (level, c, s, float(m["df"]), df_ref)
                stats["max_rel_excess"] = max(stats["max_rel_excess"], abs(m["df"] - df_ref) / tol)
                margin = tol + 2.0 ** -18 * T
                u2 = det["u2"]
                firm = O.accept(df_ref - margin, T, u2) == O.accept(df_ref + margin, T, u2)
                if firm:
                    assert bool(m["accept"]) == take, (level, c, s)
                else:
                    stats["ambiguous"] += 1
            else:
                stats["learned"] += 1
                mu, sl, t, bmu, bs = pr["mu"], pr["s"], pr["t"], pr["b_mu"], pr["b_s"]
                sig = math.exp(sl)
                dl_ref = (pr["x_new"] - x_old) / w
                dl_gpu = (x_new - x_old) / w
                # rounding of x' = x + dl w and of the logged positions, in dl units
                ddl = 4 * U32 * (abs(x_old) + abs(x_new)) / w
                # network bounds on mu and s (e^s within e^{+-bs}); the draw t's
                # FP32 error -- Cauchy: the hardware sin/cos quotient (relative
                # error growing like |t| towards the poles); Gaussian: the
                # Box-Muller bound --; FP32 rounding of the fused multiply-add
                if gauss:
                    dt = gauss_draw_error(seed, problem, level, c, s)
                else:
                    dt = 2.0 ** -18 * (1 + abs(t) + t * t)
                tol_dl = (bmu + sig * abs(t) * (math.expm1(bs) + 2.0 ** -18) + sig * dt + 4 * U32 * abs(dl_ref)
                          + ddl)
                err = abs(dl_gpu - dl_ref)
                stats["max_dl_excess"] = max(stats["max_dl_excess"], err / tol_dl)
                assert err <= tol_dl, (level, c, s, dl_gpu, dl_ref, tol_dl)
                inside = lo <= x_new <= hi
                if not inside:
                    stats["outside"] += 1
                    assert m["accept"] == 0 and m["df"] == 0.0, (level, c, s)
                    tol = 0.0
                else:
                    take, det = O.learned_accept(params64, nd, func, lower=lower32, upper=upper32, shift=shift32,
                                                 seed=seed, problem=problem, level=level, chain=c, step=s, T=T,
                                                 featT=featT, plain=False, x=x, d=d, x_new=x_new, mu=mu, s=sl, hist=h)
                    df_ref = det["df"]
                    tol = 1e-5 * abs(df_ref) + df_floor(func, n, x, xn, d, shift32)
                    assert abs(m["df"] - df_ref) <= tol, (level, c, s, float(m["df"]), df_ref)
                    stats["max_rel_excess"] = max(stats["max_rel_excess"], abs(m["df"] - df_ref) / tol)
                    mu2, s2, bmu2, bs2 = det["mu2"], det["s2"], det["b_mu2"], det["b_s2"]
                    # first-order sensitivity of the two log densities to their
                    # location and log scale (and to dl's rounding)
                    e1 = (dl_gpu - mu) * math.exp(-sl)
                    e2 = (-dl_gpu - mu2) * math.exp(-s2)
                    if gauss:  # ln q = -s - r^2/2 + const: d/dmu = r e^-s, d/ds = r^2 - 1
                        tol_lq = (abs(e1) * math.exp(-sl) * (bmu + ddl) + abs(e1 * e1 - 1) * bs
                                  + abs(e2) * math.exp(-s2) * (bmu2 + ddl) + abs(e2 * e2 - 1) * bs2)
                    else:
                        tol_lq = (2 * abs(e1) * math.exp(-sl) / (1 + e1 * e1) * (bmu + ddl)
                                  + abs(1 - 2 * e1 * e1 / (1 + e1 * e1)) * bs
                                  + 2 * abs(e2) * math.exp(-s2) / (1 + e2 * e2) * (bmu2 + ddl)
                                  + abs(1 - 2 * e2 * e2 / (1 + e2 * e2)) * bs2)
                    r = det["log_ratio"]
                    tol_r = 2 * tol_lq + tol / T + 2.0 ** -16 * (1 + abs(r))
                    u2 = det["u2"]
                    lu = math.log(u2) if u2 > 0 else -math.inf
                    if abs(lu - r) > tol_r:
                        assert bool(m["accept"]) == take, (level, c, s, lu, r, tol_r)
                    else:
                        stats["ambiguous"] += 1
            if m["accept"]:
                h = [(x_new - x_old) / w] + h[:3]
                x = xn
                f_acc_err += tol + 2 * U32 * abs(O.f(func, x, shift32))
            stats["moves"] += 1
        f_ref = O.f(func, x, shift32)
        start_err = 2 * U32 * abs(O.f(func, x_start, shift32)) + 1e-12
        assert abs(final_f[c] - f_ref) <= f_acc_err + start_err + 2 * U32 * abs(f_ref), (level, c, final_f[c], f_ref)
    return stats
