"""FP64 CPU oracle for synchronous parallel simulated annealing.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg load it; the GPU library never does.  It shares no code with
the GPU library.  The arithmetic lives in ``sa_oracle.c`` (plain C, FP64); this
module only marshals arguments through ctypes.

Paper: Ferreiro, Garcia, Lopez-Salas, Vazquez, "An efficient implementation of
parallel simulated annealing algorithm in GPUs" -- Sec. 2.1 (sequential SA,
eqs. (4)-(5), Steps 1-5), Sec. 2.2.2 (synchronous multiple Markov chains),
Sec. 3.3 (synchronous kernel listing), Sec. 4.1 eq. (6) (normalized Schwefel),
Appendix Tests 1 and 13 (Ackley, Rastrigin).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SCHWEFEL, RASTRIGIN, ACKLEY = 0, 1, 2
GRIEWANK, LEVY_MONTALVO, ROSENBROCK = 3, 4, 5
SHEKEL5, SHEKEL7, SHEKEL10, FOXHOLES, LANGERMAN = 6, 7, 8, 9, 10  # centre families (Tests 18, 19, 11)
MOVE_RADIUS, MOVE_RESAMPLE = 0, 1

CFLAGS = ["-O2", "-shared", "-fPIC", "-fno-fast-math", "-ffp-contract=off", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_d = ctypes.c_double
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_i = ctypes.c_int
_p = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_philox4x32_10.argtypes = [_p, _p, _p]
        L.orc_philox4x32_10.restype = None
        L.orc_uniform.argtypes = [_u32]
        L.orc_uniform.restype = _d
        L.orc_pick.argtypes = [_u32, _u32]
        L.orc_pick.restype = _u32
        L.orc_move_draw.argtypes = [_u64, _u32, _u32, _u32, _u32, _u32, _p, _p, _p]
        L.orc_move_draw.restype = None
        L.orc_init_point.argtypes = [_u64, _u32, _u32, _u32, _p, _p, _p]
        L.orc_init_point.restype = None
        L.orc_schwefel_term.argtypes = [_d]
        L.orc_schwefel_term.restype = _d
        L.orc_rastrigin_term.argtypes = [_d]
        L.orc_rastrigin_term.restype = _d
        L.orc_ackley_from_sums.argtypes = [_d, _d, _u32]
        L.orc_ackley_from_sums.restype = _d
        L.orc_f.argtypes = [_i, _u32, _p, _p]
        L.orc_f.restype = _d
        L.orc_centres.argtypes = [_i, _p, _p]
        L.orc_centres.restype = _u32
        L.orc_accept.argtypes = [_d, _d, _d]
        L.orc_accept.restype = _i
        L.orc_neighbour.argtypes = [_i, _d, _d, _d, _d, _d]
        L.orc_neighbour.restype = _d
        L.orc_temperature.argtypes = [_d, _d, _u32]
        L.orc_temperature.restype = _d
        L.orc_sa_run.argtypes = [_i, _u32, _p, _p, _p, _u64, _u32, _u32, _u32, _d, _d, _d, _i, _u32, _u32, _u32,
                                 _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p]
        L.orc_sa_run.restype = _i
        L.orc_sa_run_v.argtypes = [_i, _u32, _p, _p, _p, _u64, _u32, _u32, _u32, _d, _d, _d, _i, _u32, _u32, _u32,
                                    _u32, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p]
        L.orc_sa_run_v.restype = _i
        L.orc_sos_uniform.argtypes = [_u64, _u32, _u32, _u32]
        L.orc_sos_uniform.restype = _d
        L.orc_set_net_kind.argtypes = [_i]
        L.orc_set_net_kind.restype = None
        L.orc_replay_level.argtypes = [_i, _u32, _p, _p, _p, _u64, _u32, _u32, _d, _d, _i, _u32, _p, _u32, _u32,
                                       _p, _p, _p, _p, _p, _p, _p]
        L.orc_replay_level.restype = _i
        L.orc_mlp_nparam.argtypes = []
        L.orc_mlp_nparam.restype = _u32
        L.orc_act.argtypes = [_d]
        L.orc_act.restype = _d
        L.orc_act_grad.argtypes = [_d]
        L.orc_act_grad.restype = _d
        L.orc_mlp_forward.argtypes = [_p, _p, _p, _p, _p]
        L.orc_mlp_forward.restype = None
        L.orc_mlp_loss_grad.argtypes = [_p, _u32, _p, _p, _p]
        L.orc_mlp_loss_grad.restype = _d
        L.orc_adam_step.argtypes = [_p, _p, _p, _p, _u32, _u32, _d, _d, _d, _d]
        L.orc_adam_step.restype = None
        L.orc_proposal_logpdf.argtypes = [_d, _d, _d]
        L.orc_proposal_logpdf.restype = _d
        L.orc_hist_feature.argtypes = [_d]
        L.orc_hist_feature.restype = _d
        L.orc_mlp_forward_bound.argtypes = [_p, _p, _p, _p]
        L.orc_mlp_forward_bound.restype = None
        L.orc_learn_draw.argtypes = [_u64, _u32, _u32, _u32, _u32]
        L.orc_learn_draw.restype = _d
        L.orc_learn_mix.argtypes = [_u64, _u32, _u32, _u32, _u32]
        L.orc_learn_mix.restype = _d
        L.orc_sa_run_capture.argtypes = [_i, _u32, _p, _p, _p, _u64, _u32, _u32, _u32, _d, _d, _d, _i, _u32, _u32,
                                         _p, _d, _p, ctypes.c_uint64, _p]
        L.orc_sa_run_capture.restype = _i
        L.orc_nelder_mead.argtypes = [_i, _u32, _p, _p, _p, _p, _u32, _d, _d, _p, _p, _p, _p, _p, _p]
        L.orc_nelder_mead.restype = _i
        L.orc_set_threads.argtypes = [_i]
        L.orc_set_threads.restype = None
        L.orc_mlp_forward_device.argtypes = [_p, _p, _p, _p, _p]
        L.orc_mlp_forward_device.restype = None
        L.orc_learned_propose.argtypes = [_p, _i, _u64, _u32, _u32, _u32, _u32, _u32, _p, _p, _p, _d, _d, _d, _p,
                                          _p, _p]
        L.orc_learned_propose.restype = None
        L.orc_learned_accept.argtypes = [_p, _i, _i, _u32, _p, _p, _p, _u64, _u32, _u32, _u32, _u32, _d, _d, _i, _p,
                                         _u32, _d, _d, _d, _p, _p]
        L.orc_learned_accept.restype = _i
        L.orc_learned_run.argtypes = [_p, _i, _i, _u32, _p, _p, _p, _u64, _u32, _u32, _u32, _u32, _u32, _d, _d, _d,
                                      _d, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p]
        L.orc_learned_run.restype = _i
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(r: int) -> float:
    return lib().orc_uniform(r)


def pick(r: int, n: int) -> int:
    return lib().orc_pick(r, n)


def move_draw(seed, problem, level, chain, step, n):
    """(coordinate, change uniform, acceptance uniform) of move `step`: words
    3 step .. 3 step + 2 of the chain's move stream at `level`."""
    d = ctypes.c_uint32()
    u1 = ctypes.c_double()
    u2 = ctypes.c_double()
    lib().orc_move_draw(seed, problem, level, chain, step, n, ctypes.byref(d), ctypes.byref(u1), ctypes.byref(u2))
    return d.value, u1.value, u2.value


def init_point(seed, problem, chain, lower, upper):
    lo, hi = _f64(lower), _f64(upper)
    x = np.zeros(lo.size)
    lib().orc_init_point(seed, problem, chain, lo.size, _ptr(lo), _ptr(hi), _ptr(x))
    return x


def f(func, x, shift=None):
    x = _f64(x)
    s = _f64(shift)
    return lib().orc_f(func, x.size, _ptr(x), _ptr(s))


def centres(func):
    """(a [m, 10], c [m]) of a centre family's table (Shekel's last six
    coordinates zero); None for another function."""
    a = np.zeros((30, 10))
    c = np.zeros(30)
    m = lib().orc_centres(func, _ptr(a), _ptr(c))
    return (a[:m], c[:m]) if m else None


def schwefel_term(y):
    return lib().orc_schwefel_term(y)


def rastrigin_term(y):
    return lib().orc_rastrigin_term(y)


def ackley_from_sums(s1, s2, n):
    return lib().orc_ackley_from_sums(s1, s2, n)


def accept(df, T, u2) -> bool:
    return bool(lib().orc_accept(df, T, u2))


def neighbour(move_rule, xd, lo, hi, radius_frac, u1):
    return lib().orc_neighbour(move_rule, xd, lo, hi, radius_frac, u1)


def temperature(T0, alpha, level):
    return lib().orc_temperature(T0, alpha, level)


def set_threads(threads: int):
    """Threads the oracle's multi-chain runs use for the chains of a level
    (results are identical for every count)."""
    lib().orc_set_threads(int(threads))


VARIANT_SOS, VARIANT_BEST_SEEN, VARIANT_ELITIST, VARIANT_FULL = 1, 2, 4, 8


def sos_uniform(seed, problem, level, chain) -> float:
    """Uniform of the stochastic exchange decision of `chain` at `level`."""
    return lib().orc_sos_uniform(seed, problem, level, chain)


def sa_run(func, lower, upper, shift=None, *, seed, chains, steps, T0, alpha, levels, radius_frac=0.1,
           move_rule=MOVE_RADIUS, exchange=True, problem=0, level_begin=0, x_start=None, chain_x=None,
           chain_cost=None, record=None, keep_x_best=True, final_f=False, sos=False, best_seen=False,
           f_win_prev=None, kept=False, elitist=False, full_eval=False):
    """Run levels [level_begin, level_begin+levels) of the multi-chain SA.

    ``exchange``: levels between broadcasts of the winner -- 1 or True: every
    level (synchronous); k > 1: every k-th level (periodic); 0 or False:
    never (asynchronous).  Without a broadcast a chain continues from its own
    state and carried cost (``chain_x`` [chains, n] and ``chain_cost``
    [chains, 3] = f, s1, s2, carried in from an earlier call and returned).
    ``record`` = (x_rec, f_rec, rec_level) carried in from an earlier call.
    ``sos``: stochastic exchange at the levels that start with one (each
    chain keeps its own state with probability exp(-(f_own - f_win)/T_prev));
    ``best_seen``: each chain's best-seen state of a level stands in for its
    final state in the argmin, broadcast and record.  ``f_win_prev``: the
    winner cost of level level_begin - 1 (sos runs that start past level 0).
    ``kept``: also return, for the last level, which chains kept their state.
    ``elitist``: an exchange broadcasts the record instead of the last
    level's winner (with ``x_start`` the record's state when resuming).
    ``full_eval``: every move's cost is f evaluated in full at the moved
    state instead of the separable families' increment.
    Returns a dict of per-level outputs and the record."""
    lo, hi, s = _f64(lower), _f64(upper), _f64(shift)
    n = lo.size
    period = 1 if exchange is True else 0 if exchange is False else int(exchange)
    variant = ((VARIANT_SOS if sos else 0) | (VARIANT_BEST_SEEN if best_seen else 0)
               | (VARIANT_ELITIST if elitist else 0) | (VARIANT_FULL if full_eval else 0))
    xs = np.zeros(n) if x_start is None else _f64(x_start).copy()
    cx = cc = None
    if period != 1 or sos:
        cx = np.zeros(chains * n) if chain_x is None else _f64(chain_x).copy().reshape(-1)
        cc = np.zeros(chains * 3) if chain_cost is None else _f64(chain_cost).copy().reshape(-1)
    if record is None:
        x_rec = np.zeros(n)
        f_rec_io = ctypes.c_double(np.inf)
        rec_level = ctypes.c_uint32(0)
    else:
        x_rec = _f64(record[0]).copy()
        f_rec_io = ctypes.c_double(record[1])
        rec_level = ctypes.c_uint32(record[2])
    win = np.zeros(levels, dtype=np.uint32)
    f_win = np.zeros(levels)
    f_best = np.zeros(levels)
    f_rec = np.zeros(levels)
    xb = np.zeros(levels * n) if keep_x_best else None
    acc = np.zeros(levels, dtype=np.uint64)
    ff = np.zeros(chains) if final_f else None
    fw = ctypes.c_double(0.0 if f_win_prev is None else f_win_prev)
    kp = np.zeros(chains, dtype=np.uint8) if kept else None
    rc = lib().orc_sa_run_v(func, n, _ptr(lo), _ptr(hi), _ptr(s), seed, problem, chains, steps, T0, alpha,
                            radius_frac, move_rule, period, variant, level_begin, levels, _ptr(xs), _ptr(cx),
                            _ptr(cc), ctypes.byref(fw), _ptr(x_rec), ctypes.byref(f_rec_io), ctypes.byref(rec_level),
                            _ptr(win), _ptr(f_win), _ptr(f_best), _ptr(f_rec), _ptr(xb), _ptr(acc), _ptr(ff),
                            _ptr(kp))
    if rc != 0:
        raise RuntimeError(f"orc_sa_run failed: {rc}")
    out = dict(win_chain=win, f_win=f_win, f_best=f_best, f_rec=f_rec, accepts=acc, x_last=xs,
               x_rec=x_rec, f_rec_final=f_rec_io.value, rec_level=rec_level.value)
    if keep_x_best:
        out["x_best"] = xb.reshape(levels, n)
    if final_f:
        out["final_f"] = ff
    if period != 1 or sos:
        out["chain_x"] = cx.reshape(chains, n)
        out["chain_cost"] = cc.reshape(chains, 3)
    out["f_win_last"] = fw.value
    if kept:
        out["kept"] = kp.astype(bool)
    return out


def replay_level(func, lower, upper, shift=None, *, seed, steps, T, level, x_start, chain0, nchains,
                 radius_frac=0.1, move_rule=MOVE_RADIUS, problem=0):
    """Replay one level for a range of chains from a given start, logging moves."""
    lo, hi, s = _f64(lower), _f64(upper), _f64(shift)
    n = lo.size
    xs = _f64(x_start)
    m = nchains * steps
    log_d = np.zeros(m, dtype=np.uint32)
    log_xold = np.zeros(m)
    log_xnew = np.zeros(m)
    log_df = np.zeros(m)
    log_acc = np.zeros(m, dtype=np.uint8)
    x_final = np.zeros(nchains * n)
    f_final = np.zeros(nchains)
    rc = lib().orc_replay_level(func, n, _ptr(lo), _ptr(hi), _ptr(s), seed, problem, steps, T, radius_frac,
                                move_rule, level, _ptr(xs), chain0, nchains, _ptr(log_d), _ptr(log_xold),
                                _ptr(log_xnew), _ptr(log_df), _ptr(log_acc), _ptr(x_final), _ptr(f_final))
    if rc != 0:
        raise RuntimeError(f"orc_replay_level failed: {rc}")
    sh = (nchains, steps)
    return dict(d=log_d.reshape(sh), x_old=log_xold.reshape(sh), x_new=log_xnew.reshape(sh),
                df=log_df.reshape(sh), acc=log_acc.reshape(sh).astype(bool), x_final=x_final.reshape(nchains, n),
                f_final=f_final)


# ---------------------------------------------------------------------------
# Learned proposal network (FP64 reference)
# ---------------------------------------------------------------------------
MLP_HIDDEN = 128
MLP_INPUTS = 6
# Network kinds: relu + Cauchy output + log-magnitude history features, or the
# written configuration (GELU + Gaussian output + raw history features).
NET_RELU_CAUCHY, NET_GELU_GAUSS = 0, 1


def set_net_kind(kind: int):
    """Kind of the proposal network every network function below uses."""
    lib().orc_set_net_kind(int(kind))


def mlp_nparam() -> int:
    return lib().orc_mlp_nparam()


def act(a: float) -> float:
    return lib().orc_act(a)


def act_grad(a: float) -> float:
    return lib().orc_act_grad(a)


def mlp_forward(params, z):
    """(mu, s) for one feature vector; also the two pre-activation vectors."""
    p = _f64(params)
    zz = _f64(z)
    out = np.zeros(2)
    a1 = np.zeros(MLP_HIDDEN)
    a2 = np.zeros(MLP_HIDDEN)
    lib().orc_mlp_forward(_ptr(p), _ptr(zz), _ptr(out), _ptr(a1), _ptr(a2))
    return out, a1, a2


def mlp_loss_grad(params, Z, delta, with_grad=True):
    p = _f64(params)
    Zc = _f64(Z).reshape(-1, MLP_INPUTS)
    d = _f64(delta)
    g = np.zeros(p.size) if with_grad else None
    loss = lib().orc_mlp_loss_grad(_ptr(p), Zc.shape[0], _ptr(Zc), _ptr(d), _ptr(g))
    return (loss, g) if with_grad else loss


def adam_step(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.size, t, lr, beta1, beta2, eps)


def proposal_logpdf(delta, mu, s):
    return lib().orc_proposal_logpdf(delta, mu, s)


def mlp_unpack(params):
    """Split the parameter vector into (W1, b1, W2, b2, W3, b3)."""
    p = _f64(params)
    H, I = MLP_HIDDEN, MLP_INPUTS
    sizes = [I * H, H, H * H, H, H * 2, 2]
    shapes = [(I, H), (H,), (H, H), (H,), (H, 2), (2,)]
    out, o = [], 0
    for sz, sh in zip(sizes, shapes):
        out.append(p[o:o + sz].reshape(sh))
        o += sz
    return out


def mlp_forward_bound(params, z):
    """(mu, s) and the per-output error bound of a BF16-activation evaluation."""
    p = _f64(params)
    zz = _f64(z)
    out = np.zeros(2)
    bound = np.zeros(2)
    lib().orc_mlp_forward_bound(_ptr(p), _ptr(zz), _ptr(out), _ptr(bound))
    return out, bound


def hist_feature(h: float) -> float:
    """History feature of a scaled displacement: sign(h) ln(1 + 2^24 |h|) / 16."""
    return lib().orc_hist_feature(h)


def learn_draw(seed, problem, level, chain, step) -> float:
    """Standard Cauchy draw of a learned move (inversion, Philox tag 3)."""
    return lib().orc_learn_draw(seed, problem, level, chain, step)


def learn_mix(seed, problem, level, chain, step) -> float:
    """Uniform that chooses the mixture component of a learned-mode move (the
    plain move iff it is below eps): second word of the learned block."""
    return lib().orc_learn_mix(seed, problem, level, chain, step)


def feature_tau(func, n):
    """Scale of the temperature feature ln(tau T): n for the objectives
    normalised by n (Schwefel, Ackley), 1 for Rastrigin."""
    return 1.0 if func == RASTRIGIN else float(n)


def sa_run_capture(func, lower, upper, shift=None, *, seed, chains, steps, T0, alpha, levels, level_begin=0,
                   x_start=None, radius_frac=0.1, move_rule=MOVE_RADIUS, problem=0, capacity=1 << 20, tau=None):
    """Synchronous run over levels [level_begin, level_begin+levels) that
    records every accepted move, with the temperature feature ln(tau T)
    (tau = feature_tau(func, n) unless given; 1 for the Gaussian network
    kind's ln T) and the history features of the network kind in force;
    returns (records float32 [k, 7], count)."""
    lo, hi, s = _f64(lower), _f64(upper), _f64(shift)
    n = lo.size
    xs = np.zeros(n) if x_start is None else _f64(x_start).copy()
    rec = np.zeros((capacity, 7), dtype=np.float32)
    cnt = ctypes.c_uint64()
    rc = lib().orc_sa_run_capture(func, n, _ptr(lo), _ptr(hi), _ptr(s), seed, problem, chains, steps, T0, alpha,
                                  radius_frac, move_rule, level_begin, levels, _ptr(xs),
                                  feature_tau(func, n) if tau is None else float(tau),
                                  _ptr(rec), capacity, ctypes.byref(cnt))
    if rc != 0:
        raise RuntimeError(f"orc_sa_run_capture failed: {rc}")
    return rec[:min(cnt.value, capacity)], cnt.value


# ---------------------------------------------------------------------------
# Learned-proposal mixture move (oracle side; an extension of the method)
# ---------------------------------------------------------------------------
NET_FP64, NET_DEVICE = 0, 1


def mlp_forward_device(params, z, ez=None):
    """(mu, s) of the network under the device's stated precision (BF16 weight
    matrices -- already rounded in params --, BF16 hidden activations, features
    as BF16 high part plus remainder, FP32 accumulation) carried out in FP64,
    and a bound on the deviation of any FP32 accumulation order (plus feature
    errors ez)."""
    p = _f64(params)
    zz = _f64(z)
    e = None if ez is None else _f64(ez)
    out = np.zeros(2)
    bound = np.zeros(2)
    lib().orc_mlp_forward_device(_ptr(p), _ptr(zz), _ptr(e), _ptr(out), _ptr(bound))
    return out, bound


def learned_propose(params, mode, *, seed, problem=0, level, chain, step, x, lower, upper, radius_frac=0.1, featT,
                    eps, hist):
    """Proposal of one learned-mixture move from state x with history hist (the
    chain's last four accepted scaled displacements, most recent first)."""
    p, xx, lo, hi = _f64(params), _f64(x), _f64(lower), _f64(upper)
    h = _f64(hist)
    ou = np.zeros(2, dtype=np.uint32)
    od = np.zeros(7)
    lib().orc_learned_propose(_ptr(p), mode, seed, problem, level, chain, step, xx.size, _ptr(xx), _ptr(lo), _ptr(hi),
                              radius_frac, featT, eps, _ptr(h), _ptr(ou), _ptr(od))
    return dict(d=int(ou[0]), plain=bool(ou[1]), x_old=od[0], x_new=od[1], mu=od[2], s=od[3], t=od[4], b_mu=od[5],
                b_s=od[6])


def learned_accept(params, mode, func, *, lower, upper, shift=None, seed, problem=0, level, chain, step, T, featT,
                   plain, x, d, x_new, mu, s, hist):
    """Metropolis-Hastings decision on the proposal x_new for coordinate d of
    the state x (network at x: mu, s).  Returns (taken, details)."""
    p, xx, lo, hi, sh = _f64(params), _f64(x), _f64(lower), _f64(upper), _f64(shift)
    h = _f64(hist)
    out = np.zeros(8)
    take = lib().orc_learned_accept(_ptr(p), mode, func, xx.size, _ptr(lo), _ptr(hi), _ptr(sh), seed, problem, level,
                                    chain, step, T, featT, int(plain), _ptr(xx), d, x_new, mu, s, _ptr(h), _ptr(out))
    return bool(take), dict(df=out[0], lq=out[1], log_ratio=out[2], u2=out[3], mu2=out[4], s2=out[5], b_mu2=out[6],
                            b_s2=out[7])


def learned_run(params, mode, func, lower, upper, shift=None, *, seed, problem=0, level, chain0=0, nchains, steps,
                T, featT, eps, radius_frac=0.1, x_start, log=False, trace0=False):
    """One learned-mixture level for chains [chain0, chain0 + nchains) from
    x_start (empty history), in the oracle.  Returns a dict with final states,
    costs, accepted counts, and optionally the per-move log and x[0] path."""
    p, lo, hi, sh, xs = _f64(params), _f64(lower), _f64(upper), _f64(shift), _f64(x_start)
    n = lo.size
    m = nchains * steps
    out = dict(x_final=np.zeros((nchains, n)), f_final=np.zeros(nchains), accepts=np.zeros(nchains, dtype=np.uint64))
    if log:
        out.update(d=np.zeros(m, dtype=np.uint32), plain=np.zeros(m, dtype=np.uint8), x_old=np.zeros(m),
                   x_new=np.zeros(m), df=np.zeros(m), accept=np.zeros(m, dtype=np.uint8))
    if trace0:
        out["trace0"] = np.zeros(m)
    g = out.get
    rc = lib().orc_learned_run(_ptr(p), mode, func, n, _ptr(lo), _ptr(hi), _ptr(sh), seed, problem, level, chain0,
                               nchains, steps, T, featT, eps, radius_frac, _ptr(xs), _ptr(g("d")), _ptr(g("plain")),
                               _ptr(g("x_old")), _ptr(g("x_new")), _ptr(g("df")), _ptr(g("accept")),
                               _ptr(out["x_final"]), _ptr(out["f_final"]), _ptr(out["accepts"]), _ptr(g("trace0")))
    if rc != 0:
        raise RuntimeError(f"orc_learned_run failed: {rc}")
    return out


# ---------------------------------------------------------------------------
# Nelder-Mead polish (the paper's hybrid strategy)
# ---------------------------------------------------------------------------
NM_REFLECT, NM_EXPAND, NM_OUTSIDE, NM_INSIDE, NM_SHRINK = 0, 1, 2, 3, 4


def nelder_mead(func, lower, upper, shift=None, *, x0, maxiter=10000, ftol=1e-12, xtol=1e-10):
    """Box-projected Nelder-Mead from x0; returns dict(x, f, iters, evals, steps,
    gaps): steps[i] is iteration i's step code, gaps[i] = f_w - f_b at its start."""
    lo, hi, s, x = _f64(lower), _f64(upper), _f64(shift), _f64(x0)
    n = lo.size
    xo = np.zeros(n)
    f = ctypes.c_double()
    it = ctypes.c_uint32()
    ev = ctypes.c_uint32()
    log = np.zeros(maxiter, dtype=np.uint8)
    gaps = np.zeros(maxiter)
    rc = lib().orc_nelder_mead(func, n, _ptr(lo), _ptr(hi), _ptr(s), _ptr(x), maxiter, ftol, xtol, _ptr(xo),
                               ctypes.byref(f), ctypes.byref(it), ctypes.byref(ev), _ptr(log), _ptr(gaps))
    if rc != 0:
        raise RuntimeError(f"orc_nelder_mead failed: {rc}")
    return dict(x=xo, f=f.value, iters=it.value, evals=ev.value, steps=log[:it.value].copy(),
                gaps=gaps[:it.value].copy())
