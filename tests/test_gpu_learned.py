"""GPU parity of the learned proposal against the FP64 oracle.

- In-kernel network inference (the BF16-MFMA wave routine the annealing
  kernels run) against the oracle's forward pass: every output within the
  oracle's first-order bound for BF16 activations, and close to a numpy model
  of the documented rounding.
- Capture of accepted moves: FP64 runs give exactly the oracle's records (as
  a multiset; slots are reserved in device order); FP32 runs keep count and
  feature invariants, and stop storing at capacity.
- Start states: an FP64 run started at level k from x equals the oracle's
  run over the same levels from the same broadcast state.
- Learned-mixture levels: every logged move replayed against the oracle
  (coordinate and plain/learned choice bit-exact, proposal within the network
  bound, Metropolis-Hastings decision equal where the bounds cannot flip it),
  level winners and records as in the plain path, and graph replay equal to
  eager launches.  The decisions come from the oracle's learned move
  (oracle.learned_propose / learned_accept), not from the checker.
- The network the time-to-target comparison trains (learned.collect and
  learned.train on the device), replayed the same way at the benchmark shape.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_util import (bf16_matrices, box32, check_learned_level, check_record, f32, fp32_init_state,
                         learned_params, lexi_argmin)

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


def bf16_round64(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def emulated_forward(p64, Z):
    """numpy model of the device arithmetic: BF16 weight matrices (already in
    p64), hidden activations rounded to BF16, everything else in float64."""
    W1, b1, W2, b2, W3, b3 = O.mlp_unpack(p64)
    h1 = bf16_round64(np.maximum(Z @ W1 + b1, 0.0))
    h2 = bf16_round64(np.maximum(h1 @ W2 + b2, 0.0))
    return h2 @ W3 + b3


def feature_rows(rng, rows):
    return np.column_stack([rng.uniform(0, 1, rows), rng.uniform(-6, 8, rows),
                            rng.normal(0, 0.05, (rows, 4))]).astype(np.float32)


@pytest.mark.parametrize("rows,scale", [(1000, 0.1), (64, 0.3), (4099, 0.05)])
def test_infer_matches_oracle(S, rows, scale):
    import torch
    rng = np.random.default_rng(rows)
    p = learned_params(rows, scale=scale)
    Z = feature_rows(rng, rows)
    say(f"[gpu learned] infer rows={rows} scale={scale}")
    tr = S.MLPTrainer(max_batch=64)
    tr.set_params(p)
    out = tr.infer(torch.from_numpy(Z).cuda()).cpu().numpy().astype(np.float64)
    tr.close()
    q = bf16_matrices(p)
    Z64 = Z.astype(np.float64)
    worst = 0.0
    for r in range(rows):
        o, b = O.mlp_forward_bound(q, Z64[r])
        e = np.abs(out[r] - o)
        worst = max(worst, float(np.max(e / b)))
        assert np.all(e <= b), (r, out[r], o, b)
    emu = emulated_forward(q, Z64)
    dev = np.abs(out - emu)
    say(f"[gpu learned] infer worst err/bound {worst:.3f}, max |gpu - bf16 model| {dev.max():.3e}")
    # the model differs only where an FP32 pre-activation crosses a BF16
    # rounding boundary differently from float64: one BF16 ulp of one unit
    assert np.all(dev <= 2e-3 * (1.0 + np.abs(emu)))


def capture_run(S, wl, chains, levels, steps, T0, alpha, seed, capacity, precision):
    import torch
    sched = S.Schedule(chains=chains, levels=levels, steps=steps, T0=T0, alpha=alpha, seed=seed, precision=precision,
                       trace_x=True)
    rec = torch.zeros((capacity, 7), dtype=torch.float32, device="cuda")
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
        ann.capture(rec)
        ann.run()
        count = ann.capture_count()
        trace = ann.trace()
    return rec.cpu().numpy(), count, trace


def sort_rows(a):
    return a[np.lexsort(a.T[::-1])]


@pytest.mark.parametrize("case", ["schwefel_n4", "rastrigin_n7_table", "ackley_n5"])
def test_capture_fp64_equals_oracle(S, case):
    rng = np.random.default_rng(3)
    if case == "schwefel_n4":
        wl = W.schwefel_n4_fp64()
    elif case == "rastrigin_n7_table":
        lo, hi = W.uneven_box(7, 3)
        wl = W.Workload(case, W.RASTRIGIN, 7, lo, hi, W.inner_shift(lo, hi, rng), chains=0, levels=0, steps=0,
                        T0=0, alpha=0, seed=0, precision=W.FP64)
    else:
        wl = W.Workload(case, W.ACKLEY, 5, np.full(5, -32.768), np.full(5, 32.768), None, chains=0, levels=0,
                        steps=0, T0=0, alpha=0, seed=0, precision=W.FP64)
    kw = dict(chains=192, levels=4, steps=24, T0=5.0, alpha=0.8, seed=11)
    say(f"[gpu learned] capture fp64 {case}")
    got, count, trace = capture_run(S, wl, capacity=1 << 16, precision=S.FP64, **kw)
    ref, rcount = O.sa_run_capture(wl.func, wl.lower, wl.upper, wl.shift, capacity=1 << 16, **kw)
    assert count == rcount == int(trace["accepts"].sum())
    assert np.array_equal(sort_rows(got[:count]), sort_rows(ref))
    assert not np.any(got[count:])


def test_capture_fp32_invariants_and_capacity(S):
    wl = W.schwefel_n100_fp32()
    kw = dict(chains=1024, levels=5, steps=50, T0=10.0, alpha=0.9, seed=4)
    say("[gpu learned] capture fp32 schwefel n=100")
    got, count, trace = capture_run(S, wl, capacity=1 << 18, precision=S.FP32, **kw)
    assert count == int(trace["accepts"].sum()) and count < (1 << 18)
    r = got[:count]
    assert np.all(r[:, 0] >= 0) and np.all(r[:, 0] <= 1)
    featT = {np.float32(math.log(wl.n * O.temperature(kw["T0"], kw["alpha"], k))) for k in range(kw["levels"])}
    assert set(np.unique(r[:, 1])) <= featT
    assert np.all(np.abs(r[:, 6]) <= 0.1 * (1 + 1e-6))  # radius 0.1 (u - l)
    assert np.all(np.abs(r[:, 2:6]) <= math.log1p(2.0 ** 24 * 0.1) / 16 * (1 + 1e-6))
    # a zero displacement is a radius move clamped back onto the box edge it started on
    assert np.all((r[:, 6] != 0) | (r[:, 0] == 0) | (r[:, 0] == 1))
    # a smaller buffer: every slot written, the count still complete
    small = 1000
    got2, count2, _ = capture_run(S, wl, capacity=small, precision=S.FP32, **kw)
    assert count2 == count
    assert np.all(np.isin(got2[:, 1], list(featT)))


def test_set_start_fp64_matches_oracle(S):
    wl = W.schwefel_n4_fp64()
    rng = np.random.default_rng(9)
    x0 = np.clip(W.SCHWEFEL_X_STAR + rng.uniform(-50, 50, wl.n), -500, 500)
    sched = S.Schedule(chains=256, levels=12, steps=30, T0=10.0, alpha=0.9, seed=5, precision=S.FP64, trace_x=True)
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
        ann.set_start(7, x0)
        assert ann.levels_done() == 7
        ann.run()
        rec, xb = ann.trace(7, 5, with_x=True)
        x_rec, f_rec, lvl = ann.best()
        with pytest.raises(S.SAError):
            ann.trace(0, 1)
    o = O.sa_run(wl.func, wl.lower, wl.upper, wl.shift, seed=5, chains=256, steps=30, T0=10.0, alpha=0.9, levels=5,
                 level_begin=7, x_start=x0)
    assert np.array_equal(rec["win_chain"], o["win_chain"])
    assert np.array_equal(rec["accepts"], o["accepts"])
    np.testing.assert_allclose(rec["f_best"], o["f_best"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(xb, o["x_best"], rtol=1e-12, atol=1e-12)
    assert lvl == o["rec_level"] and abs(f_rec - o["f_rec_final"]) <= 1e-12


def learned_case(name):
    rng = np.random.default_rng(17)
    if name == "schwefel_n16":
        return W.Workload(name, W.SCHWEFEL, 16, np.full(16, -500.0), np.full(16, 500.0), None, chains=0, levels=0,
                          steps=0, T0=0, alpha=0, seed=0, precision=W.FP32)
    if name == "rastrigin_n9_table":
        lo, hi = W.uneven_box(9, 4)
        return W.Workload(name, W.RASTRIGIN, 9, lo, hi, W.inner_shift(lo, hi, rng), chains=0, levels=0, steps=0,
                          T0=0, alpha=0, seed=0, precision=W.FP32)
    return W.Workload(name, W.ACKLEY, 12, np.full(12, -32.768), np.full(12, 32.768), None, chains=0, levels=0,
                      steps=0, T0=0, alpha=0, seed=0, precision=W.FP32)


def run_learned(S, wl, params, eps, *, chains, levels, steps, T0, alpha, seed, log_chains=0, graph=False,
                chunks=None):
    sched = S.Schedule(chains=chains, levels=levels, steps=steps, T0=T0, alpha=alpha, seed=seed, precision=S.FP32,
                       trace_x=True, learned=True, graph=graph, log_chains=log_chains, log_level=0,
                       log_levels=levels if log_chains else 0)
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
        ann.set_proposal(params, eps)
        for c in (chunks or [0]):
            ann.run(c)
        rec, xb = ann.trace(with_x=True)
        x_rec, f_rec, lvl = ann.best()
        out = dict(rec=rec, xb=xb, x_rec=x_rec, f_rec=f_rec, rec_level=lvl)
        if log_chains:
            out["moves"], out["final_f"] = ann.move_log()
    return out


@pytest.mark.parametrize("name,steps", [("schwefel_n16", 32), ("rastrigin_n9_table", 32), ("ackley_n12", 32),
                                        ("schwefel_n16", 31)])
def test_learned_per_move_parity(S, name, steps):
    wl = learned_case(name)
    kw = dict(chains=512, levels=3, steps=steps, T0=5.0 if wl.func != W.SCHWEFEL else 20.0, alpha=0.7, seed=23)
    eps = 0.25
    # random weights at the scale of a trained network's hidden layers; the
    # oracle's device-precision network bound decides which
    # Metropolis-Hastings decisions are checkable
    p = learned_params(31, scale=0.05, sigma0=0.1)
    say(f"[gpu learned] per-move {name}")
    g = run_learned(S, wl, p, eps, log_chains=64, **kw)
    lo32, hi32 = box32(wl.lower, wl.upper)
    sh32 = None if wl.shift is None else f32(wl.shift)
    q = bf16_matrices(p)
    tau = O.feature_tau(wl.func, wl.n)
    totals = dict(moves=0, learned=0, outside=0, ambiguous=0, max_dl_excess=0.0, max_rel_excess=0.0)
    wl_run = wl.with_(chains=kw["chains"], seed=kw["seed"])
    for level in range(kw["levels"]):
        T = O.temperature(kw["T0"], kw["alpha"], level)
        featT = float(np.float32(math.log(tau * T)))
        fin = g["final_f"][level]
        win = lexi_argmin(fin)
        assert g["rec"]["win_chain"][level] == win and g["rec"]["f_win"][level] == fin[win]
        fb = O.f(wl.func, g["xb"][level], sh32)
        assert abs(g["rec"]["f_best"][level] - fb) <= 1e-11 * max(1.0, abs(fb))
        for c in range(0, 64, 3):
            x0 = fp32_init_state(wl_run, c) if level == 0 else g["xb"][level - 1]
            st = check_learned_level(wl.func, wl.n, lo32, hi32, sh32, kw["seed"], level, T, featT,
                                     float(np.float32(eps)), q, 0.1, x0, g["moves"][level, c:c + 1], fin, [c])
            for k in totals:
                totals[k] = max(totals[k], st[k]) if k.startswith("max") else totals[k] + st[k]
    say(f"[gpu learned] {name}: {totals}")
    assert totals["learned"] > 0.5 * totals["moves"]
    assert totals["ambiguous"] <= 0.05 * totals["moves"]
    check_record(wl_run.with_(levels=kw["levels"]), g)


def test_learned_graph_and_chunks_equal_eager(S):
    wl = learned_case("schwefel_n16")
    p = learned_params(5, scale=0.05, sigma0=0.02)
    kw = dict(chains=1024, levels=6, steps=20, T0=10.0, alpha=0.8, seed=2)
    a = run_learned(S, wl, p, 0.1, **kw)
    b = run_learned(S, wl, p, 0.1, graph=True, chunks=[2, 4], **kw)
    cols = ["win_chain", "accepts", "f_win", "f_best", "f_rec"]
    assert np.array_equal(a["rec"][cols], b["rec"][cols])
    assert np.array_equal(a["xb"], b["xb"])


def test_learned_from_a_later_level(S):
    """The learned mixture switched on after k plain levels (the late arm of
    the time-to-target comparison): levels before k equal a plain run's bit
    for bit, later levels use the network (they differ from the plain run's)
    and equal a run that switches at the same level through learned.time_to_target's
    sequence of calls (plain run(k), set_proposal, run)."""
    from paper_2408_00018_amd import learned as Lp
    wl = learned_case("schwefel_n16")
    p = learned_params(5, scale=0.05, sigma0=0.02)
    kw = dict(chains=1024, levels=8, steps=20, T0=10.0, alpha=0.8, seed=2)
    k = 5
    cols = ["win_chain", "accepts", "f_win", "f_best", "f_rec"]

    def run(learned, switch):
        sched = S.Schedule(precision=S.FP32, trace_x=True, learned=learned, **kw)
        with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
            if switch is not None:
                ann.run(switch)
                ann.set_proposal(p, 0.1)
            ann.run(0)
            return ann.trace(with_x=True)

    plain, plain_x = run(False, None)
    late, late_x = run(True, k)
    assert np.array_equal(late[cols][:k], plain[cols][:k])
    assert np.array_equal(late_x[:k], plain_x[:k])
    assert not np.array_equal(late_x[k:], plain_x[k:])
    again, again_x = run(True, k)
    assert np.array_equal(again[cols], late[cols]) and np.array_equal(again_x, late_x)
    sched = S.Schedule(precision=S.FP32, **kw)
    r = Lp.time_to_target(wl.func, wl.lower, wl.upper, wl.shift, sched, W.SCHWEFEL_F_STAR, 1e9, params=p, eps=0.1,
                          learn_from=k, chunk=3)
    assert r.hit and r.level == 0 and r.levels_run == 3  # a target every level meets: the first chunk ends it


def test_learned_rejects_unsupported(S):
    wl = W.schwefel_n4_fp64()
    sched = S.Schedule(chains=64, levels=2, steps=4, T0=1.0, alpha=0.9, precision=S.FP64, learned=True)
    with pytest.raises(S.SAError) as e:
        S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched)
    assert e.value.status == -5
    sched = S.Schedule(chains=64, levels=2, steps=4, T0=1.0, alpha=0.9, precision=S.FP32)
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
        with pytest.raises(S.SAError) as e:
            ann.set_proposal(learned_params(1), 0.1)
        assert e.value.status == -4


def test_trained_network_replay_at_the_bench_shape(S):
    """The network as the time-to-target comparison uses it -- trained by
    learned.collect / learned.train on the device -- replayed move by move
    against the oracle's learned move at the benchmark shape (n = 100
    Schwefel, 65536 chains, 100 steps, eps = 0.1), at a late level started
    near the minimizer (where the learned proposal matters): 16 of the
    logged chains, every move."""
    from paper_2408_00018_amd import learned as Lp
    wl = W.schwefel_n100_fp32()
    col = S.Schedule(chains=4096, levels=1600, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=1001,
                     precision=S.FP32)
    say("[gpu learned] trained network: collect + train")
    rec = Lp.collect(wl.func, wl.lower, wl.upper, wl.shift, col, every=16, per_level=2000)
    params, trace = Lp.train(rec, steps=1500, batch=4096, lr=1e-3, seed=0)
    say(f"[gpu learned] trained: {rec.shape[0]} records, loss {float(trace[:20].mean()):.3f} -> "
        f"{float(trace[-50:].mean()):.3f}")
    assert float(trace[-50:].mean()) < float(trace[:20].mean())
    q = bf16_matrices(params)
    rng = np.random.default_rng(7)
    x0 = W.SCHWEFEL_X_STAR + rng.uniform(-2, 2, wl.n)
    eps = 0.1
    for level in (900, 1500):
        sched = S.Schedule(chains=wl.chains, levels=level + 1, steps=wl.steps, T0=wl.T0, alpha=wl.alpha,
                           seed=wl.seed, precision=S.FP32, trace_x=True, learned=True, log_chains=64,
                           log_level=level, log_levels=1)
        say(f"[gpu learned] bench shape level {level}")
        with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
            ann.set_start(level, x0)
            ann.set_proposal(params, eps)
            ann.run(0)
            moves, final_f = ann.move_log()
            rec_l, xb = ann.trace(level, 1, with_x=True)
        T = O.temperature(wl.T0, wl.alpha, level)
        featT = float(np.float32(math.log(O.feature_tau(wl.func, wl.n) * T)))
        lo32, hi32 = box32(wl.lower, wl.upper)
        fin = final_f[0]
        win = lexi_argmin(fin)
        assert rec_l["win_chain"][0] == win and rec_l["f_win"][0] == fin[win]
        totals = dict(moves=0, learned=0, outside=0, ambiguous=0)
        for c in range(0, 64, 4):
            st = check_learned_level(wl.func, wl.n, lo32, hi32, None, wl.seed, level, T, featT,
                                     float(np.float32(eps)), q, wl.radius_frac, f32(x0), moves[0, c:c + 1], fin, [c])
            for k in totals:
                totals[k] += st[k]
        say(f"[gpu learned] trained network, level {level}: {totals}")
        assert totals["learned"] > 0.8 * totals["moves"]
        assert totals["ambiguous"] <= 0.05 * totals["moves"]
