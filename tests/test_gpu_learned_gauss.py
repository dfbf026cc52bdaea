"""GPU parity of the Gaussian proposal network kind (GELU hidden activations,
a Gaussian over the scaled displacement, raw history features, ln T) against
the FP64 oracle under the same kind.

- In-wave inference (sa_mlp_infer) within the oracle's device-precision
  bound for an FP32 GELU rounded to BF16.
- The training kernels' minibatch gradient of the Gaussian negative
  log-likelihood against the oracle's FP64 gradient (same bounds as the relu
  kind's test).
- Capture under the kind: FP64 runs give exactly the oracle's records (raw
  history, temperature feature ln T).
- Learned-mixture levels: every logged move replayed against the oracle's
  learned move (Box-Muller draw, Gaussian Metropolis-Hastings ratio), with at
  most 5% of the decisions within the bounds' reach.
- The network trained as the learned-proposal configuration is written (on
  the accepted moves of n = 4 Schwefel runs in FP64), replayed move by move at
  the benchmark shape (n = 100, 65536 chains).
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_util import (bf16_matrices, box32, check_learned_level, check_record, f32, fp32_init_state,
                         learned_params, lexi_argmin)
from test_gpu_learned import learned_case, sort_rows
from test_gpu_mlp import records

pytestmark = pytest.mark.gpu

GAUSS = O.NET_GELU_GAUSS


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


@pytest.fixture
def gauss():
    O.set_net_kind(GAUSS)
    try:
        yield
    finally:
        O.set_net_kind(O.NET_RELU_CAUCHY)


@pytest.mark.parametrize("rows,scale", [(1000, 0.1), (4099, 0.05)])
def test_infer_within_the_device_bound(S, gauss, rows, scale):
    import torch
    rng = np.random.default_rng(100 + rows)
    p = learned_params(rows, scale=scale)
    Z = np.column_stack([rng.uniform(0, 1, rows), rng.uniform(-14, 3, rows),
                         rng.normal(0, 0.05, (rows, 4))]).astype(np.float32)
    say(f"[gpu gauss] infer rows={rows} scale={scale}")
    tr = S.MLPTrainer(max_batch=64)
    tr.set_kind(S.NET_GELU_GAUSS)
    tr.set_params(p)
    out = tr.infer(torch.from_numpy(Z).cuda()).cpu().numpy().astype(np.float64)
    tr.close()
    q = bf16_matrices(p)
    worst = 0.0
    for r in range(rows):
        o, b = O.mlp_forward_device(q, Z[r].astype(np.float64))
        e = np.abs(out[r] - o)
        worst = max(worst, float(np.max(e / b)))
        assert np.all(e <= b), (r, out[r], o, b)
    say(f"[gpu gauss] infer worst err/bound {worst:.3f}")


@pytest.mark.parametrize("batch", [64, 1024])
def test_gradient_matches_oracle(S, gauss, batch):
    """Same bounds as the relu kind's gradient test: BF16 hidden activations
    and layer-2 gradient (u = 2^-9) give normwise errors of a few u per block
    and a median elementwise error below 2u."""
    import torch
    rng = np.random.default_rng(batch + 7)
    p = rng.normal(0, 0.15, S.MLP_PARAMS).astype(np.float32)
    rec = records(4096, seed=batch + 11)
    idx = rng.choice(4096, batch, replace=False).astype(np.uint32)
    say(f"[gpu gauss] gradient batch={batch}")
    tr = S.MLPTrainer(max_batch=1024)
    tr.set_kind(S.NET_GELU_GAUSS)
    tr.set_params(p)
    g, loss = tr.grad(torch.from_numpy(rec).cuda(), idx)
    tr.close()
    q = bf16_matrices(p)
    sel = rec[idx].astype(np.float64)
    lref, gref = O.mlp_loss_grad(q, sel[:, :6], sel[:, 6])
    H, I = 128, 6
    blocks = {"W1": slice(0, I * H), "b1": slice(I * H, I * H + H), "W2": slice(I * H + H, I * H + H + H * H),
              "b2": slice(I * H + H + H * H, I * H + 2 * H + H * H),
              "W3": slice(I * H + 2 * H + H * H, I * H + 4 * H + H * H),
              "b3": slice(I * H + 4 * H + H * H, I * H + 4 * H + H * H + 2)}
    u = 2.0 ** -9
    cos = float(np.dot(g, gref) / (np.linalg.norm(g) * np.linalg.norm(gref)))
    big = np.abs(gref) > 1e-2 * np.max(np.abs(gref))
    rel = np.abs(g[big] - gref[big]) / np.abs(gref[big])
    normwise = {k: float(np.linalg.norm(g[sl] - gref[sl]) / np.linalg.norm(gref[sl])) for k, sl in blocks.items()}
    say(f"[gpu gauss] batch={batch} loss {loss:.6f} vs {lref:.6f} cosine {cos:.6f} median rel {np.median(rel):.3e} "
        f"normwise {{{', '.join(f'{k}: {v:.2e}' for k, v in normwise.items())}}}")
    assert abs(loss - lref) <= 2e-3 * max(1.0, abs(lref)), (loss, lref)
    assert cos >= 0.9999
    for k, v in normwise.items():
        assert v <= 8 * u, (k, v)
    assert np.median(rel) <= 2 * u


def test_training_reduces_the_gaussian_loss(S):
    """A feature-dependent scale is learnable: displacements whose spread
    grows with the first feature; the trained network's s follows it."""
    import torch
    rng = np.random.default_rng(21)
    n = 1 << 16
    z = np.column_stack([rng.uniform(0, 1, n), np.zeros(n), rng.normal(0, 0.01, (n, 4))])
    d = rng.normal(0, 1, n) * np.exp(-6.0 + 3.0 * z[:, 0])
    rec = torch.from_numpy(np.column_stack([z, d]).astype(np.float32)).cuda()
    from paper_2408_00018_amd import learned as Lp
    params, trace = Lp.train(rec, steps=2000, batch=1024, lr=1e-3, seed=3, kind=S.NET_GELU_GAUSS)
    say(f"[gpu gauss] training loss {float(trace[:20].mean()):.3f} -> {float(trace[-50:].mean()):.3f}")
    assert float(trace[-50:].mean()) < float(trace[:20].mean()) - 1.0
    tr = S.MLPTrainer(max_batch=64)
    tr.set_kind(S.NET_GELU_GAUSS)
    tr.set_params(params)
    probe = np.zeros((3, 6), dtype=np.float32)
    probe[:, 0] = [0.1, 0.5, 0.9]
    out = tr.infer(torch.from_numpy(probe).cuda()).cpu().numpy()
    tr.close()
    say(f"[gpu gauss] learned log scales at z0 = 0.1, 0.5, 0.9: {out[:, 1]}")
    assert np.all(np.abs(out[:, 1] - (-6.0 + 3.0 * probe[:, 0])) < 0.5)


def test_capture_fp64_equals_oracle(S, gauss):
    """Records under the Gaussian kind: raw history, ln T (tau = 1)."""
    wl = W.schwefel_n4_fp64()
    kw = dict(chains=192, levels=4, steps=24, T0=5.0, alpha=0.8, seed=11)
    say("[gpu gauss] capture fp64 schwefel n=4")
    import torch
    sched = S.Schedule(precision=S.FP64, trace_x=True, **kw)
    rec = torch.zeros((1 << 16, 7), dtype=torch.float32, device="cuda")
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
        ann.set_network_kind(S.NET_GELU_GAUSS)
        ann.capture(rec)
        ann.run()
        count = ann.capture_count()
        trace = ann.trace()
    got = rec.cpu().numpy()
    ref, rcount = O.sa_run_capture(wl.func, wl.lower, wl.upper, wl.shift, capacity=1 << 16, tau=1.0, **kw)
    assert count == rcount == int(trace["accepts"].sum())
    assert np.array_equal(sort_rows(got[:count]), sort_rows(ref))
    # raw history: the features are accepted scaled displacements themselves
    assert np.all(np.abs(got[:count, 2:6]) <= 0.1 + 1e-7)
    assert np.array_equal(np.unique(got[:count, 1]), np.sort(np.float32(np.log(5.0 * 0.8 ** np.arange(4)))))


@pytest.mark.parametrize("name,steps", [("schwefel_n16", 32), ("rastrigin_n9_table", 32), ("ackley_n12", 31)])
def test_learned_per_move_parity(S, name, steps):
    wl = learned_case(name)
    kw = dict(chains=512, levels=3, steps=steps, T0=5.0 if wl.func != W.SCHWEFEL else 20.0, alpha=0.7, seed=29)
    eps = 0.25
    p = learned_params(37, scale=0.05, sigma0=0.1)
    say(f"[gpu gauss] per-move {name}")
    sched = S.Schedule(chains=kw["chains"], levels=kw["levels"], steps=steps, T0=kw["T0"], alpha=kw["alpha"],
                       seed=kw["seed"], precision=S.FP32, trace_x=True, learned=True, log_chains=64, log_level=0,
                       log_levels=kw["levels"])
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
        ann.set_network_kind(S.NET_GELU_GAUSS)
        ann.set_proposal(p, eps)
        ann.run()
        rec, xb = ann.trace(with_x=True)
        x_rec, f_rec, rec_level = ann.best()
        moves, final_f = ann.move_log()
    g = dict(rec=rec, xb=xb, x_rec=x_rec, f_rec=f_rec, rec_level=rec_level)
    lo32, hi32 = box32(wl.lower, wl.upper)
    sh32 = None if wl.shift is None else f32(wl.shift)
    q = bf16_matrices(p)
    totals = dict(moves=0, learned=0, outside=0, ambiguous=0, max_dl_excess=0.0, max_rel_excess=0.0)
    wl_run = wl.with_(chains=kw["chains"], seed=kw["seed"])
    for level in range(kw["levels"]):
        T = O.temperature(kw["T0"], kw["alpha"], level)
        featT = float(np.float32(math.log(T)))
        fin = final_f[level]
        win = lexi_argmin(fin)
        assert rec["win_chain"][level] == win and rec["f_win"][level] == fin[win]
        for c in range(0, 64, 3):
            x0 = fp32_init_state(wl_run, c) if level == 0 else xb[level - 1]
            st = check_learned_level(wl.func, wl.n, lo32, hi32, sh32, kw["seed"], level, T, featT,
                                     float(np.float32(eps)), q, 0.1, x0, moves[level, c:c + 1], fin, [c],
                                     kind=GAUSS)
            for k in totals:
                totals[k] = max(totals[k], st[k]) if k.startswith("max") else totals[k] + st[k]
    say(f"[gpu gauss] {name}: {totals}")
    assert totals["learned"] > 0.5 * totals["moves"]
    assert totals["ambiguous"] <= 0.05 * totals["moves"]
    check_record(wl_run.with_(levels=kw["levels"]), g)


def test_kind_switch_and_graph_replay(S):
    """Graph-replayed Gaussian-kind levels equal eager ones; switching the
    kind back gives the relu network's run bit for bit."""
    wl = learned_case("schwefel_n16")
    p = learned_params(5, scale=0.05, sigma0=0.02)
    kw = dict(chains=1024, levels=6, steps=20, T0=10.0, alpha=0.8, seed=2)
    cols = ["win_chain", "accepts", "f_win", "f_best", "f_rec"]

    def run(kinds, graph=False, chunks=None):
        sched = S.Schedule(precision=S.FP32, trace_x=True, learned=True, graph=graph, **kw)
        with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
            for k in kinds:
                ann.set_network_kind(k)
            ann.set_proposal(p, 0.1)
            for c in (chunks or [0]):
                ann.run(c)
            return ann.trace(with_x=True)

    a, ax = run([S.NET_GELU_GAUSS])
    b, bx = run([S.NET_GELU_GAUSS], graph=True, chunks=[2, 4])
    assert np.array_equal(a[cols], b[cols]) and np.array_equal(ax, bx)
    relu, rx = run([])
    back, bkx = run([S.NET_GELU_GAUSS, S.NET_RELU_CAUCHY])
    assert np.array_equal(relu[cols], back[cols]) and np.array_equal(rx, bkx)
    assert not np.array_equal(ax, rx)


def test_written_configuration_network_at_the_bench_shape(S):
    """The learned-proposal configuration as written: GELU/Gaussian network
    trained on accepted moves of n = 4 Schwefel runs (FP64, 256 chains, T0 10,
    alpha 0.99, 200 levels x 50 steps, successive seeds), replayed move by
    move at the benchmark shape (n = 100, 65536 chains, eps = 0.1) at a level
    inside the training runs' temperature range, started near x*."""
    from paper_2408_00018_amd import learned as Lp
    cfg1 = W.schwefel_n4_fp64()
    col = S.Schedule(chains=cfg1.chains, levels=cfg1.levels, steps=cfg1.steps, T0=cfg1.T0, alpha=cfg1.alpha,
                     seed=cfg1.seed, precision=S.FP64)
    say("[gpu gauss] written configuration: collect n=4 runs + train")
    rec, runs = Lp.collect_runs(cfg1.func, cfg1.lower, cfg1.upper, cfg1.shift, col, records=1 << 20,
                                kind=S.NET_GELU_GAUSS)
    params, trace = Lp.train(rec, steps=800, batch=4096, lr=1e-3, seed=0, kind=S.NET_GELU_GAUSS)
    say(f"[gpu gauss] {rec.shape[0]} records from {runs} runs, loss {float(trace[:20].mean()):.3f} -> "
        f"{float(trace[-50:].mean()):.3f}")
    assert float(trace[-50:].mean()) < float(trace[:20].mean())
    q = bf16_matrices(params)
    wl = W.schwefel_n100_fp32()
    rng = np.random.default_rng(9)
    x0 = W.SCHWEFEL_X_STAR + rng.uniform(-20, 20, wl.n)
    eps, level = 0.1, 100
    sched = S.Schedule(chains=wl.chains, levels=level + 1, steps=wl.steps, T0=wl.T0, alpha=wl.alpha, seed=wl.seed,
                       precision=S.FP32, trace_x=True, learned=True, log_chains=64, log_level=level, log_levels=1)
    with S.Annealer(wl.func, wl.lower, wl.upper, wl.shift, schedule=sched) as ann:
        ann.set_network_kind(S.NET_GELU_GAUSS)
        ann.set_start(level, x0)
        ann.set_proposal(params, eps)
        ann.run(0)
        moves, final_f = ann.move_log()
        rec_l, _ = ann.trace(level, 1, with_x=True)
    T = O.temperature(wl.T0, wl.alpha, level)
    featT = float(np.float32(math.log(T)))
    lo32, hi32 = box32(wl.lower, wl.upper)
    fin = final_f[0]
    assert rec_l["win_chain"][0] == lexi_argmin(fin)
    totals = dict(moves=0, learned=0, outside=0, ambiguous=0)
    for c in range(0, 64, 4):
        st = check_learned_level(wl.func, wl.n, lo32, hi32, None, wl.seed, level, T, featT, float(np.float32(eps)),
                                 q, wl.radius_frac, f32(x0), moves[0, c:c + 1], fin, [c], kind=GAUSS)
        for k in totals:
            totals[k] += st[k]
    say(f"[gpu gauss] written-configuration network at the bench shape, level {level}: {totals}")
    assert totals["learned"] > 0.8 * totals["moves"]
    assert totals["ambiguous"] <= 0.05 * totals["moves"]
