"""Pins of the oracle's learned-proposal network (FP64): forward pass, loss,
gradient, activation, optimiser, proposal density and draws, each against a
library routine (PyTorch CPU float64 autograd / functional / optimiser,
scipy), a finite difference, or a closed form."""
import math

import numpy as np
import pytest

import oracle as O


def random_params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, O.mlp_nparam())


def random_batch(seed, b=16):
    rng = np.random.default_rng(seed)
    Z = np.column_stack([rng.uniform(0, 1, b), rng.uniform(-3, 3, b), rng.normal(0, 0.05, (b, 4))])
    d = rng.normal(0, 0.05, b)
    return Z, d


def test_parameter_count():
    # 6*128 + 128 + 128*128 + 128 + 128*2 + 2
    assert O.mlp_nparam() == 17666


def test_activation_against_torch_and_identities():
    torch = pytest.importorskip("torch")
    xs = np.linspace(-8, 8, 161)
    ref = torch.relu(torch.tensor(xs, dtype=torch.float64)).numpy()
    got = np.array([O.act(x) for x in xs])
    assert np.array_equal(got, ref)
    for x in (0.3, 1.7, 5.0):
        assert O.act(x) - O.act(-x) == x
    assert O.act(0.0) == 0.0 and O.act_grad(0.0) == 0.0
    # derivative against a central difference away from the kink
    for x in np.concatenate([np.linspace(-4, -0.1, 9), np.linspace(0.1, 4, 9)]):
        fd = (O.act(x + 1e-6) - O.act(x - 1e-6)) / 2e-6
        assert abs(O.act_grad(x) - fd) < 1e-8


def test_forward_zero_weights_closed_form():
    p = np.zeros(O.mlp_nparam())
    p[-2], p[-1] = 0.3, -1.2  # b3: mu, ln sigma
    out, a1, a2 = O.mlp_forward(p, [0.5, 1.0, 0.1, 0.2, 0.3, 0.4])
    assert out[0] == 0.3 and out[1] == -1.2
    assert np.all(a1 == 0) and np.all(a2 == 0)
    # Cauchy negative log-likelihood of d = 0.7: s + ln pi + ln(1 + ((d - mu)/e^s)^2)
    loss = O.mlp_loss_grad(p, np.zeros((1, 6)), [0.7], with_grad=False)
    assert abs(loss - (-1.2 + math.log(math.pi) + math.log1p((0.4 * math.exp(1.2)) ** 2))) < 1e-12


def _torch_loss_grad(params, Z, d):
    torch = pytest.importorskip("torch")
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in O.mlp_unpack(params)]
    z = torch.tensor(Z, dtype=torch.float64)
    h1 = torch.relu(z @ W1 + b1)
    h2 = torch.relu(h1 @ W2 + b2)
    o = h2 @ W3 + b3
    mu, s = o[:, 0], o[:, 1]
    dd = torch.tensor(d, dtype=torch.float64)
    loss = -torch.distributions.Cauchy(mu, torch.exp(s)).log_prob(dd).mean()
    loss.backward()
    g = np.concatenate([t.grad.numpy().ravel() for t in (W1, b1, W2, b2, W3, b3)])
    return float(loss.detach()), g


def test_loss_and_gradient_against_torch_autograd():
    p = random_params(1)
    Z, d = random_batch(2, 24)
    loss, g = O.mlp_loss_grad(p, Z, d)
    tl, tg = _torch_loss_grad(p, Z, d)
    assert abs(loss - tl) < 1e-12 * max(1.0, abs(tl))
    assert np.max(np.abs(g - tg)) < 1e-11 * max(1.0, np.max(np.abs(tg)))


def test_gradient_against_central_differences():
    p = random_params(3)
    Z, d = random_batch(4, 8)
    _, g = O.mlp_loss_grad(p, Z, d)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(768, 20, replace=False),  # W1
                          768 + rng.choice(128, 10, replace=False),  # b1
                          896 + rng.choice(16384, 40, replace=False),  # W2
                          17280 + rng.choice(128, 10, replace=False),  # b2
                          17408 + rng.choice(256, 20, replace=False),  # W3
                          [17664, 17665]])  # b3
    h = 1e-6
    for i in idx:
        pp = p.copy()
        pp[i] += h
        lp = O.mlp_loss_grad(pp, Z, d, with_grad=False)
        pp[i] -= 2 * h
        lm = O.mlp_loss_grad(pp, Z, d, with_grad=False)
        fd = (lp - lm) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(abs(fd), 1e-3), (i, g[i], fd)


def test_adam_against_torch_optimizer():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    p0 = rng.normal(0, 1, 50)
    grads = [rng.normal(0, 1, 50) for _ in range(5)]
    p = p0.copy()
    m = np.zeros(50)
    v = np.zeros(50)
    for t, gr in enumerate(grads, 1):
        O.adam_step(p, gr.copy(), m, v, t, lr=1e-2)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for gr in grads:
        opt.zero_grad()
        tp.grad = torch.tensor(gr, dtype=torch.float64)
        opt.step()
    assert np.max(np.abs(p - tp.detach().numpy())) < 1e-12


def test_proposal_logpdf_is_a_cauchy_density():
    from scipy.stats import cauchy
    for mu, s in ((0.0, 0.0), (0.1, -2.0), (-0.3, 0.5)):
        for x in (-1.0, 0.0, 0.05, 2.0):
            assert abs(O.proposal_logpdf(x, mu, s) - cauchy.logpdf(x, loc=mu, scale=math.exp(s))) < 1e-12
    from scipy.integrate import quad
    total, err = quad(lambda x: math.exp(O.proposal_logpdf(x, 0.02, -3.0)), -np.inf, np.inf, points=None)
    assert abs(total - 1.0) < 1e-8


def test_training_reduces_loss_on_synthetic_data():
    """A few hundred Adam steps on records whose displacement scale depends on
    the first feature reduce the NLL well below its starting value, and the
    network learns sigma as a function of that feature."""
    rng = np.random.default_rng(11)
    n = 512
    Z = np.column_stack([rng.uniform(0, 1, n), np.zeros(n), np.zeros((n, 4))])
    sig = np.where(Z[:, 0] < 0.5, 0.01, 0.1)
    d = rng.normal(0, 1, n) * sig
    p = random_params(12, scale=0.05)
    m, v = np.zeros_like(p), np.zeros_like(p)
    l0 = O.mlp_loss_grad(p, Z, d, with_grad=False)
    for t in range(1, 301):
        _, g = O.mlp_loss_grad(p, Z, d)
        O.adam_step(p, g, m, v, t, lr=3e-3)
    l1 = O.mlp_loss_grad(p, Z, d, with_grad=False)
    assert l1 < l0 - 1.0
    s_lo = O.mlp_forward(p, [0.25, 0, 0, 0, 0, 0])[0][1]
    s_hi = O.mlp_forward(p, [0.75, 0, 0, 0, 0, 0])[0][1]
    assert s_hi - s_lo > 1.0  # ln(0.1 / 0.01) = 2.3


def test_learn_draw_is_standard_cauchy_and_follows_its_counters():
    """Draws of learned moves: a standard Cauchy sample (KS test, median and
    quartiles), each the inverse distribution function at the first uniform
    of its Philox block, and a different stream per problem id."""
    from scipy import stats
    t = np.array([O.learn_draw(5, 0, lv, ch, st) for lv in range(4) for ch in range(50) for st in range(100)])
    assert stats.kstest(t, "cauchy").pvalue > 1e-3
    assert abs(np.median(t)) < 0.05
    assert abs(np.quantile(t, 0.75) - 1.0) < 0.06 and abs(np.quantile(t, 0.25) + 1.0) < 0.06
    r = O.philox4x32_10([7, 3, 11, 3], [5, 0])
    u0 = O.uniform(int(r[0]))
    # the Cauchy distribution function 1/2 + atan(t)/pi returns the uniform
    assert abs(0.5 + math.atan(O.learn_draw(5, 0, 3, 11, 7)) / math.pi - u0) < 1e-12
    assert O.learn_draw(5, 1, 3, 11, 7) != O.learn_draw(5, 0, 3, 11, 7)


def _bf16(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_forward_bound_covers_bf16_activations():
    """The first-order bound holds for an evaluation that rounds every hidden
    activation to BF16, is not vacuous, and is zero for a zero network."""
    rng = np.random.default_rng(3)
    worst, ratios = 0.0, []
    for t in range(200):
        p = random_params(100 + t, scale=rng.choice([0.05, 0.1, 0.3]))
        z = rng.normal(0, 1, 6)
        out, bound = O.mlp_forward_bound(p, z)
        W1, b1, W2, b2, W3, b3 = O.mlp_unpack(p)
        h1 = _bf16(np.maximum(z @ W1 + b1, 0))
        h2 = _bf16(np.maximum(h1 @ W2 + b2, 0))
        o = h2 @ W3 + b3
        e = np.abs(o - out)
        assert np.all(e <= bound)
        worst = max(worst, float(np.max(e / bound)))
        ratios.append(np.max(bound / (np.abs(out) + 1e-12)))
    assert worst > 1e-3          # the bound is of the right order, not vacuous
    assert np.median(ratios) < 1.0
    out, bound = O.mlp_forward_bound(np.zeros(O.mlp_nparam()), np.ones(6))
    assert np.all(bound == 0)


def test_capture_records_match_the_replayed_moves():
    """Records of a capture run equal what the replay log of the same levels
    implies: features at the old state, history of the last four accepted
    scaled displacements (reset at each level), the accepted displacement;
    their number is the run's accepted-move count."""
    lo, hi = np.full(3, -500.0), np.full(3, 500.0)
    kw = dict(seed=9, chains=8, steps=30, T0=20.0, alpha=0.8)
    run = O.sa_run(O.SCHWEFEL, lo, hi, levels=3, level_begin=0, **kw)
    rec, count = O.sa_run_capture(O.SCHWEFEL, lo, hi, levels=3, capacity=4096, **kw)
    assert count == int(run["accepts"].sum()) == rec.shape[0]
    expect = []
    # levels 1 and 2 start from the previous winner; replay them
    for level in (1, 2):
        T = O.temperature(kw["T0"], kw["alpha"], level)
        logs = O.replay_level(O.SCHWEFEL, lo, hi, None, seed=9, steps=30, T=T, level=level,
                              x_start=run["x_best"][level - 1], chain0=0, nchains=8)
        for c in range(8):
            h = [0.0] * 4
            for s in range(30):
                if logs["acc"][c, s]:
                    d = logs["d"][c, s]
                    w = hi[d] - lo[d]
                    dl = (logs["x_new"][c, s] - logs["x_old"][c, s]) / w
                    feats = [math.copysign(math.log1p(2.0 ** 24 * abs(v)) / 16, v) for v in h]
                    expect.append([(logs["x_old"][c, s] - lo[d]) / w, math.log(3 * T)] + feats + [dl])
                    h = [dl] + h[:3]
    got_late = rec[-len(expect):]
    assert np.array_equal(got_late, np.array(expect, dtype=np.float32))
