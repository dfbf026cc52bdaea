"""Pins of the oracle's second proposal-network kind, the written learned-proposal
configuration: GELU hidden activations (exact erf form), a Gaussian
distribution over the scaled displacement (mean, log standard deviation), the
last accepted scaled displacements entered as they are.

- Forward pass, Gaussian negative log-likelihood and its gradient against
  PyTorch float64 autograd (torch's exact GELU, torch.distributions.Normal),
  and the gradient against central differences.
- The proposal density against scipy's normal log density; the move's draw is
  standard normal (Kolmogorov-Smirnov, moments).
- Stationarity: a one-coordinate chain at fixed T under an asymmetric GELU
  network samples exp(-f/T)/Z, for the pure learned move and the mixture
  (max |z| about 1.1, total variation below 0.004).  Power, measured by
  planting each mistake in a copy of the oracle: with the Hastings term
  dropped the histogram misses by 26 and 6 standard errors (total variation
  0.86 and 0.56 at eps = 0 and 0.1), with it inverted by total variation 1.
- The device-precision forward pass (BF16 weights and activations after an
  FP32 GELU, FP32 accumulation) lies within its bound of an independent torch
  evaluation of the same contract.
- The kind switch leaves the other kind's functions unchanged.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from test_oracle_learned import (EDGES, HI, LO, OFF_B1, OFF_B2, OFF_B3, OFF_W1, OFF_W2, OFF_W3, SHIFT, T,
                                 asymmetric_net, histogram_check, run_chains)


@pytest.fixture
def gelu_kind():
    O.set_net_kind(O.NET_GELU_GAUSS)
    try:
        yield
    finally:
        O.set_net_kind(O.NET_RELU_CAUCHY)


def torch_loss(p64, Z, delta):
    import torch
    p = torch.tensor(p64, dtype=torch.float64, requires_grad=True)
    W1, b1, W2, b2, W3, b3 = (t for t in torch.split(p, [6 * 128, 128, 128 * 128, 128, 256, 2]))
    z = torch.tensor(Z, dtype=torch.float64)
    h1 = torch.nn.functional.gelu(z @ W1.view(6, 128) + b1)
    h2 = torch.nn.functional.gelu(h1 @ W2.view(128, 128) + b2)
    o = h2 @ W3.view(128, 2) + b3
    dist = torch.distributions.Normal(o[:, 0], torch.exp(o[:, 1]))
    loss = -dist.log_prob(torch.tensor(delta, dtype=torch.float64)).mean()
    loss.backward()
    return float(loss), p.grad.numpy(), o.detach().numpy()


def test_forward_loss_gradient_against_torch(gelu_kind):
    rng = np.random.default_rng(3)
    p = rng.normal(0.0, 0.15, O.mlp_nparam())
    Z = rng.normal(0.0, 1.0, (9, 6))
    delta = rng.normal(0.0, 0.05, 9)
    loss_t, grad_t, out_t = torch_loss(p, Z, delta)
    for r in range(9):
        out, _, _ = O.mlp_forward(p, Z[r])
        assert np.allclose(out, out_t[r], rtol=1e-12, atol=1e-13)
    loss, grad = O.mlp_loss_grad(p, Z, delta)
    assert abs(loss - loss_t) <= 1e-12 * abs(loss_t)
    assert np.allclose(grad, grad_t, rtol=1e-9, atol=1e-12)
    # central differences on sampled parameters
    for i in rng.choice(p.size, 40, replace=False):
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp = O.mlp_loss_grad(pp, Z, delta, with_grad=False)
        lm = O.mlp_loss_grad(pm, Z, delta, with_grad=False)
        assert abs((lp - lm) / (2 * h) - grad[i]) <= 1e-6 * max(1.0, abs(grad[i]))


def test_activation_and_density(gelu_kind):
    import torch
    a = np.linspace(-6, 6, 241)
    g = torch.nn.functional.gelu(torch.tensor(a, dtype=torch.float64)).numpy()
    assert np.allclose([O.act(v) for v in a], g, rtol=1e-14, atol=1e-16)
    for v in (-2.0, -0.7, 0.0, 0.3, 2.5):
        h = 1e-6
        assert abs(O.act_grad(v) - (O.act(v + h) - O.act(v - h)) / (2 * h)) < 1e-8
    for d, mu, s in ((0.01, 0.0, -3.0), (-0.2, 0.1, -1.0), (0.5, -0.5, 0.3)):
        assert abs(O.proposal_logpdf(d, mu, s) - stats.norm.logpdf(d, mu, math.exp(s))) < 1e-12
    assert O.hist_feature(0.0123) == 0.0123 and O.hist_feature(-0.5) == -0.5


def test_draw_is_standard_normal(gelu_kind):
    t = np.array([O.learn_draw(9, 0, 4, c, s) for c in range(40) for s in range(500)])
    ks = stats.kstest(t, "norm")
    assert ks.pvalue > 1e-3, ks
    assert abs(t.mean()) < 0.03 and abs(t.std() - 1.0) < 0.02


def gelu_asymmetric_net(c_mu=0.25, c_s=24.0, sigma=0.03):
    """asymmetric_net's wiring under GELU, centred where the chains run: with
    z0 the scaled coordinate, h = gelu(gelu(z0)) is increasing on [0, 1], and
    mu = k c_mu (h - h_c), s = ln(sigma) + k c_s (h - h_c) with h_c = h at the
    minimum's location and k = 1 / h'(z0) there, so that mu and s vary with x
    as in the relu network and q(x' | x) != q(x | x')."""
    p = asymmetric_net(c_mu=c_mu, c_s=c_s, sigma=sigma)
    zc = (SHIFT - LO) / (HI - LO)
    hc = O.act(O.act(zc))
    k = 1.0 / (O.act_grad(zc) * O.act_grad(O.act(zc)))
    p[OFF_W3 + 0] = k * c_mu
    p[OFF_W3 + 1] = k * c_s
    p[OFF_B3 + 0] = -k * c_mu * hc
    p[OFF_B3 + 1] = math.log(sigma) - k * c_s * hc
    return p


@pytest.mark.parametrize("eps", [0.0, 0.1])
def test_mixture_samples_exp_minus_f_over_T(gelu_kind, eps):
    paths, acc = run_chains(gelu_asymmetric_net(), eps)
    z, tv, pe, mean = histogram_check(paths, EDGES)
    print(f"gelu/gauss eps={eps}: accepts={acc} max|z|={np.abs(z).max():.2f} TV={tv:.4f}")
    assert acc > 20000
    assert np.abs(z).max() < 5.0, (z, pe, mean)
    assert tv < 0.02


def _bf16(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def contract_forward_torch_gelu(p64, z, rng):
    """The device's contract under GELU, evaluated independently: FP32
    accumulation in a random order, torch's FP32 GELU, BF16 rounding."""
    import torch
    W1, b1, W2, b2, W3, b3 = O.mlp_unpack(p64)
    zf = np.asarray(z, dtype=np.float32)
    hi = _bf16(zf)
    lo = _bf16((zf.astype(np.float64) - hi).astype(np.float32))

    def layer(inp, Wm, b):
        out = np.zeros(Wm.shape[1], dtype=np.float32)
        for j in range(Wm.shape[1]):
            terms = (inp * Wm[:, j]).astype(np.float32)
            acc = np.float32(b[j])
            for k in rng.permutation(len(terms)):
                acc = np.float32(acc + terms[k])
            out[j] = acc
        return out

    def act(a):
        return _bf16(torch.nn.functional.gelu(torch.from_numpy(a)).numpy())
    h1 = act(layer(np.concatenate([hi, lo]), np.vstack([W1, W1]), b1))
    h2 = act(layer(h1, W2, b2))
    return layer(h2, W3, b3).astype(np.float64)


def test_device_precision_forward_within_its_bound(gelu_kind):
    rng = np.random.default_rng(12)
    for case in range(10):
        p = rng.normal(0.0, 0.08, O.mlp_nparam()).astype(np.float32)
        p[-1] = -3.0
        for a, b in ((OFF_W1, OFF_B1), (OFF_W2, OFF_B2), (OFF_W3, OFF_B3)):
            p[a:b] = _bf16(p[a:b])
        p64 = p.astype(np.float64)
        z = np.concatenate([rng.uniform(0, 1, 1), rng.uniform(-6, 8, 1), rng.normal(0, 0.05, 4)])
        z = z.astype(np.float32).astype(np.float64)
        out, bound = O.mlp_forward_device(p64, z)
        ref = contract_forward_torch_gelu(p64, z, rng)
        _, loose = O.mlp_forward_bound(p64, z)
        assert np.all(np.abs(out - ref) <= bound), (case, out, ref, bound)
        assert np.all(bound < 0.1 * loose), (bound, loose)


def test_kind_switch_leaves_the_other_kind_alone():
    rng = np.random.default_rng(5)
    p = rng.normal(0.0, 0.1, O.mlp_nparam())
    z = rng.normal(0.0, 1.0, 6)
    before, _, _ = O.mlp_forward(p, z)
    O.set_net_kind(O.NET_GELU_GAUSS)
    try:
        gelu, _, _ = O.mlp_forward(p, z)
    finally:
        O.set_net_kind(O.NET_RELU_CAUCHY)
    after, _, _ = O.mlp_forward(p, z)
    assert np.array_equal(before, after) and not np.allclose(before, gelu)
    assert O.act(-1.0) == 0.0 and O.hist_feature(0.0) == 0.0
