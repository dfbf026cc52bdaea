"""Pins of the oracle's learned-proposal mixture move (an extension of the
method: the Metropolis acceptance of Sec. 2.1, eq. (5), in its
Metropolis-Hastings form, with a network proposal mixed with the plain move).

- Stationarity: at a fixed temperature a one-coordinate chain must sample
  exp(-f/T)/Z.  With a network that ignores the history features the kernel
  is exactly reversible, so the visited histogram must match the density
  integrated independently here, for the pure learned move (eps = 0), the
  mixture (eps = 0.1) and the plain move (eps = 1).  The network is built so
  that its proposal is strongly asymmetric (its scale grows e-fold over a
  few units of x, its location drifts with x): a missing or inverted
  Hastings term shifts the histogram far outside the tolerance (checked by
  planting both mistakes in a copy of the oracle).
- With history features the chain is adaptive; its deviation from
  exp(-f/T)/Z is measured and bounded.
- eps = 1 reproduces the plain replay (orc_replay_level) bit for bit.
- The device-precision forward pass (BF16 weight matrices and activations,
  FP32 accumulation) lies within its own bound of an independent torch/numpy
  evaluation of the same contract, and its bound is far tighter than the
  first-order worst case.
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O

H, I = O.MLP_HIDDEN, O.MLP_INPUTS
OFF_W1, OFF_B1 = 0, I * H
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + 2 * H

# Ackley (Appendix, Test 1) in one dimension, box of the configurations used
# here, shifted; at T = 1 its density exp(-f/T) lives in |x - s| < 5, far
# from the box edges (where the plain move's clamp would add atoms).
LO, HI, SHIFT, T = -32.768, 32.768, 1.7, 1.0
W = HI - LO


def ackley1(x):
    y = np.asarray(x, dtype=np.float64) - SHIFT
    return -20.0 * np.exp(-0.2 * np.abs(y)) - np.exp(np.cos(2.0 * np.pi * y)) + 20.0 + math.e


def asymmetric_net(history=False, c_mu=0.25, c_s=24.0, sigma=0.03):
    """mu = c_mu (z0 - 1/2), s = ln(sigma) + c_s (z0 - 1/2) [+ |history feature 0| / 2]:
    a location drift of 0.03 (2 units of x) and a log scale that changes by
    about 3 over the density's support, so q(x' | x) != q(x | x').  Measured
    power: with the Hastings term dropped the histogram misses by 7-14
    standard errors (total variation 0.04-0.07), with it inverted by 20-30
    (0.76-0.86), against at most 2 (0.005) for the correct kernel."""
    p = np.zeros(O.mlp_nparam())
    p[OFF_W1 + 0 * H + 0] = 1.0          # a1_0 = z0
    p[OFF_W2 + 0 * H + 0] = 1.0          # a2_0 = h1_0
    p[OFF_W3 + 0 * 2 + 0] = c_mu         # mu
    p[OFF_W3 + 0 * 2 + 1] = c_s          # s
    p[OFF_B3 + 0] = -0.5 * c_mu
    p[OFF_B3 + 1] = math.log(sigma) - 0.5 * c_s
    if history:
        p[OFF_W1 + 2 * H + 1] = 1.0      # relu(+h0) and relu(-h0): |h0|
        p[OFF_W1 + 2 * H + 2] = -1.0
        p[OFF_W2 + 1 * H + 1] = 1.0
        p[OFF_W2 + 2 * H + 1] = 1.0
        p[OFF_W3 + 1 * 2 + 1] = 0.5      # s grows with the last accepted step
    return p


def expected_bins(edges):
    xs = np.linspace(LO, HI, 2_000_001)
    dens = np.exp(-ackley1(xs) / T)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(xs))])
    cdf /= cdf[-1]
    return np.diff(np.interp(edges, xs, cdf))


def run_chains(params, eps, chains=16, steps=40000, burn=2000, thin=5):
    def one(c):
        r = O.learned_run(params, O.NET_FP64, O.ACKLEY, [LO], [HI], [SHIFT], seed=77, level=0, chain0=c, nchains=1,
                          steps=steps, T=T, featT=0.0, eps=eps, x_start=[SHIFT + 0.3], trace0=True)
        return r["trace0"][burn::thin], int(r["accepts"][0])
    with ThreadPoolExecutor(max_workers=8) as ex:
        out = list(ex.map(one, range(chains)))
    return [o[0] for o in out], sum(o[1] for o in out)


def histogram_check(paths, edges):
    """Per-chain bin frequencies, their across-chain standard errors, and the
    z-score of the pooled frequency against the exact bin probability."""
    pe = expected_bins(edges)
    freqs = np.array([np.histogram(p, bins=edges)[0] / len(p) for p in paths])
    mean = freqs.mean(axis=0)
    se = freqs.std(axis=0, ddof=1) / math.sqrt(len(paths)) + 1e-4
    z = (mean - pe) / se
    tv = 0.5 * np.abs(mean - pe).sum()
    return z, tv, pe, mean


EDGES = np.concatenate([[LO], SHIFT + np.linspace(-4.0, 4.0, 25), [HI]])


@pytest.mark.parametrize("eps", [0.0, 0.1, 1.0])
def test_mixture_samples_exp_minus_f_over_T(eps):
    paths, acc = run_chains(asymmetric_net(), eps)
    z, tv, pe, mean = histogram_check(paths, EDGES)
    print(f"eps={eps}: accepts={acc} max|z|={np.abs(z).max():.2f} TV={tv:.4f}")
    assert acc > 20000
    assert np.abs(z).max() < 5.0, (z, pe, mean)
    assert tv < 0.02


def test_histogram_check_rejects_a_nearby_density():
    """Power of the check: the same chains judged against exp(-f/(1.3 T)), a
    density they were not drawn from, fail it."""
    paths, _ = run_chains(asymmetric_net(), 0.1, chains=8, steps=20000)
    global T
    saved = T
    try:
        T = 1.3 * saved
        z, tv, _, _ = histogram_check(paths, EDGES)
    finally:
        T = saved
    assert np.abs(z).max() > 5.0 and tv > 0.02


def test_history_features_bias_is_small():
    """With the last accepted step in the proposal scale the chain is adaptive
    (the reverse move sees another history), so exactness is lost; the
    deviation from exp(-f/T)/Z is measured and must stay small."""
    paths, _ = run_chains(asymmetric_net(history=True), 0.1)
    z, tv, _, _ = histogram_check(paths, EDGES)
    print(f"history: max|z|={np.abs(z).max():.2f} TV={tv:.4f}")
    assert tv < 0.05


def test_eps_one_is_the_plain_replay_bit_for_bit():
    n = 5
    rng = np.random.default_rng(3)
    lo, hi = np.full(n, -500.0), np.full(n, 500.0)
    sh = rng.uniform(-50, 50, n)
    x0 = rng.uniform(-400, 400, n)
    for func in (O.SCHWEFEL, O.RASTRIGIN, O.ACKLEY):
        if func != O.SCHWEFEL:
            lo, hi = np.full(n, -5.12 if func == O.RASTRIGIN else -32.768), np.full(n, 5.12 if func == O.RASTRIGIN
                                                                                    else 32.768)
            sh = rng.uniform(lo * 0.5, hi * 0.5)
            x0 = rng.uniform(lo * 0.8, hi * 0.8)
        T_ = 3.0
        ref = O.replay_level(func, lo, hi, sh, seed=9, steps=300, T=T_, level=4, x_start=x0, chain0=10, nchains=6)
        got = O.learned_run(asymmetric_net(history=True), O.NET_FP64, func, lo, hi, sh, seed=9, level=4, chain0=10,
                            nchains=6, steps=300, T=T_, featT=1.0, eps=1.0, x_start=x0, log=True)
        assert np.array_equal(got["d"], ref["d"].ravel())
        for k in ("x_old", "x_new", "df"):
            assert np.array_equal(got[k], ref[k].ravel()), k
        assert np.array_equal(got["accept"].astype(bool), ref["acc"].ravel())
        assert np.array_equal(got["x_final"], ref["x_final"])


def test_proposal_components():
    """A learned proposal is x_d + (mu + e^s t)(u_d - l_d) with (mu, s) the
    network at x_d's features and t the move's Cauchy draw; the component is
    plain exactly when the mixture uniform is below eps; an out-of-box
    learned proposal is rejected with no cost change."""
    p = asymmetric_net(history=True, sigma=0.4)
    lo, hi = np.full(3, LO), np.full(3, HI)
    x = np.array([1.0, -3.0, 20.0])
    hist = [0.01, -0.2, 0.0, 0.003]
    seen_out = seen_plain = 0
    for step in range(200):
        pr = O.learned_propose(p, O.NET_FP64, seed=5, level=2, chain=7, step=step, x=x, lower=lo, upper=hi, featT=0.5,
                               eps=0.3, hist=hist)
        d = pr["d"]
        assert pr["plain"] == (O.learn_mix(5, 0, 2, 7, step) < 0.3)
        if pr["plain"]:
            seen_plain += 1
            continue
        z = [(x[d] - LO) / W, 0.5] + [O.hist_feature(h) for h in hist]
        (mu, s), _, _ = O.mlp_forward(p, z)
        t = O.learn_draw(5, 0, 2, 7, step)
        assert pr["mu"] == mu and pr["s"] == s and pr["t"] == t
        assert abs(pr["x_new"] - (x[d] + (mu + math.exp(s) * t) * W)) <= 1e-12 * (abs(x[d]) + W * (1 + abs(t)))
        take, det = O.learned_accept(p, O.NET_FP64, O.ACKLEY, lower=lo, upper=hi, shift=None, seed=5, level=2,
                                     chain=7, step=step, T=2.0, featT=0.5, plain=False, x=x, d=d, x_new=pr["x_new"],
                                     mu=mu, s=s, hist=hist)
        if not (LO <= pr["x_new"] <= HI):
            seen_out += 1
            assert not take and det["df"] == 0.0
        else:
            assert take == (det["u2"] < math.exp(det["log_ratio"]))
    assert seen_out > 5 and seen_plain > 20


def _bf16(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def contract_forward_torch(p64, z, rng):
    """The device's precision contract evaluated independently: torch's BF16
    rounding, FP32 accumulation in a random order per output."""
    W1, b1, W2, b2, W3, b3 = O.mlp_unpack(p64)
    zf = np.asarray(z, dtype=np.float32)
    hi = _bf16(zf)
    lo = _bf16((zf.astype(np.float64) - hi).astype(np.float32))

    def layer(inp, Wm, b):
        out = np.zeros(Wm.shape[1])
        for j in range(Wm.shape[1]):
            terms = (inp * Wm[:, j]).astype(np.float32)
            acc = np.float32(b[j])
            for k in rng.permutation(len(terms)):
                acc = np.float32(acc + terms[k])
            out[j] = acc
        return out
    a1 = layer(np.concatenate([hi, lo]), np.vstack([W1, W1]), b1)
    h1 = _bf16(np.maximum(a1, 0.0))
    a2 = layer(h1, W2, b2)
    h2 = _bf16(np.maximum(a2, 0.0))
    return layer(h2, W3, b3)


def test_device_precision_forward_within_its_bound():
    import torch  # noqa: F401
    rng = np.random.default_rng(11)
    worst = 0.0
    for case in range(12):
        p = rng.normal(0.0, 0.08, O.mlp_nparam()).astype(np.float32)
        p[-1] = -3.0
        # the device's weight matrices are BF16
        for a, b in ((OFF_W1, OFF_B1), (OFF_W2, OFF_B2), (OFF_W3, OFF_B3)):
            p[a:b] = _bf16(p[a:b])
        p64 = p.astype(np.float64)
        z = np.concatenate([rng.uniform(0, 1, 1), rng.uniform(-6, 8, 1), rng.normal(0, 0.5, 4)])
        z = z.astype(np.float32).astype(np.float64)
        out, bound = O.mlp_forward_device(p64, z)
        ref = contract_forward_torch(p64, z, rng)
        _, loose = O.mlp_forward_bound(p64, z)
        assert np.all(np.abs(out - ref) <= bound), (case, out, ref, bound)
        assert np.all(bound < 0.05 * loose), (bound, loose)
        worst = max(worst, float(np.max(np.abs(out - ref) / np.maximum(bound, 1e-300))))
        fp64, _, _ = O.mlp_forward(p64, z)
        # BF16 activations move the outputs, by about the loose first-order bound
        assert np.all(np.abs(out - fp64) <= loose)
    print(f"worst |device model - torch contract| / bound = {worst:.3f}")


def test_device_precision_forward_exact_case():
    """Dyadic weights and features that BF16 and FP32 hold exactly: every
    rounding is the identity, so the device-precision pass equals the FP64
    definition and its bound only carries the feature-error allowance."""
    # the contract keeps biases in FP32
    p = asymmetric_net(history=True).astype(np.float32).astype(np.float64)
    z = [0.5, 0.25, 0.125, -0.25, 0.0, 0.0]
    out, bound = O.mlp_forward_device(p, z, np.zeros(6))
    ref, _, _ = O.mlp_forward(p, z)
    assert np.array_equal(out, ref)
    assert np.all(bound < 1e-5)
