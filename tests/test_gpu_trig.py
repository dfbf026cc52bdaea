"""Error of the gfx950 FP32 transcendental instructions the kernels use
(v_sin_f32 and v_cos_f32 on revolutions, v_sqrt_f32, v_exp_f32, v_log_f32),
of the FP32 e^x - 1 of the Ackley increment and of the FP32 GELU of the
Gaussian proposal network built on them, measured against FP64 evaluations
of the same FP32 inputs.

The per-move tolerances of the FP32 parity tests take the sine/cosine error
as an absolute bound (parity_util.E_TRIG, for arguments up to 64
revolutions, and E_TRIG_WIDE up to 256 revolutions, which Griewank's
cos(y_i / sqrt(i)) reaches) and the square root and 2^t errors as relative
bounds (E_SQRT, E_EXP2).  These tests check that the hardware stays within
them over the argument ranges the kernels use, and print the measured
maxima.
"""
import ctypes
import math
import os
import sys

import numpy as np
import pytest
from scipy import special

import oracle as O
import parity_util as P

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def probe():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2408_00018_amd", "libsa_peak.so"))
    lib.sa_peak_accuracy.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]
    lib.sa_peak_accuracy.restype = ctypes.c_int

    def run(op, x):
        xin = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
        out = torch.empty_like(xin)
        torch.cuda.synchronize()
        rc = lib.sa_peak_accuracy(op, xin.data_ptr(), out.data_ptr(), xin.numel())
        assert rc == 0, rc
        return out.cpu().numpy().astype(np.float64)
    return run


def rev_samples(bound, count, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-bound, bound, count).astype(np.float32)
    # quarter and eighth revolutions, where the result is 0, +-1 or +-sqrt(1/2)
    k = np.arange(-8 * int(bound), 8 * int(bound) + 1, dtype=np.float64) / 8.0
    return np.concatenate([x, k.astype(np.float32)])


def sin_cos_ref(t):
    frac = t - np.round(t)  # exact in FP64 for FP32 inputs
    return np.sin(2 * np.pi * frac), np.cos(2 * np.pi * frac)


@pytest.mark.parametrize("bound,limit_name", [(1.0, "E_TRIG"), (8.0, "E_TRIG"), (64.0, "E_TRIG"),
                                              (256.0, "E_TRIG_WIDE")])
def test_sin_cos_absolute_error(probe, bound, limit_name):
    t = rev_samples(bound, 1 << 21, int(bound))
    ref_s, ref_c = sin_cos_ref(t.astype(np.float64))
    es = np.max(np.abs(probe(0, t) - ref_s))
    ec = np.max(np.abs(probe(1, t) - ref_c))
    limit = getattr(P, limit_name)
    say(f"[trig] |t| <= {bound} rev: max |sin err| = {es:.3e}, max |cos err| = {ec:.3e} "
        f"({es / 2 ** -24:.2f}, {ec / 2 ** -24:.2f} x 2^-24); {limit_name} = {limit:.3e}")
    assert es <= limit and ec <= limit


def test_sqrt_relative_error(probe):
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(0, 1, 1 << 20), rng.uniform(0, 30, 1 << 20),
                        np.exp(rng.uniform(-40, 10, 1 << 20))]).astype(np.float32)
    x = x[x > 0]
    ref = np.sqrt(x.astype(np.float64))
    err = np.max(np.abs(probe(2, x) - ref) / ref)
    say(f"[trig] sqrt: max relative error {err:.3e} ({err / 2 ** -24:.2f} x 2^-24); E_SQRT = {P.E_SQRT:.3e}")
    assert err <= P.E_SQRT


def test_exp2_relative_error(probe):
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.uniform(-30, 24, 1 << 21), rng.uniform(-1, 1, 1 << 20)]).astype(np.float32)
    ref = np.exp2(x.astype(np.float64))
    err = np.max(np.abs(probe(3, x) - ref) / ref)
    say(f"[trig] exp2: max relative error {err:.3e} ({err / 2 ** -24:.2f} x 2^-24); E_EXP2 = {P.E_EXP2:.3e}")
    assert err <= P.E_EXP2
    assert math.isfinite(err)


def test_expm1_relative_error(probe):
    """The Ackley increment's e^x - 1: polynomial for |x| <= 1/2, hardware
    exponential minus one beyond; relative error against FP64 expm1 over the
    arguments the increment takes (|x| up to ~7 for the Gaussian-term
    exponent at small n, tiny ones near the end of a run)."""
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.uniform(-0.5, 0.5, 1 << 20), rng.uniform(-8, 3, 1 << 20),
                        np.sign(rng.uniform(-1, 1, 1 << 18)) * np.exp(rng.uniform(-40, -1, 1 << 18))])
    x = x.astype(np.float32)
    x = x[x != 0]
    ref = np.expm1(x.astype(np.float64))
    rel = np.abs(probe(4, x) - ref) / np.abs(ref)
    small = np.abs(x) <= 0.5
    es, el = rel[small].max(), rel[~small].max()
    say(f"[trig] expm1_f32: max relative error {es:.3e} (|x| <= 1/2, {es / 2 ** -24:.2f} x 2^-24), "
        f"{el:.3e} beyond ({el / 2 ** -24:.2f} x 2^-24); E_EXPM1 = {P.E_EXPM1:.3e}")
    assert es <= P.E_EXPM1 and el <= P.E_EXPM1


def test_log2_relative_error(probe):
    """v_log_f32 over (0, 1]: the Box-Muller radius of the Gaussian proposal
    takes log2(1 - U) for U on the 2^-24 grid, every one of which is tried
    (the results near 1 are tiny, so the error is taken relative)."""
    k = np.arange(1, 1 << 24, dtype=np.float64)
    x = (1.0 - k * 2.0 ** -24).astype(np.float32)
    rng = np.random.default_rng(8)
    x = np.concatenate([x, rng.uniform(1e-7, 1.0, 1 << 20).astype(np.float32)])
    ref = np.log2(x.astype(np.float64))
    err = np.max(np.abs(probe(7, x) - ref) / np.abs(ref))
    say(f"[trig] log2: max relative error {err:.3e} ({err / 2 ** -24:.2f} x 2^-24) over 1 - U and (0, 1); "
        f"E_LOG2 = {P.E_LOG2:.3e}")
    assert err <= P.E_LOG2


def test_rcp_relative_error(probe):
    """v_rcp_f32 over the arguments the centre families give it (d + c with
    c >= 0.1 and d up to a few thousand), log-uniform, and every FP32 value
    of one binade: within E_RCP relative."""
    rng = np.random.default_rng(9)
    x = np.exp(rng.uniform(np.log(0.05), np.log(4096.0), 1 << 22)).astype(np.float32)
    one = (1.0 + np.arange(1 << 23, dtype=np.float64) * 2.0 ** -23).astype(np.float32)
    x = np.concatenate([x, one])
    ref = 1.0 / x.astype(np.float64)
    err = np.max(np.abs(probe(8, x) - ref) / ref)
    say(f"[trig] rcp: max relative error {err:.3e} ({err / 2 ** -24:.2f} x 2^-24); E_RCP = {P.E_RCP:.3e}")
    assert err <= P.E_RCP


def test_gelu_within_the_oracle_device_bound(probe):
    """The device GELU (FP32, Abramowitz-Stegun 26.2.17 for the normal
    distribution function) against the exact x Phi(x) in FP64: within the
    deviation the oracle's device-precision network bound allows
    (|gelu(a)| 2^-20 + |a| 2^-22), over the pre-activations a network sees;
    its derivative within 2^-20 + 2^-22 |a| absolute."""
    rng = np.random.default_rng(9)
    a = np.concatenate([np.linspace(-12, 12, 1 << 20), rng.normal(0, 2, 1 << 20),
                        np.sign(rng.uniform(-1, 1, 1 << 16)) * np.exp(rng.uniform(-30, 2, 1 << 16))]).astype(np.float32)
    a64 = a.astype(np.float64)
    cdf = 0.5 * (1.0 + special.erf(a64 / math.sqrt(2.0)))
    ref = a64 * cdf
    dref = cdf + a64 * np.exp(-0.5 * a64 * a64) / math.sqrt(2.0 * math.pi)
    # the same allowance as the oracle's device-precision model, checked there
    O.set_net_kind(O.NET_GELU_GAUSS)
    try:
        assert all(abs(O.act(v) - r) <= 1e-15 * (1 + abs(r)) for v, r in zip(a64[::4099], ref[::4099]))
    finally:
        O.set_net_kind(O.NET_RELU_CAUCHY)
    err = np.abs(probe(5, a) - ref)
    allow = np.abs(ref) * 2.0 ** -20 + np.abs(a64) * 2.0 ** -22
    derr = np.abs(probe(6, a) - dref)
    dallow = 2.0 ** -20 + np.abs(a64) * 2.0 ** -22
    say(f"[trig] gelu: max err/allowance {np.max(err / allow):.3f}, max abs err {err.max():.3e}; "
        f"derivative max err/allowance {np.max(derr / dallow):.3f}")
    assert np.all(err <= allow)
    assert np.all(derr <= dallow)
