"""GPU training kernels of the learned proposal network against the FP64
oracle: the minibatch gradient computed with BF16 MFMA (FP32 accumulate)
must match the oracle's FP64 gradient on the same BF16-rounded weights, and
training must reduce the loss and learn a feature-dependent scale."""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2408_00018_amd import sa
    sa.load_library()
    return sa


def records(n, seed):
    rng = np.random.default_rng(seed)
    z = np.column_stack([rng.uniform(0, 1, n), rng.uniform(-4, 3, n), rng.normal(0, 0.05, (n, 4))])
    d = rng.normal(0, 0.05, n)
    return np.column_stack([z, d]).astype(np.float32)


@pytest.mark.parametrize("batch", [32, 256, 1024])
def test_gradient_matches_oracle(S, batch):
    import torch
    rng = np.random.default_rng(batch)
    p = rng.normal(0, 0.15, S.MLP_PARAMS).astype(np.float32)
    rec = records(4096, seed=batch + 1)
    idx = rng.choice(4096, batch, replace=False).astype(np.uint32)
    say(f"[gpu mlp] gradient batch={batch}")
    tr = S.MLPTrainer(max_batch=1024)
    tr.set_params(p)
    g, loss = tr.grad(torch.from_numpy(rec).cuda(), idx)
    tr.close()
    # oracle on the same BF16-rounded weight matrices (biases FP32) and FP32 inputs
    q = p.astype(np.float64)
    H, I = 128, 6
    w1 = slice(0, I * H)
    w2 = slice(I * H + H, I * H + H + H * H)
    w3 = slice(I * H + 2 * H + H * H, I * H + 2 * H + H * H + 2 * H)
    for sl in (w1, w2, w3):
        q[sl] = S.bf16_round(p[sl]).astype(np.float64)
    sel = rec[idx].astype(np.float64)
    lref, gref = O.mlp_loss_grad(q, sel[:, :6], sel[:, 6])
    # The device rounds hidden activations (and the layer-2 gradient) to BF16,
    # unit roundoff u = 2^-9, so each gradient term carries a relative error of
    # a few u; a relu unit whose pre-activation lies within rounding distance of
    # 0 can switch sides, which moves single entries of small batches far more
    # than their norm.  Hence normwise bounds per parameter block (8u) and a
    # median elementwise bound (2u) rather than an elementwise maximum.
    u = 2.0 ** -9
    assert abs(loss - lref) <= 2e-3 * max(1.0, abs(lref)), (loss, lref)
    cos = float(np.dot(g, gref) / (np.linalg.norm(g) * np.linalg.norm(gref)))
    big = np.abs(gref) > 1e-2 * np.max(np.abs(gref))
    rel = np.abs(g[big] - gref[big]) / np.abs(gref[big])
    blocks = {"W1": w1, "b1": slice(I * H, I * H + H), "W2": w2, "b2": slice(I * H + H + H * H, I * H + 2 * H + H * H),
              "W3": w3, "b3": slice(w3.stop, w3.stop + 2)}
    normwise = {k: float(np.linalg.norm(g[sl] - gref[sl]) / np.linalg.norm(gref[sl])) for k, sl in blocks.items()}
    say(f"[gpu mlp] batch={batch} loss {loss:.6f} vs {lref:.6f} cosine {cos:.6f} median rel {np.median(rel):.3e} "
        f"normwise {{{', '.join(f'{k}: {v:.2e}' for k, v in normwise.items())}}}")
    assert cos >= 0.9999
    for k, v in normwise.items():
        assert v <= 8 * u, (k, v)
    assert np.median(rel) <= 2 * u


def test_training_reduces_loss_and_learns_scale(S):
    import torch
    rng = np.random.default_rng(21)
    n = 8192
    z = np.column_stack([rng.uniform(0, 1, n), np.zeros(n), np.zeros((n, 4))])
    sig = np.where(z[:, 0] < 0.5, 0.01, 0.1)
    d = rng.normal(0, 1, n) * sig
    rec = torch.from_numpy(np.column_stack([z, d]).astype(np.float32)).cuda()
    p0 = rng.normal(0, 0.05, S.MLP_PARAMS).astype(np.float32)
    tr = S.MLPTrainer(max_batch=512)
    tr.set_params(p0)
    trace = tr.train(rec, batch=512, steps=400, lr=3e-3, seed=5)
    p = tr.params()
    tr.close()
    say(f"[gpu mlp] loss {trace[:5].mean():.4f} -> {trace[-20:].mean():.4f}")
    assert trace[-20:].mean() < trace[:5].mean() - 1.0
    s_lo = O.mlp_forward(p.astype(np.float64), [0.25, 0, 0, 0, 0, 0])[0][1]
    s_hi = O.mlp_forward(p.astype(np.float64), [0.75, 0, 0, 0, 0, 0])[0][1]
    assert s_hi - s_lo > 1.0
