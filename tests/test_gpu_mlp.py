"""The surrogate's BF16-MFMA kernels against the CPU FP64 oracle run with
the same bfloat16 rounding points: forward outputs, gradients, Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from paper_2509_26361_amd import ebit as E
from paper_2509_26361_amd import inputs as I

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_bf16_rows(X):
    """(m, 20) float64 -> (m, 32) bfloat16 rows on the device (zero padded)."""
    m = X.shape[0]
    P = np.zeros((m, 32), dtype=np.float32)
    P[:, :20] = X
    return torch.from_numpy(P).to(dev()).to(torch.bfloat16)


def theta32(seed):
    th = I.mlp_init(seed)
    return th, torch.from_numpy(th.astype(np.float32)).to(dev())


@pytest.mark.parametrize("m", [1, 17, 1000, 4099])
def test_forward_matches_oracle(m):
    rng = np.random.default_rng(m)
    th, tg = theta32(1)
    X = np.concatenate([rng.uniform(0, 1, size=(m, 12)), rng.integers(0, 2, size=(m, 8))], axis=1)
    y = E.mlp_forward(tg, to_bf16_rows(X)).cpu().numpy()
    yo = M.forward(th.astype(np.float32).astype(np.float64), X, bf16_mode=True)
    assert np.max(np.abs(y - yo)) < 2e-3, np.max(np.abs(y - yo))
    assert np.mean(np.abs(y - yo)) < 2e-4


def _abs_terms(th, X, c):
    """For every gradient entry, the sum of the absolute values of the terms
    the kernel adds (the bf16-mode oracle's products with every factor made
    non-negative): the scale of the entry's rounding error."""
    p = M.unpack(th)
    y, t = M.forward(th, X, bf16_mode=True, keep=True)
    m = X.shape[0]
    dz3 = np.abs((2.0 / m) * (y - c) * y * (1.0 - y))
    g = {}
    g["w3"] = np.abs(t["h2"]).T @ dz3
    g["b3"] = np.array([dz3.sum()])
    dz2 = np.outer(dz3, np.abs(p["w3"])) * (t["z2"] > 0)
    g["b2"] = dz2.sum(axis=0)
    dz2r = M.bf16(dz2)
    g["W2"] = np.abs(t["h1r"]).T @ dz2r
    dh1 = dz2r @ np.abs(t["W2"]).T
    dz1 = dh1 * (t["z1"] > 0)
    g["b1"] = dz1.sum(axis=0)
    g["W1"] = np.abs(t["X"]).T @ M.bf16(dz1)
    return M.pack(g)


@pytest.mark.parametrize("m", [64, 333, 5000])
def test_gradient_matches_oracle(m):
    """Element by element against the oracle evaluated with the kernels'
    bfloat16 rounding points: each entry within 2^-6 of the sum of the
    absolute values of its terms (a bfloat16 rounding that goes the other
    way in one term moves the entry by at most 2^-8 of that term; FP32
    accumulation adds m 2^-24), and 99.9 % of the entries within 2^-10."""
    rng = np.random.default_rng(m + 7)
    th, tg = theta32(2)
    th = th.astype(np.float32).astype(np.float64)
    X = np.concatenate([rng.uniform(0, 1, size=(m, 12)), rng.integers(0, 2, size=(m, 8))], axis=1)
    c = rng.uniform(0, 1, size=m)
    tr = E.MlpTrainer(tg, dev())
    g, loss = tr.gradient(to_bf16_rows(X), torch.from_numpy(c.astype(np.float32)).to(dev()))
    lo, go = M.loss_and_grad(th, X, c, bf16_mode=True)
    g = g.cpu().numpy().astype(np.float64)
    scale = _abs_terms(th, X, c) + 1e-30
    r = np.abs(g - go) / scale
    o = 0
    for name, shp in M.SIZES:
        k = int(np.prod(shp))
        assert r[o:o + k].max() <= 2.0 ** -6, (name, float(r[o:o + k].max()))
        o += k
    assert np.quantile(r, 0.999) <= 2.0 ** -10, float(np.quantile(r, 0.999))
    assert abs(float(loss.item()) - lo) < 1e-4 * max(1.0, lo)


def test_gradient_is_deterministic():
    rng = np.random.default_rng(3)
    _, tg = theta32(3)
    X = to_bf16_rows(rng.uniform(0, 1, size=(3000, 20)))
    c = torch.from_numpy(rng.uniform(0, 1, 3000).astype(np.float32)).to(dev())
    tr = E.MlpTrainer(tg, dev())
    g1 = tr.gradient(X, c)[0].clone()
    g2 = tr.gradient(X, c)[0].clone()
    assert torch.equal(g1, g2)


def test_adam_matches_oracle_and_training_reduces_loss():
    rng = np.random.default_rng(5)
    th, tg = theta32(4)
    m = 2048
    X = np.concatenate([rng.uniform(0, 1, size=(m, 12)), rng.integers(0, 2, size=(m, 8))], axis=1)
    c = 1.0 / (1.0 + np.exp(-(X[:, :12].sum(axis=1) - 6.0)))        # a smooth target
    xb = to_bf16_rows(X)
    cg = torch.from_numpy(c.astype(np.float32)).to(dev())
    tr = E.MlpTrainer(tg, dev())
    g = tr.gradient(xb, cg)[0].cpu().numpy().astype(np.float64)
    th0 = tg.cpu().numpy().astype(np.float64)
    opt = M.Adam(len(th0), lr=1e-3)
    want = opt.step(th0, g)
    tr.t = 1
    E.lib().ebit_mlp_adam(E._ptr(tr.theta), E._ptr(tr.m1), E._ptr(tr.m2), E._ptr(tr.grad), 1, 1e-3, E._stream())
    got = tr.theta.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - want)) < 1e-6
    losses = [float(tr.step(xb, cg, 1e-3).item()) for _ in range(300)]
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])


def test_native_training_loop_equals_step_by_step():
    """ebit_mlp_train (gather inside the gradient kernel, reduction fused with
    Adam, weights image updated in place) against gradient + Adam calls on
    rows gathered by torch: parameters, moments and losses bit for bit, over
    steps with repeated rows and a ragged last gradient group."""
    rng = np.random.default_rng(11)
    _, tg = theta32(6)
    m, batch, steps = 3000, 520, 7
    X = to_bf16_rows(np.concatenate([rng.uniform(0, 1, size=(m, 12)), rng.integers(0, 2, size=(m, 8))], axis=1))
    c = torch.from_numpy(rng.uniform(0, 1, m).astype(np.float32)).to(dev())
    idx = torch.from_numpy(rng.integers(0, m, size=steps * batch)).to(dev())
    lrs = [1e-3 * (1.0 + 0.1 * s) for s in range(steps)]
    a = E.MlpTrainer(tg.clone(), dev())
    b = E.MlpTrainer(tg.clone(), dev())
    la = a.train(X, c, idx, lrs).cpu().numpy()
    lb = []
    for s in range(steps):
        rows = idx[s * batch:(s + 1) * batch]
        lb.append(float(b.step(X.index_select(0, rows), c.index_select(0, rows), lrs[s]).item()))
    torch.cuda.synchronize()
    assert a.t == b.t == steps
    assert torch.equal(a.theta, b.theta)
    assert torch.equal(a.m1, b.m1) and torch.equal(a.m2, b.m2)
    assert np.array_equal(la, np.array(lb, dtype=np.float32))
    # a second call continues from the same state (step count, image rebuilt)
    la2 = a.train(X, c, idx[:2 * batch].contiguous(), lrs[:2]).cpu().numpy()
    for s in range(2):
        rows = idx[s * batch:(s + 1) * batch]
        assert float(b.step(X.index_select(0, rows), c.index_select(0, rows), lrs[s]).item()) == la2[s]
    assert torch.equal(a.theta, b.theta)


def test_native_training_loop_rejects_bad_indices():
    _, tg = theta32(7)
    X = to_bf16_rows(np.zeros((100, 20)))
    c = torch.zeros(100, dtype=torch.float32, device=dev())
    tr = E.MlpTrainer(tg.clone(), dev())
    for bad in (torch.tensor([0, 100], device=dev()), torch.tensor([-1, 3], device=dev()),
                torch.tensor([0, 1, 2], device=dev())):
        with pytest.raises(ValueError):
            tr.train(X, c, bad, [1e-3, 1e-3])
    assert torch.equal(tr.theta, tg)
