"""ebit_mlp_gradient_static (work space in the library's static device
array, no allocation) against ebit_mlp_gradient (caller's work space): the
same gradient and loss bit for bit, on two calls in a row, the second with
fewer rows, so the second reads an array the first left filled."""
import numpy as np
import pytest
import torch

from paper_2509_26361_amd import ebit as E
from paper_2509_26361_amd import inputs as I

pytestmark = pytest.mark.gpu


def _rows(rng, m, dev):
    P = np.zeros((m, 32), dtype=np.float32)
    P[:, :12] = rng.uniform(0, 1, size=(m, 12))
    P[:, 12:20] = rng.integers(0, 2, size=(m, 8))
    x = torch.from_numpy(P).to(dev).to(torch.bfloat16)
    c = torch.from_numpy(rng.uniform(0, 1, m).astype(np.float32)).to(dev)
    return x, c


def test_static_gradient_equals_allocating_gradient():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(21)
    theta = torch.from_numpy(I.mlp_init(5).astype(np.float32)).to(dev)
    tr = E.MlpTrainer(theta, dev)
    npar = E.mlp_param_count()
    for m in (E.EBIT_MLP_STATIC_MAX_ROWS, 1337):
        x, c = _rows(rng, m, dev)
        g_ref, l_ref = tr.gradient(x, c)
        g_ref, l_ref = g_ref.clone(), l_ref.clone()
        g = torch.full((npar,), float("nan"), dtype=torch.float32, device=dev)
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
        E.mlp_gradient_static(theta, x, c, g, loss)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), (m, float((g - g_ref).abs().max()))
        assert torch.equal(loss, l_ref), (m, float(loss), float(l_ref))


def test_static_gradient_rejects_too_many_rows():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    theta = torch.zeros(E.mlp_param_count(), dtype=torch.float32, device=dev)
    x = torch.zeros((E.EBIT_MLP_STATIC_MAX_ROWS + 1, 32), dtype=torch.bfloat16, device=dev)
    c = torch.zeros(E.EBIT_MLP_STATIC_MAX_ROWS + 1, dtype=torch.float32, device=dev)
    g = torch.zeros_like(theta)
    with pytest.raises(E.EbitError) as ei:
        E.mlp_gradient_static(theta, x, c, g)
    assert ei.value.code == E.EBIT_ETOOBIG
