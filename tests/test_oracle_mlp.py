"""Pins of the surrogate's CPU oracle: gradients against central finite
differences, Adam's first step against its closed form, degenerate networks,
feature extraction on a hand-made cell, bfloat16 rounding."""
import numpy as np

from oracle import mlp_oracle as M
from oracle import oracle as O
from tests.ebit_states import make_state


def rand_theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(scale=scale, size=M.NPARAM)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    th = rand_theta(2)
    X = rng.uniform(0, 1, size=(9, M.NIN))
    c = rng.uniform(0, 1, size=9)
    _, g = M.loss_and_grad(th, X, c)
    idx = np.concatenate([rng.choice(M.NPARAM - 129, 150, replace=False), np.arange(M.NPARAM - 129, M.NPARAM)])
    h = 1e-6
    for i in idx:
        tp = th.copy(); tp[i] += h
        tm = th.copy(); tm[i] -= h
        fd = (M.loss_and_grad(tp, X, c)[0] - M.loss_and_grad(tm, X, c)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_adam_first_step_closed_form():
    """First step: m_hat = g, v_hat = g^2, so each parameter moves by
    -lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    opt = M.Adam(50, lr=0.01)
    th1 = opt.step(th, g)
    assert np.allclose(th1, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_zero_network_outputs_sigmoid_of_bias():
    th = np.zeros(M.NPARAM)
    th[-1] = 0.7
    X = np.random.default_rng(0).uniform(size=(5, M.NIN))
    assert np.allclose(M.forward(th, X), 1 / (1 + np.exp(-0.7)))


def test_bf16_rounding_ties_to_even():
    one = 1.0
    assert M.bf16(one) == 1.0
    assert M.bf16(1 + 2 ** -8) == 1.0                      # tie, even neighbour
    assert M.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6          # tie, round up to even
    assert M.bf16(1 + 2 ** -8 + 2 ** -12) == 1 + 2 ** -7   # above the tie
    assert M.bf16(-2.5) == -2.5


def test_features_of_a_corner_cell():
    n = 8
    col = np.zeros((n, n, n), np.uint8)
    col[4, 4, 4] = 1
    rng = np.random.default_rng(4)
    s = [rng.uniform(0.1, 0.9, size=(n, n, n)) for _ in range(3)]
    st = make_state(col, s)
    q = 4 + n * (4 + n * 4)                # cell whose corner (0,0,0) is the phase-1 node
    X = M.cell_features(st.flags, st.s, [q])[0]
    want = np.zeros(20)
    want[0] = s[0][4, 4, 4]                # x-edge from the corner
    want[4] = s[1][4, 4, 4]                # y-edge
    want[8] = s[2][4, 4, 4]                # z-edge
    want[12] = 1.0                         # corner 0 colour
    assert np.array_equal(X, want)
    C, _ = O.f2v(st)
    assert abs(C[4, 4, 4] - want[0] * want[4] * want[8] / 6) < 1e-15
