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


def _hand_network(shift):
    """A hand-set network whose output has a closed form: hidden unit j of
    the first layer copies input k(j) = j mod 20 minus 1/2 (so ReLU cuts),
    the second layer sends unit j to unit (j + shift) mod 128 (a permutation
    that is not its own transpose), the last layer weighs unit j by
    w(j) = (j - 64) / 64 and adds 1/4.  Every value is a short dyadic
    fraction, exact in bfloat16."""
    W1 = np.zeros((M.NIN, M.NH))
    for j in range(M.NH):
        W1[j % M.NIN, j] = 1.0
    b1 = np.full(M.NH, -0.5)
    W2 = np.zeros((M.NH, M.NH))
    for j in range(M.NH):
        W2[j, (j + shift) % M.NH] = 1.0
    b2 = np.zeros(M.NH)
    w3 = (np.arange(M.NH) - 64) / 64.0
    b3 = np.array([0.25])
    return M.pack(dict(W1=W1, b1=b1, W2=W2, b2=b2, w3=w3, b3=b3))


def _hand_output(X, shift):
    """The closed form of _hand_network: unit (j + shift) of the second layer
    holds max(x_{j mod 20} - 1/2, 0)."""
    z = np.full(X.shape[0], 0.25)
    for j in range(M.NH):
        z += ((j + shift) % M.NH - 64) / 64.0 * np.maximum(X[:, j % M.NIN] - 0.5, 0.0)
    return 1.0 / (1.0 + np.exp(-z))


def test_forward_of_a_hand_set_network_has_its_closed_form():
    """Pins the layer order, the orientation of W1 (in x out) and W2 (a
    transposed W2 moves units the other way), biases, ReLU and sigmoid; in
    bfloat16 mode too, since every operand is exact there."""
    rng = np.random.default_rng(9)
    X = np.floor(rng.uniform(0, 1, size=(40, M.NIN)) * 256) / 256     # exact in bfloat16
    X[:, 12:] = rng.integers(0, 2, size=(40, 8))
    for shift in (1, 37):
        th = _hand_network(shift)
        want = _hand_output(X, shift)
        assert np.max(np.abs(M.forward(th, X) - want)) < 1e-15
        assert np.max(np.abs(M.forward(th, X, bf16_mode=True) - want)) < 1e-15
        # the transposed second layer would give the other shift
        assert np.max(np.abs(_hand_output(X, -shift) - want)) > 1e-2


def test_gradient_of_a_hand_set_network_on_one_row():
    """Backward pass on one row against the chain rule written out for the
    hand-set network: dL/db3 = 2 (y - c) y (1 - y); dL/dw3_j = that times
    h2_j; dL/db1_j = that times w3 at unit (j + shift) when x_{j mod 20}
    > 1/2, else 0."""
    shift = 5
    th = _hand_network(shift)
    x = np.array([[0.75, 0.25, 0.5625, 0.125] * 3 + [1, 0, 1, 1, 0, 0, 1, 0]], dtype=np.float64)
    c = np.array([0.3])
    loss, g = M.loss_and_grad(th, x, c)
    y = _hand_output(x, shift)[0]
    dz3 = 2.0 * (y - 0.3) * y * (1.0 - y)
    p = M.unpack(g)
    assert abs(loss - (y - 0.3) ** 2) < 1e-15
    assert abs(p["b3"][0] - dz3) < 1e-15
    h1 = np.maximum(x[0, np.arange(M.NH) % M.NIN] - 0.5, 0.0)
    h2 = np.zeros(M.NH)
    h2[(np.arange(M.NH) + shift) % M.NH] = h1
    assert np.max(np.abs(p["w3"] - dz3 * h2)) < 1e-15
    w3 = (np.arange(M.NH) - 64) / 64.0
    want_b1 = np.where(x[0, np.arange(M.NH) % M.NIN] > 0.5, dz3 * w3[(np.arange(M.NH) + shift) % M.NH], 0.0)
    assert np.max(np.abs(p["b1"] - want_b1)) < 1e-15
