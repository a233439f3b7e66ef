"""Pins of the oracle MLP: backprop against central finite differences (FP64),
softmax normalisation, Adam against its closed-form first step, the label
rule on hand-made masks, and the BF16 inference: the rounding on hand-worked
values and the forward pass on hand-made networks."""
import numpy as np

import workloads as W
from oracle import mlp


def _setup(K=4, B=32, seed=0):
    th = W.mlp_init_params(K, seed)
    rng = np.random.default_rng(seed + 1)
    X = rng.normal(size=(B, mlp.NF))
    y = rng.integers(0, K, size=B)
    th[-2 * mlp.NF:-mlp.NF] = rng.normal(size=mlp.NF) * 0.1      # mean
    th[-mlp.NF:] = rng.uniform(0.5, 2.0, size=mlp.NF)             # std
    return th, X, y


def test_backprop_matches_finite_differences():
    K = 4
    th, X, y = _setup(K)
    loss, g, _ = mlp.loss_and_grad(th, X, y, K)
    rng = np.random.default_rng(7)
    idx = rng.choice(len(th) - 2 * mlp.NF, size=60, replace=False)
    eps = 1e-6
    for i in idx:
        tp = th.copy(); tp[i] += eps
        tm = th.copy(); tm[i] -= eps
        fd = (mlp.loss_and_grad(tp, X, y, K)[0] - mlp.loss_and_grad(tm, X, y, K)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_softmax_rows_sum_to_one():
    th, X, y = _setup()
    _, p, _ = mlp.forward(th, X, 4)
    assert np.allclose(p.sum(1), 1.0, atol=1e-14)


def test_adam_first_step_is_signed_lr():
    th, X, y = _setup()
    _, g, _ = mlp.loss_and_grad(th, X, y, 4)
    th1, m, v = mlp.adam_step(th, g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    n = len(th) - 2 * mlp.NF
    d = th1[:n] - th[:n]
    nz = np.abs(g[:n]) > 1e-3
    assert np.allclose(d[nz], -1e-3 * np.sign(g[:n][nz]), rtol=1e-4)


def test_training_reduces_loss():
    th, X, y = _setup(B=256)
    m = np.zeros_like(th); v = np.zeros_like(th)
    l0 = mlp.loss_and_grad(th, X, y, 4)[0]
    for t in range(1, 200):
        _, g, _ = mlp.loss_and_grad(th, X, y, 4)
        th, m, v = mlp.adam_step(th, g, m, v, t, lr=3e-3)
    assert mlp.loss_and_grad(th, X, y, 4)[0] < 0.5 * l0


def test_label_rule():
    reps = np.array([[0, 0, 0], [1, 1, 0], [3, 3, 3]], np.uint8)
    sizes = [100, 60, 10]
    cells = np.array([[3, 3, 3], [1, 2, 0], [0, 3, 3], [2, 1, 1]], np.uint8)
    assert list(mlp.label_from_masks(cells, reps, sizes)) == [2, 1, 0, 1]


def test_bf16_round_known_values():
    # spacing 2^-7 just above 1: halfway cases go to the even significand
    cases = [(1.0, 1.0),
             (1.0 + 2.0 ** -8, 1.0),
             (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),
             (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),
             (np.pi, 3.140625),
             (-0.1, -0.10009765625),
             (0.0, 0.0)]
    x = np.array([c[0] for c in cases])
    assert np.array_equal(mlp.bf16_round(x), np.array([c[1] for c in cases]))


def _tiny_net(K, H, rng):
    """Integer weights, biases and inputs: every value on the way is a small
    integer, exact in bfloat16."""
    th = np.zeros(mlp.n_params(K, H))
    o = 0
    for rows, cols in ((H, mlp.NF), (H, H), (K, H)):
        th[o:o + rows * cols] = rng.integers(-1, 2, size=rows * cols)
        o += rows * cols
        th[o:o + rows] = rng.integers(-2, 3, size=rows)
        o += rows
    th[o + mlp.NF:] = 1.0                     # mean 0, std 1
    return th


def test_bf16_forward_is_exact_on_representable_values():
    rng = np.random.default_rng(3)
    K, H = 4, 8
    th = _tiny_net(K, H, rng)
    X = rng.integers(-3, 4, size=(50, mlp.NF)).astype(np.float64)
    z, p, _ = mlp.forward(th, X, K, H)
    zb, pb = mlp.forward_bf16(th, X, K, H)
    assert np.max(np.abs(z)) < 256           # integers below 2^8: exact in bfloat16
    assert np.array_equal(z, zb) and np.array_equal(p, pb)


def test_bf16_forward_rounds_weights_and_activations():
    K, H = 2, 8
    base = np.zeros(mlp.n_params(K, H))
    o_w2 = H * mlp.NF + H
    o_w3 = o_w2 + H * H + H
    base[-mlp.NF:] = 1.0
    base[o_w2] = 1.0                          # W2[0][0]
    base[o_w3] = 1.0                          # W3[0][0]
    x = np.zeros((1, mlp.NF))
    # a weight of 1 + 2^-8 is a tie in bfloat16 and rounds to 1
    th = base.copy()
    th[0] = 1.0 + 2.0 ** -8                   # W1[0][0]
    x[0, 0] = 1.0
    assert mlp.forward(th, x, K, H)[0][0, 0] == 1.0 + 2.0 ** -8
    assert mlp.forward_bf16(th, x, K, H)[0][0, 0] == 1.0
    # exact weights whose sum 1 + 2^-8 is rounded as an activation
    th = base.copy()
    th[0], th[1] = 1.0, 2.0 ** -8             # W1[0][0], W1[0][1]
    x[0, :2] = 1.0
    assert mlp.forward(th, x, K, H)[0][0, 0] == 1.0 + 2.0 ** -8
    assert mlp.forward_bf16(th, x, K, H)[0][0, 0] == 1.0
