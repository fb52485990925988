"""Pins of the oracle's surrogate MLP: bf16 rounding (hand-written fixture and
torch's CPU conversion), a hand-computed one-hidden-unit network, zero
weights, finite-difference gradients and the Adam update."""
import math
import os

import numpy as np
import pytest

from oracle import mlp
from workloads import generators

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_bf16_golden_fixture():
    rows = np.loadtxt(os.path.join(GOLD, "bf16_rounding.txt"))
    for x, want in rows:
        assert mlp.bf16(x) == want, (x, want)


def test_bf16_matches_torch_cpu_conversion():
    torch = pytest.importorskip("torch")
    v = np.concatenate([generators.normal(20000, seed=1) * 10.0 ** generators.uniform(20000, -6, 6, seed=2),
                        [0.0, -0.0, 1e-38, 3.4e38]]).astype(np.float32)
    t = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(v), t)


def test_gelu_against_math_erf_and_its_derivative():
    for u in (-3.0, -0.7, 0.0, 0.3, 2.2):
        assert abs(mlp.gelu(u) - 0.5 * u * (1 + math.erf(u / math.sqrt(2)))) < 1e-15
        h = 1e-6
        fd = (mlp.gelu(u + h) - mlp.gelu(u - h)) / (2 * h)
        assert abs(fd - mlp.gelu_grad(u)) < 1e-9


def test_one_hidden_unit_hand_computed():
    """y = w2 * G(w1 . x + b1) + b2 with a single hidden unit."""
    W1 = np.array([[0.5, -1.0]])
    b1 = np.array([0.25])
    W2 = np.array([[2.0]])
    b2 = np.array([-0.5])
    x = np.array([[1.0, 0.125]])
    y, _ = mlp.forward([(W1, b1), (W2, b2)], x, bf16_mode=False)
    u = 0.5 * 1.0 - 1.0 * 0.125 + 0.25
    want = 2.0 * 0.5 * u * (1 + math.erf(u / math.sqrt(2))) - 0.5
    assert abs(y[0, 0] - want) < 1e-15
    # all these values are exact in bf16, so the bf16 path agrees except for G(u) rounding
    yb, _ = mlp.forward([(W1, b1), (W2, b2)], x, bf16_mode=True)
    g_b = mlp.bf16(0.5 * u * (1 + math.erf(u / math.sqrt(2))))
    assert abs(yb[0, 0] - (2.0 * g_b - 0.5)) < 1e-15


def test_zero_weights_give_bias():
    params = [(np.zeros((8, 4)), np.zeros(8)), (np.zeros((3, 8)), np.array([0.1, -2.0, 7.5]))]
    x = generators.normal((5, 4), seed=1)
    y, _ = mlp.forward(params, x, bf16_mode=True)
    assert np.all(y == np.array([0.1, -2.0, 7.5]))


def small_net(seed=0, widths=(4, 16, 16, 16, 9)):
    p = generators.mlp_init(widths, seed)
    return [(W, generators.normal(W.shape[0], seed=seed + 50 + l) * 0.1) for l, (W, _) in enumerate(p)]


def test_fp64_backward_matches_central_differences():
    params = small_net()
    x = generators.uniform((6, 4), -1, 1, seed=3)
    t = generators.normal((6, 9), seed=4)
    y, cache = mlp.forward(params, x, bf16_mode=False)
    grads = mlp.backward(cache, y, t, bf16_mode=False)
    eps = 1e-6
    rng = np.random.default_rng(0)
    for l, (W, b) in enumerate(params):
        for _ in range(6):
            i, j = rng.integers(W.shape[0]), rng.integers(W.shape[1])
            for sgn_store in [None]:
                Wp = [(w.copy(), bb.copy()) for w, bb in params]
                Wm = [(w.copy(), bb.copy()) for w, bb in params]
                Wp[l][0][i, j] += eps
                Wm[l][0][i, j] -= eps
                fp = mlp.loss(mlp.forward(Wp, x, False)[0], t)
                fm = mlp.loss(mlp.forward(Wm, x, False)[0], t)
                fd = (fp - fm) / (2 * eps)
                assert abs(fd - grads[l][0][i, j]) <= 1e-6 * max(1e-3, abs(fd))
        i = rng.integers(b.shape[0])
        Bp = [(w.copy(), bb.copy()) for w, bb in params]
        Bm = [(w.copy(), bb.copy()) for w, bb in params]
        Bp[l][1][i] += eps
        Bm[l][1][i] -= eps
        fd = (mlp.loss(mlp.forward(Bp, x, False)[0], t) - mlp.loss(mlp.forward(Bm, x, False)[0], t)) / (2 * eps)
        assert abs(fd - grads[l][1][i]) <= 1e-6 * max(1e-3, abs(fd))


def test_bf16_path_close_to_fp64():
    params = small_net(1, (4, 64, 64, 64, 33))
    x = generators.uniform((32, 4), -1, 1, seed=5)
    y64, _ = mlp.forward(params, x, bf16_mode=False)
    y16, _ = mlp.forward(params, x, bf16_mode=True)
    rel = np.linalg.norm(y16 - y64) / np.linalg.norm(y64)
    assert 1e-5 < rel < 3e-2


def test_adam_first_step_closed_form():
    """From zero moments the bias-corrected first step is lr * g / (|g| + eps)."""
    W = generators.normal((3, 4), seed=1)
    b = generators.normal(3, seed=2)
    dW = generators.normal((3, 4), seed=3)
    db = generators.normal(3, seed=4)
    st = [(np.zeros_like(W), np.zeros_like(W), np.zeros_like(b), np.zeros_like(b))]
    (W2, b2), = mlp.adam_step([(W, b)], [(dW, db)], st, 1e-3, 1)[0]
    assert np.allclose(W2, W - 1e-3 * dW / (np.abs(dW) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(b2, b - 1e-3 * db / (np.abs(db) + 1e-8), rtol=0, atol=1e-15)


def test_cosine_schedule_endpoints():
    assert mlp.cosine_lr(0, 100) == pytest.approx(1e-3, rel=1e-15)
    assert mlp.cosine_lr(100, 100) == pytest.approx(1e-5, rel=1e-12)
    assert mlp.cosine_lr(50, 100) == pytest.approx(0.5 * (1e-3 + 1e-5), rel=1e-12)
