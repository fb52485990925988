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


def test_features_affine_endpoints_and_midpoint():
    """Each parameter column maps affinely onto [-1, 1]: its lower bound to
    -1, its upper bound to +1 and the midpoint to 0."""
    lo = np.array([2e-3, 1.0, -0.26, 3e6])
    hi = np.array([60e-3, 3.0, 0.26, 10e6])
    f = mlp.features(np.stack([lo, hi, 0.5 * (lo + hi), lo + 0.25 * (hi - lo)]), lo, hi)
    assert np.array_equal(f[0], -np.ones(4))
    assert np.array_equal(f[1], np.ones(4))
    assert np.max(np.abs(f[2])) < 1e-15
    assert np.max(np.abs(f[3] + 0.5)) < 1e-15


def test_kernel_scale_closed_form_hann_sums_and_floor():
    """max(sum_n w(-x_n, z), 1) with the Hann aperture of half width
    a = z / (2F): the weights at known element offsets are closed forms."""
    p, F = 0.3e-3, 1.5
    at = lambda a: a * 2 * F          # depth whose aperture half width is a
    # 3 elements at 0, +-p, a = 2p: 1 + 2 * 0.5 (1 + cos(pi/2)) = 2
    assert abs(mlp.kernel_scale(at(2 * p), F, 3, p) - 2.0) < 1e-14
    # 4 elements at +-p/2, +-3p/2, a = 3p: 2 (0.5 (1 + cos(pi/6)) + 0.5 (1 + cos(pi/2))) = 2 + sqrt(3)/2
    assert abs(mlp.kernel_scale(at(3 * p), F, 4, p) - (2.0 + math.sqrt(3) / 2)) < 1e-14
    # 5 elements, a = 4p: 1 + 2 (0.5 (1 + cos(pi/4))) + 2 (0.5 (1 + cos(pi/2))) = 3 + sqrt(2)/2
    assert abs(mlp.kernel_scale(at(4 * p), F, 5, p) - (3.0 + math.sqrt(2) / 2)) < 1e-14
    # floor: 2 elements at +-p/2 with a = 3p/4 weigh 2 * 0.5 (1 + cos(2 pi / 3)) = 0.5 -> 1
    assert mlp.kernel_scale(at(0.75 * p), F, 2, p) == 1.0
    # empty aperture (z = 0, or elements outside it) -> 1
    assert mlp.kernel_scale(0.0, F, 4, p) == 1.0
    assert mlp.kernel_scale(at(0.4 * p), F, 2, p) == 1.0


def test_bf16_backward_one_hidden_unit_by_hand():
    """y = W2 G(W1 x + b1) + b2, one sample, one hidden unit, one output,
    loss (y - t)^2.  With bf16 rounding points the backward pass rounds the
    back-propagated gradient before each weight-gradient product (and the
    product with W2); the bias gradients take it unrounded.  Every operand
    below is exact in bf16 except g = 2 (y - t) and G(u)."""
    W1 = np.array([[0.5, -1.0]])
    b1 = np.array([0.25])
    W2 = np.array([[1.5]])
    b2 = np.array([-0.5])
    x = np.array([[1.0, 0.125]])
    t = np.array([[-0.3]])
    params = [(W1, b1), (W2, b2)]
    y, cache = mlp.forward(params, x, bf16_mode=True)
    grads = mlp.backward(cache, y, t, bf16_mode=True)
    u = 0.5 * 1.0 - 1.0 * 0.125 + 0.25
    h = mlp.bf16(0.5 * u * (1 + math.erf(u / math.sqrt(2))))
    yy = 1.5 * h - 0.5
    g = 2.0 * (yy - (-0.3))
    gr = mlp.bf16(g)
    assert gr != g                                  # the rounding is visible here
    assert abs(grads[1][0][0, 0] - gr * h) < 1e-15 * abs(gr * h)
    assert abs(grads[1][1][0] - g) < 1e-15
    gp = 0.5 * (1 + math.erf(u / math.sqrt(2))) + u / math.sqrt(2 * math.pi) * math.exp(-0.5 * u * u)
    g1 = gr * 1.5 * gp
    g1r = mlp.bf16(g1)
    assert abs(grads[0][0][0, 0] - g1r * 1.0) < 1e-15 * abs(g1r)
    assert abs(grads[0][0][0, 1] - g1r * 0.125) < 1e-15 * abs(g1r)
    assert abs(grads[0][1][0] - g1) < 1e-15 * abs(g1)


def test_bf16_backward_within_bf16_bound_of_fp64_differences():
    """The bf16-mode gradient approximates the exact gradient of the bf16
    forward: against FP64 central differences of the FP64 loss its error is
    of the order of the bf16 unit roundoff (2^-8) per rounding point."""
    params = small_net(2, (4, 32, 32, 32, 7))
    x = generators.uniform((16, 4), -1, 1, seed=7)
    t = generators.normal((16, 7), seed=8)
    y, cache = mlp.forward(params, x, bf16_mode=False)
    g64 = mlp.backward(cache, y, t, bf16_mode=False)
    yb, cb = mlp.forward(params, x, bf16_mode=True)
    g16 = mlp.backward(cb, yb, t, bf16_mode=True)
    for (dW, db), (eW, eb) in zip(g16, g64):
        rel = np.linalg.norm(dW - eW) / np.linalg.norm(eW)
        assert 1e-4 < rel < 8 * 2.0 ** -8
        relb = np.linalg.norm(db - eb) / np.linalg.norm(eb)
        assert relb < 8 * 2.0 ** -8


def test_adam_two_steps_closed_form():
    """Two steps from zero moments: the bias-corrected moments are the
    weighted means m = (b1 g1 + g2) / (1 + b1) and v = (b2 g1^2 + g2^2) /
    (1 + b2); a constant gradient therefore takes two equal steps."""
    b1, b2, lr, eps = 0.9, 0.999, 1e-3, 1e-8
    W = generators.normal((3, 4), seed=1)
    b = generators.normal(3, seed=2)
    g1W, g1b = generators.normal((3, 4), seed=3), generators.normal(3, seed=4)
    g2W, g2b = generators.normal((3, 4), seed=5), generators.normal(3, seed=6)
    st = [(np.zeros_like(W), np.zeros_like(W), np.zeros_like(b), np.zeros_like(b))]
    p1, s1 = mlp.adam_step([(W, b)], [(g1W, g1b)], st, lr, 1)
    p2, _ = mlp.adam_step(p1, [(g2W, g2b)], s1, lr, 2)
    for P0, G1, G2, P2 in ((W, g1W, g2W, p2[0][0]), (b, g1b, g2b, p2[0][1])):
        first = P0 - lr * G1 / (np.abs(G1) + eps)
        m = (b1 * G1 + G2) / (1 + b1)
        v = (b2 * G1 * G1 + G2 * G2) / (1 + b2)
        assert np.max(np.abs(P2 - (first - lr * m / (np.sqrt(v) + eps)))) < 1e-15
    # a constant gradient: both steps are lr * g / (|g| + eps)
    pc, sc = mlp.adam_step([(W, b)], [(g1W, g1b)], st, lr, 1)
    pc, _ = mlp.adam_step(pc, [(g1W, g1b)], sc, lr, 2)
    assert np.max(np.abs(pc[0][0] - (W - 2 * lr * g1W / (np.abs(g1W) + eps)))) < 1e-15
