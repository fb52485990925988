"""GPU parity of the line model's gradient in its kernels (tidas_kernel_grad)
against the FP64 oracle, and of the autograd function that uses it.
Floating-point bar: relative L2 <= 1e-5."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2507_15464_amd as td  # noqa: E402
from oracle import tidas as o_t  # noqa: E402
from workloads import generators  # noqa: E402

pytestmark = pytest.mark.gpu
RTOL = 1e-5


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def g(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


# (B, Z, X, K): single pixel, ragged rows and columns (Z not a multiple of
# 128, X not of 32), one and several band tiles, two band passes (K = 193,
# 257), taps reaching past the image (K > 2 Z - 1), many frames
KGRAD_SHAPES = [(1, 1, 1, 1), (1, 1, 5, 3), (1, 40, 7, 5), (2, 130, 33, 65), (3, 257, 65, 129),
                (2, 300, 50, 161), (1, 200, 40, 193), (1, 150, 9, 257), (1, 64, 3, 321), (4, 128, 256, 129),
                (17, 96, 31, 33),
                # X % 4 == 0 (the split-bfloat16 kernel): one band tile (K = 1), the largest
                # band rows of one pass (K = 161, six tiles), taps past the image (K > 2 Z - 1)
                (1, 64, 8, 161), (1, 40, 4, 1), (1, 32, 12, 129)]


@pytest.mark.parametrize("B,Z,X,K", KGRAD_SHAPES)
def test_kernel_grad_matches_oracle(dev, B, Z, X, K):
    R = generators.normal((B, Z, X), seed=Z + 3 * X + B).astype(np.float32)
    Yb = generators.normal((B, Z, X), seed=Z + 5 * X + K).astype(np.float32)
    G = td.kernel_grad(g(R, dev), g(Yb, dev), K).cpu().numpy()
    ref = o_t.kernel_grad(R, Yb, K)
    assert G.shape == (Z, K)
    assert rel(G, ref) <= RTOL
    # taps whose source row leaves the image are exactly zero
    h = (K - 1) // 2
    for i in (0, Z - 1):
        for m in range(-h, h + 1):
            if not 0 <= i - m < Z:
                assert G[i, m + h] == 0.0


def test_kernel_grad_path_choice_and_float32_fallback(dev):
    """Frames readable 16 bytes at a time run the split-bfloat16 kernel; a view
    one float into its storage (rows not 16-byte aligned) runs the float32
    kernel, and both agree with the oracle."""
    B, Z, X, K = 2, 96, 32, 65
    R = generators.normal((B, Z, X), seed=60).astype(np.float32)
    Yb = generators.normal((B, Z, X), seed=61).astype(np.float32)
    ref = o_t.kernel_grad(R, Yb, K)
    Rd, Yd = g(R, dev), g(Yb, dev)
    assert td.kernel_grad_kernel(Rd, Yd) == td._lib.KGRAD_SPLIT_BF16
    G_split = td.kernel_grad(Rd, Yd, K).cpu().numpy()
    assert rel(G_split, ref) <= RTOL
    flat = torch.zeros(B * Z * X + 1, device=dev, dtype=torch.float32)
    Ro = flat[1:].view(B, Z, X)
    Ro.copy_(Rd)
    assert Ro.data_ptr() % 16 != 0
    assert td.kernel_grad_kernel(Ro, Yd) == td._lib.KGRAD_FP32
    G_f32 = td.kernel_grad(Ro, Yd, K).cpu().numpy()
    assert rel(G_f32, ref) <= RTOL
    # X not a multiple of 4 also takes the float32 kernel
    assert td.kernel_grad_kernel(Rd[..., :30].contiguous(), Yd[..., :30].contiguous()) == td._lib.KGRAD_FP32


def test_kernel_grad_two_dimensional_input(dev):
    Z, X, K = 70, 20, 31
    R = generators.normal((Z, X), seed=1).astype(np.float32)
    Yb = generators.normal((Z, X), seed=2).astype(np.float32)
    G = td.kernel_grad(g(R, dev), g(Yb, dev), K).cpu().numpy()
    assert rel(G, o_t.kernel_grad(R, Yb, K)) <= RTOL


def test_kernel_grad_full_size_sampled_and_reproducible(dev):
    """64 frames of 1024 x 256 with 129 taps: 400 sampled entries against FP64
    dot products, and a second call bit-identical to the first."""
    B, Z, X, K = 64, 1024, 256, 129
    R = generators.normal((B, Z, X), seed=31).astype(np.float32)
    Yb = generators.normal((B, Z, X), seed=32).astype(np.float32)
    Rd, Yd = g(R, dev), g(Yb, dev)
    G = td.kernel_grad(Rd, Yd, K)
    G2 = td.kernel_grad(Rd, Yd, K)
    assert torch.equal(G, G2)
    Gh = G.cpu().numpy()
    h = (K - 1) // 2
    rng = np.random.default_rng(33)
    got, want = [], []
    for _ in range(400):
        i = int(rng.integers(Z))
        m = int(rng.integers(-h, h + 1))
        s = i - m
        exp = float(np.sum(Yb[:, i, :].astype(np.float64) * R[:, s, :].astype(np.float64))) if 0 <= s < Z else 0.0
        got.append(Gh[i, m + h])
        want.append(exp)
    assert rel(got, want) <= RTOL


def test_autograd_gradients_of_reflectivity_and_kernels(dev):
    """loss = 1/2 ||A_K R - y||^2: R.grad = A^T res and K.grad = the kernel
    gradient of res, both against the oracle."""
    B, Z, X, K = 2, 160, 48, 65
    kb = (generators.normal((Z, K), seed=40) * 0.1).astype(np.float32)
    R = generators.normal((B, Z, X), seed=41).astype(np.float32)
    y = generators.normal((B, Z, X), seed=42).astype(np.float32)
    Kt = g(kb, dev).requires_grad_(True)
    Rt = g(R, dev).requires_grad_(True)
    res = td.tidas(Rt, Kt) - g(y, dev)
    (0.5 * (res * res).sum()).backward()
    res_o = o_t.apply(kb, R) - y
    assert rel(Rt.grad.cpu().numpy(), o_t.adjoint(kb, res_o)) <= RTOL
    assert rel(Kt.grad.cpu().numpy(), o_t.kernel_grad(R, res_o, K)) <= RTOL


def test_autograd_kernels_only_and_prepared_bank(dev):
    B, Z, X, K = 1, 130, 64, 33
    kb = generators.normal((Z, K), seed=50).astype(np.float32)
    R = generators.normal((B, Z, X), seed=51).astype(np.float32)
    w = generators.normal((B, Z, X), seed=52).astype(np.float32)
    Kt = g(kb, dev).requires_grad_(True)
    (td.tidas(g(R, dev), Kt) * g(w, dev)).sum().backward()
    assert rel(Kt.grad.cpu().numpy(), o_t.kernel_grad(R, w, K)) <= RTOL
    # a prepared bank is a constant: the map still gets its gradient
    Rt = g(R, dev).requires_grad_(True)
    (td.tidas(Rt, td.prepare(g(kb, dev))) * g(w, dev)).sum().backward()
    assert rel(Rt.grad.cpu().numpy(), o_t.adjoint(kb, w)) <= RTOL
