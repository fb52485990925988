"""Device scratch of the entry points that need it: a caller workspace sized
by the entry point's query (what the Python binding passes, from torch's
allocator) and the library's own stream-ordered scratch (workspace NULL, 0
bytes, called here through the C ABI) give the same bits.  The kernel build
in paper mode, which no longer waits for the stream, is checked on a stream
that is still busy with earlier work, and with its host reference map
overwritten as soon as the call returns."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2507_15464_amd as td  # noqa: E402
from paper_2507_15464_amd import _lib  # noqa: E402
from paper_2507_15464_amd.api import _descs, _ptr, _stream  # noqa: E402
from workloads import config, generators  # noqa: E402

pytestmark = pytest.mark.gpu
NUL = ctypes.c_void_p(0)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


@pytest.mark.parametrize("mode", ["paper", "line"])
def test_build_kernels_own_scratch_same_bits(dev, mode):
    s = config(1).with_grid(96, 8)
    refs = np.minimum((np.arange(s.nz) // 16) * 16 + 8, s.nz - 1).astype(np.int32)
    kb, th = td.build_kernels(s, K=33, mode=mode, ref_row=refs, with_theta=True)
    lib = _lib.load()
    kb2 = torch.empty_like(kb)
    th2 = torch.empty_like(th)
    arr, tx, rx, g = _descs(s, s)
    ref = (ctypes.c_int32 * s.nz)(*refs.tolist())
    m = _lib.MODE_PAPER if mode == "paper" else _lib.MODE_LINE
    _lib.check(lib.tidas_build_kernels(ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(g),
                                       s.n_samples, 33, m, ref, _ptr(kb2), _ptr(th2), NUL, 0, _stream()))
    torch.cuda.synchronize()
    assert torch.equal(kb, kb2) and torch.equal(th, th2)


def test_build_kernels_does_not_depend_on_the_host_map_after_return(dev):
    """The call returns without waiting for the stream: a long launch queued
    before it keeps the stream busy, and the caller's reference map is
    overwritten right after the call returns; the bank is still the one of the
    map passed in."""
    s = config(1).with_grid(64, 8)
    refs = np.full(s.nz, 20, np.int32)
    want, _ = td.build_kernels(s, K=33, mode="paper", ref_row=refs, with_theta=True)
    torch.cuda.synchronize()
    lib = _lib.load()
    busy = torch.randn((4096, 4096), device=dev)
    for _ in range(8):
        busy = busy @ busy * 1e-3  # queued ahead of the build on the same stream
    got = torch.empty_like(want)
    th = torch.empty(s.nz, device=dev)
    ws = torch.empty(lib.tidas_build_kernels_workspace_bytes(s.nz, 33, _lib.MODE_PAPER), dtype=torch.uint8,
                     device=dev)
    arr, tx, rx, g = _descs(s, s)
    ref = (ctypes.c_int32 * s.nz)(*refs.tolist())
    _lib.check(lib.tidas_build_kernels(ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(g),
                                       s.n_samples, 33, _lib.MODE_PAPER, ref, _ptr(got), _ptr(th), _ptr(ws),
                                       ws.numel(), _stream()))
    for i in range(s.nz):
        ref[i] = 50
    torch.cuda.synchronize()
    assert torch.equal(got, want)


def test_simulate_own_scratch_same_bits(dev):
    s = config(1)
    x, z, a = generators.point_scatterers(40, s.field_w, s.field_d, seed=5)
    scat = torch.tensor(np.stack([x, z, a], 1), dtype=torch.float64, device=dev)
    rf = td.simulate_rf(s, scat)
    lib = _lib.load()
    rf2 = torch.empty_like(rf)
    arr, tx, _, _ = _descs(s)
    _lib.check(lib.tidas_simulate_rf(ctypes.byref(arr), ctypes.byref(tx), _ptr(scat), scat.shape[0], s.n_samples,
                                     _ptr(rf2), NUL, 0, _stream()))
    torch.cuda.synchronize()
    assert torch.equal(rf, rf2)


def test_kernel_grad_own_scratch_same_bits(dev):
    B, Z, X, K = 3, 200, 64, 33
    R = torch.from_numpy(generators.normal((B, Z, X), seed=1).astype(np.float32)).to(dev)
    Y = torch.from_numpy(generators.normal((B, Z, X), seed=2).astype(np.float32)).to(dev)
    G = td.kernel_grad(R, Y, K)
    lib = _lib.load()
    G2 = torch.empty_like(G)
    _lib.check(lib.tidas_kernel_grad(K, _ptr(R), _ptr(Y), B, Z, X, _ptr(G2), NUL, 0, _stream()))
    torch.cuda.synchronize()
    assert torch.equal(G, G2)


@pytest.mark.parametrize("K", [17, 65])
def test_deconvolve_and_norm_own_scratch_same_bits(dev, K):
    """K = 17 takes two iterations per launch (N^2 fits the tile), K = 65 one."""
    Z, X = 128, 64
    kb = torch.from_numpy((0.1 * generators.normal((Z, K), seed=3)).astype(np.float32)).to(dev)
    y = torch.from_numpy(generators.normal((1, Z, X), seed=4).astype(np.float32)).to(dev)
    nrm = td.operator_norm_sq(kb, iters=20)
    lib = _lib.load()
    work = torch.empty(3 * Z + 4, device=dev)
    out = ctypes.c_double(0.0)
    _lib.check(lib.tidas_operator_norm_sq(_ptr(kb), K, Z, 20, _ptr(work), ctypes.byref(out), NUL, 0, _stream()))
    assert out.value == nrm
    eta = 1.0 / (nrm + 1e-2)
    r = td.deconvolve(kb, y, 1e-2, eta=eta, iters=7)
    r2 = torch.empty_like(y)
    w2 = torch.empty_like(y)
    _lib.check(lib.tidas_deconvolve(_ptr(kb), K, _ptr(y), 1, Z, X, ctypes.c_float(1e-2), ctypes.c_float(eta), 7,
                                    _ptr(r2), _ptr(w2), NUL, 0, _stream()))
    torch.cuda.synchronize()
    assert torch.equal(r.view(1, Z, X), r2)
