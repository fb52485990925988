"""The allocation-free forward operator (tidas_apply_noalloc) through the C
ABI against tidas_apply: bit-identical results on two calls in a row (the
second smaller, on the other split-bfloat16 tile), a call whose band images
exceed the library's scratch array rejected before anything is written, and
a shape outside the split tiles (no scratch needed)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2507_15464_amd import _lib  # noqa: E402
from workloads import generators  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _case(dev, B, Z, X, K, seed):
    kb = torch.from_numpy(generators.normal((Z, K), seed=seed).astype(np.float32)).to(dev)
    R = torch.from_numpy(generators.normal((B, Z, X), seed=seed + 1).astype(np.float32)).to(dev)
    return kb, R


def _both(lib, kb, R, K):
    B, Z, X = R.shape
    ref = torch.empty_like(R)
    got = torch.full_like(R, float("nan"))
    assert lib.tidas_apply(_p(kb), K, _p(R), B, Z, X, _p(ref), _stream()) == 0
    assert lib.tidas_apply_noalloc(_p(kb), K, _p(R), B, Z, X, _p(got), _stream()) == 0
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_equals_apply_on_two_calls_in_a_row(dev):
    lib = _lib.load()
    print("no-alloc: 64 x 1024 x 256, K 129 (four-block tile)", flush=True)
    kb, R = _case(dev, 64, 1024, 256, 129, 5)
    assert lib.tidas_line_kernel(129, 64, 1024, 256) == _lib.LINE_FOUR_BLOCK
    ref, got = _both(lib, kb, R, 129)
    assert torch.equal(ref, got)
    print("no-alloc: 3 x 300 x 100, K 65 (two-block tile)", flush=True)
    kb2, R2 = _case(dev, 3, 300, 100, 65, 7)
    assert lib.tidas_line_kernel(65, 3, 300, 100) == _lib.LINE_TWO_BLOCK
    ref2, got2 = _both(lib, kb2, R2, 65)
    assert torch.equal(ref2, got2)


def test_noalloc_rejects_banks_beyond_its_scratch(dev):
    lib = _lib.load()
    Z, K = 20000, 129     # two-block images of one mode: about 23 MB
    kb = torch.zeros((Z, K), device=dev, dtype=torch.float32)
    R = torch.zeros((1, Z, 8), device=dev, dtype=torch.float32)
    out = torch.full_like(R, 7.0)
    assert lib.tidas_apply_noalloc(_p(kb), K, _p(R), 1, Z, 8, _p(out), _stream()) == _lib.TIDAS_EUNSUPPORTED
    assert b"scratch" in lib.tidas_last_error()
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())


def test_noalloc_outside_the_split_tiles(dev):
    lib = _lib.load()
    print("no-alloc: 2 x 300 x 40, K 401 (float32 matrix kernel)", flush=True)
    kb, R = _case(dev, 2, 300, 40, 401, 11)
    assert lib.tidas_line_kernel(401, 2, 300, 40) not in (_lib.LINE_FOUR_BLOCK, _lib.LINE_TWO_BLOCK)
    ref, got = _both(lib, kb, R, 401)
    assert torch.equal(ref, got)
