"""DAS through the frame-interleaved copy (one plane wave, eight or more
frames: das_interleave_kernel, then das_kernel reading four frames per 16-byte
load) against the FP64 oracle frame by frame, including a last group of fewer
than four frames and reads at both ends of the record; the caller's workspace
and the library's own scratch give the same bits."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2507_15464_amd as td  # noqa: E402
from paper_2507_15464_amd import _lib  # noqa: E402
from paper_2507_15464_amd.api import _descs, _ptr, _stream  # noqa: E402
from oracle import das as o_das, simulate as o_sim  # noqa: E402
from workloads import config, generators  # noqa: E402
from tests.helpers import axes, das_kw, sim_kw  # noqa: E402

pytestmark = pytest.mark.gpu
RTOL = 1e-5
NUL = ctypes.c_void_p(0)


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


def point_frames(s, B, seed0):
    frames = []
    for b in range(B):
        x, z, a = generators.point_scatterers(20, s.field_w, s.field_d, seed=seed0 + b)
        frames.append(o_sim.to_fp32(o_sim.simulate_rf(x, z, a, **sim_kw(s))))
    return np.stack(frames)


@pytest.mark.parametrize("B", [8, 10, 13])
def test_interleaved_frames_match_oracle(dev, B):
    """Groups of four with a last group of 4, 2 and 1 frames."""
    s = config(1).with_grid(140, 72)
    assert _lib.load().das_beamform_workspace_bytes(1, s.n_elem, s.n_samples, B) > 0
    rf = point_frames(s, B, 300 + B)
    img = td.das_beamform(g(rf, dev), s).cpu().numpy()
    xs, zs = axes(s)
    for b in range(B):
        ref = o_das.das(rf[b], xs, zs, **das_kw(s))
        assert np.max(np.abs(img[b] - ref)) <= 1e-5 * np.max(np.abs(ref)), b
        assert rel(img[b], ref) <= RTOL, b


def test_interleaved_compounding_matches_oracle(dev):
    """Eleven compounded angles, nine frames (groups of 4, 4, 1)."""
    s = config(3).with_grid(160, 96)
    B = 9
    rf = point_frames(s, B, 600)
    assert rf.shape[1] == 11
    img = td.das_beamform(g(rf, dev), s).cpu().numpy()
    xs, zs = axes(s)
    for b in range(B):
        ref = o_das.das(rf[b], xs, zs, **das_kw(s))
        assert np.max(np.abs(img[b] - ref)) <= 1e-5 * np.max(np.abs(ref)), b
        assert rel(img[b], ref) <= RTOL, b


def test_interleaved_odd_record_and_unaligned_rf(dev):
    """A record of A C T samples not a multiple of four, and RF starting 4
    bytes past a 16-byte boundary: the copy takes its one-sample-per-thread
    form; same results as through an aligned copy of the same frames."""
    s = config(1).replace(n_elem=63, n_samples=1501).with_grid(90, 40)
    B = 9
    rf = point_frames(s, B, 500)
    img = td.das_beamform(g(rf, dev), s).cpu().numpy()
    xs, zs = axes(s)
    for b in range(B):
        ref = o_das.das(rf[b], xs, zs, **das_kw(s))
        assert rel(img[b], ref) <= RTOL, b
    s2 = config(1).with_grid(90, 40)
    rf2 = point_frames(s2, B, 510)
    flat = torch.zeros(rf2.size + 1, device=dev)
    flat[1:] = g(rf2.reshape(-1), dev)
    shifted = flat[1:].view(rf2.shape)
    assert shifted.data_ptr() % 16 == 4
    assert torch.equal(td.das_beamform(shifted, s2), td.das_beamform(g(rf2, dev), s2))


def test_interleaved_reads_at_both_ends_of_the_record(dev):
    """As the single-frame sweep: the depth axis takes the sample index from
    1.5 samples before the record to 1.5 after it, now for nine frames of
    different channel data read through the interleaved copy."""
    T = 64
    base = config(1).replace(n_elem=1, n_samples=T, angles=(0.0,))
    z_min = 2e-3
    t0 = 2 * z_min / base.c + 1.5 / base.fs
    nz = 500
    dz = (T + 3.0) / (nz - 1) * base.c / (2 * base.fs)
    s = base.replace(t0=t0, nz=nz, nx=1, z0=z_min, dz=dz, x0=0.0, dx=1e-4)
    rf = generators.normal((9, 1, 1, T), seed=17).astype(np.float32)
    img = td.das_beamform(g(rf, dev), s).cpu().numpy()
    xs, zs = axes(s)
    u = (2 * zs / s.c - s.t0) * s.fs
    edge = ((u > -1) & (u < 0)) | ((u > T - 1) & (u < T))
    assert edge.sum() > 10
    for b in range(9):
        ref = o_das.das(rf[b], xs, zs, **das_kw(s))
        assert np.max(np.abs(img[b] - ref)) <= 2e-6, b
        assert np.all(np.abs(img[b][edge, 0]) > 0), b


def test_interleaved_benchmark_workload_sampled(dev):
    """The benchmark's launch shape (64 frames of 128 x 4096 -> 1024 x 256):
    frames from the first, a middle and the last group against the oracle."""
    s = config(2)
    B = 64
    rf = torch.empty((B, 1, s.n_elem, s.n_samples), device=dev)
    want = {}
    for b in range(B):
        x, z, a = generators.point_scatterers(300, s.field_w, s.field_d, seed=900 + b)
        if b in (0, 34, 63):
            r = o_sim.to_fp32(o_sim.simulate_rf(x, z, a, **sim_kw(s)))
            rf[b] = g(r, dev)
            want[b] = r
        else:
            td.simulate_rf(s, torch.tensor(np.stack([x, z, a], 1), dtype=torch.float64, device=dev), out=rf[b])
    img = td.das_beamform(rf, s)
    xs, zs = axes(s)
    for b, r in want.items():
        ref = o_das.das(r, xs, zs, **das_kw(s))
        got = img[b].cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref)), b
        assert rel(got, ref) <= RTOL, b


def test_interleaved_own_scratch_same_bits(dev):
    s = config(1).with_grid(120, 64)
    B = 9
    rd = g(point_frames(s, B, 400), dev)
    want = td.das_beamform(rd, s)  # caller workspace from torch's allocator
    lib = _lib.load()
    got = torch.empty_like(want)
    arr, tx, rx, gd = _descs(s, s)
    _lib.check(lib.das_beamform(ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(gd), _ptr(rd),
                                s.n_samples, B, _ptr(got), NUL, 0, _stream()))
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    # and a workspace larger than the query, reused by a second call
    ws = torch.empty(lib.das_beamform_workspace_bytes(1, s.n_elem, s.n_samples, B) + 4096, dtype=torch.uint8,
                     device=dev)
    for _ in range(2):
        got.fill_(7.0)
        _lib.check(lib.das_beamform(ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(gd),
                                    _ptr(rd), s.n_samples, B, _ptr(got), _ptr(ws), ws.numel(), _stream()))
        torch.cuda.synchronize()
        assert torch.equal(got, want)


def test_fixed_delay_interleaved_own_scratch_same_bits(dev):
    """tidas_beamform reads eight or more frames through the same copy: the
    caller's workspace and the library's own scratch give the same bits."""
    s = config(1).with_grid(120, 64)
    B = 10
    rd = g(point_frames(s, B, 450), dev)
    refs = torch.from_numpy(np.minimum((np.arange(s.nz) // 16) * 16 + 8, s.nz - 1).astype(np.int32)).to(dev)
    theta = g(1.0 + 0.2 * generators.normal(s.nz, seed=3), dev)
    want = td.tidas_beamform(rd, s, ref_row=refs, theta=theta)
    lib = _lib.load()
    got = torch.empty_like(want)
    arr, tx, rx, gd = _descs(s, s)
    _lib.check(lib.tidas_beamform(ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(gd), _ptr(rd),
                                  s.n_samples, B, _ptr(refs), _ptr(theta), _ptr(got), NUL, 0, _stream()))
    torch.cuda.synchronize()
    assert torch.equal(got, want)
