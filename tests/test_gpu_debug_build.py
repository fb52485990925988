"""The debug build (libtidas_debug.so, -DTIDAS_DEBUG): the kernels' device-side
checks stay silent on valid inputs, and the non-finite input check fires when
a NaN or an infinity is planted in an input (it flows through as in the
release build; no kernel traps), in the line model and in DAS read frame by
frame and through the interleaved copy.  The study's check tests its
echo-support table on every skipped read."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2507_15464_amd as td  # noqa: E402
from paper_2507_15464_amd import _lib  # noqa: E402
from workloads import config, generators  # noqa: E402
from workloads.configs import Setup  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dbg():
    """The package's entry points bound to the debug library for this module."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    lib = _lib.load(_lib.DEBUG_LIB_PATH)
    saved = _lib.load()
    _lib._lib = lib
    try:
        yield lib
    finally:
        _lib._lib = saved


def flags(lib, reset=True):
    v = ctypes.c_uint32(0)
    _lib.check(lib.tidas_debug_flags(ctypes.byref(v), 1 if reset else 0))
    return v.value


def g(x, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).cuda()


def speckle_rf(s, n_frames, seed0):
    rf = torch.empty((n_frames, len(s.angles), s.n_elem, s.n_samples), device="cuda")
    for b in range(n_frames):
        x, z, a = generators.point_scatterers(60, s.field_w, s.field_d, seed=seed0 + b)
        td.simulate_rf(s, g(np.stack([x, z, a], 1), np.float64), out=rf[b])
    return rf


def test_nonfinite_inputs_are_flagged(dbg):
    s = config(1).with_grid(256, 64)
    kb = td.build_kernels(s, K=65, mode="exact")
    R = g(generators.normal((4, s.nz, s.nx), seed=1))
    flags(dbg)
    td.apply(kb, R)
    td.adjoint(td.prepare(kb), R)
    td.das_beamform(speckle_rf(s, 1, 800), s)
    rf8 = speckle_rf(s, 8, 810)
    td.das_beamform(rf8, s)  # eight frames: the interleaved copy
    assert flags(dbg) == 0
    R[2, 100, 10] = float("nan")
    td.apply(td.prepare(kb), R)
    assert flags(dbg) & _lib.DBG_NONFINITE_IN
    rf = speckle_rf(s, 1, 801)
    rf[0, 0, 32, 800] = float("inf")  # a centre channel inside the imaged depths
    td.das_beamform(rf, s)
    assert flags(dbg) & _lib.DBG_NONFINITE_IN
    rf8[5, 0, 32, 800] = float("inf")
    td.das_beamform(rf8, s)
    assert flags(dbg) & _lib.DBG_NONFINITE_IN
    assert flags(dbg) == 0  # reset by the previous query


def test_study_support_table_holds(dbg):
    flags(dbg)
    s = Setup(n_elem=33, pitch=0.3e-3, c=1540.0, fs=40e6, t0=0.0, fc=5e6, cycles=2.0, n_samples=1400,
              angles=(0.0,), fnumber=1.0, nz=1, nx=1, z0=0.0, dz=1.0, x0=0.0, dx=1.0, K=1, field_w=1.0, field_d=1.0)
    P, z_step = 12, 2.0e-3
    Ql = int(np.ceil((P - 1) * z_step / (s.c / (2 * s.fs))))
    td.point_study(s, 9, P, 6e-3, z_step, 5, Ql, stats_half=150)
    assert flags(dbg) == 0
