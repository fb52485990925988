"""Host-side checks of the C ABI: the library loads, exports every function
include/tidas.h declares, and rejects invalid arguments before touching the
device (these calls never reach a kernel launch)."""
import ctypes
import os
import re

import pytest

from paper_2507_15464_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tidas.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libtidas.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_lists_the_entry_points():
    names = declared_functions()
    for n in ("das_beamform", "tidas_build_kernels", "tidas_apply", "tidas_adjoint", "tidas_simulate_rf",
              "tidas_last_error", "tidas_version"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    # and the binding knows every declared entry point
    assert set(declared_functions()) <= set(_lib.exported_symbols())


def test_version_string(lib):
    assert b"gfx950" in lib.tidas_version()


def test_debug_flags_in_the_release_and_debug_builds(lib):
    """The release library has no device checks: tidas_debug_flags answers
    EUNSUPPORTED with 0 flags; both builds export every declared symbol."""
    v = ctypes.c_uint32(7)
    assert lib.tidas_debug_flags(ctypes.byref(v), 0) == _lib.TIDAS_EUNSUPPORTED and v.value == 0
    assert lib.tidas_debug_flags(None, 0) == _lib.TIDAS_EINVAL
    if not os.path.exists(_lib.DEBUG_LIB_PATH):
        pytest.fail("libtidas_debug.so is not built (run __graft_entry__.build())")
    dbg = _lib.load(_lib.DEBUG_LIB_PATH)
    for name in declared_functions():
        assert hasattr(dbg, name), name
    assert dbg.tidas_debug_flags(None, 0) == _lib.TIDAS_EINVAL


def _geom():
    arr = _lib.make_array(64, 0.3e-3, 1540.0)
    tx = _lib.make_tx([0.0], 40e6, 0.0, 5e6, 2.0)
    rx = _lib.make_rx(1.5)
    g = _lib.make_grid(256, 128, 7.8e-5, 1.56e-4, -9.4e-3, 1.48e-4)
    return arr, tx, rx, g


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
NUL = ctypes.c_void_p(0)


def test_lateral_pass_rejects_invalid_arguments(lib):
    out = ctypes.c_void_p(0x2000)
    f = lib.tidas_apply_lateral
    assert f(NUL, 33, FAKE, 1, 16, 16, out, NUL) == _lib.TIDAS_EINVAL            # null kernels
    assert f(FAKE, 32, ctypes.c_void_p(0x3000), 1, 16, 16, out, NUL) == _lib.TIDAS_EINVAL  # even K
    assert f(FAKE, 33, ctypes.c_void_p(0x3000), 0, 16, 16, out, NUL) == _lib.TIDAS_EINVAL  # B = 0
    assert f(FAKE, 33, ctypes.c_void_p(0x3000), 1, 16, 16, ctypes.c_void_p(0x3000), NUL) == _lib.TIDAS_EINVAL
    assert f(FAKE, 1537, ctypes.c_void_p(0x3000), 1, 16, 16, out, NUL) == _lib.TIDAS_EUNSUPPORTED
    assert lib.tidas_last_error()


@pytest.mark.parametrize("args", [
    (NUL, 65, FAKE, 1, 16, 16, FAKE),       # null kernels
    (FAKE, 64, FAKE, 1, 16, 16, ctypes.c_void_p(0x2000)),  # even K
    (FAKE, 0, FAKE, 1, 16, 16, ctypes.c_void_p(0x2000)),   # K = 0
    (FAKE, 5, FAKE, 0, 16, 16, ctypes.c_void_p(0x2000)),   # B = 0
    (FAKE, 5, FAKE, 1, 0, 16, ctypes.c_void_p(0x2000)),    # Z = 0
    (FAKE, 5, FAKE, 1, 16, -3, ctypes.c_void_p(0x2000)),   # X < 0
    (FAKE, 5, ctypes.c_void_p(0x2000), 1, 16, 16, ctypes.c_void_p(0x2000)),  # output aliases input
])
def test_conv_rejects_invalid_arguments(lib, args):
    for fn in (lib.tidas_apply, lib.tidas_adjoint):
        assert fn(*args, NUL) == _lib.TIDAS_EINVAL
        assert lib.tidas_last_error()


def test_das_rejects_invalid_arguments(lib):
    arr, tx, rx, g = _geom()
    ok = (ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(g))
    assert lib.das_beamform(*ok, NUL, 2048, 1, FAKE, NUL, 0, NUL) == _lib.TIDAS_EINVAL
    assert lib.das_beamform(*ok, FAKE, 1, 1, ctypes.c_void_p(0x2000), NUL, 0, NUL) == _lib.TIDAS_EINVAL
    assert lib.das_beamform(*ok, FAKE, 2048, 0, ctypes.c_void_p(0x2000), NUL, 0, NUL) == _lib.TIDAS_EINVAL
    assert lib.das_beamform(*ok, FAKE, 2048, 1, FAKE, NUL, 0, NUL) == _lib.TIDAS_EINVAL  # aliasing
    for bad in (_lib.make_array(0, 0.3e-3, 1540.0), _lib.make_array(64, -1.0, 1540.0),
                _lib.make_array(64, 0.3e-3, 0.0)):
        assert lib.das_beamform(ctypes.byref(bad), *ok[1:], FAKE, 2048, 1, ctypes.c_void_p(0x2000), NUL, 0, NUL) == -1
    for badtx in (_lib.make_tx([], 40e6, 0, 5e6, 2), _lib.make_tx([0.0], 0.0, 0, 5e6, 2),
                  _lib.make_tx([2.0], 40e6, 0, 5e6, 2)):
        assert lib.das_beamform(ok[0], ctypes.byref(badtx), *ok[2:], FAKE, 2048, 1, ctypes.c_void_p(0x2000),
                                NUL, 0, NUL) == -1
    badrx = _lib.make_rx(0.0)
    assert lib.das_beamform(ok[0], ok[1], ctypes.byref(badrx), ok[3], FAKE, 2048, 1, ctypes.c_void_p(0x2000),
                            NUL, 0, NUL) == -1
    for badg in (_lib.make_grid(0, 4, 0, 1e-4, 0, 1e-4), _lib.make_grid(4, 4, 0, -1e-4, 0, 1e-4),
                 _lib.make_grid(4, 4, float("nan"), 1e-4, 0, 1e-4)):
        assert lib.das_beamform(*ok[:3], ctypes.byref(badg), FAKE, 2048, 1, ctypes.c_void_p(0x2000), NUL, 0, NUL) == -1
    tx33 = _lib.make_tx([0.0] * 33, 40e6, 0, 5e6, 2)
    assert lib.das_beamform(ok[0], ctypes.byref(tx33), *ok[2:], FAKE, 2048, 1, ctypes.c_void_p(0x2000),
                            NUL, 0, NUL) == _lib.TIDAS_EUNSUPPORTED
    # the interleaved copy's workspace (one angle, eight frames or more)
    img = ctypes.c_void_p(0x2000)
    assert lib.das_beamform(*ok, FAKE, 2048, 8, img, NUL, 64, NUL) == _lib.TIDAS_EINVAL  # bytes without a buffer
    need = lib.das_beamform_workspace_bytes(1, 64, 2048, 8)
    assert lib.das_beamform(*ok, FAKE, 2048, 8, img, ctypes.c_void_p(0x10040), need, NUL) == _lib.TIDAS_EINVAL
    assert lib.das_beamform(*ok, FAKE, 2048, 8, img, ctypes.c_void_p(0x10000), need - 256, NUL) == _lib.TIDAS_EINVAL


def test_das_workspace_query(lib):
    """Interleaved groups of four frames, 256-byte rounded; none below eight
    frames, for angle counts other than 1 and 11 (the fixed-delay beamformer:
    other than 1) or for invalid sizes."""
    assert lib.das_beamform_workspace_bytes(1, 64, 2048, 8) == 2 * 4 * 64 * 2048 * 4
    assert lib.das_beamform_workspace_bytes(1, 128, 4096, 64) == 64 * 128 * 4096 * 4
    assert lib.das_beamform_workspace_bytes(1, 3, 5, 9) == (3 * 4 * 3 * 5 * 4 + 255) // 256 * 256
    assert lib.das_beamform_workspace_bytes(1, 64, 2048, 7) == 0
    assert lib.das_beamform_workspace_bytes(11, 64, 2048, 8) == 2 * 4 * 11 * 64 * 2048 * 4  # the compounding
    assert lib.das_beamform_workspace_bytes(3, 64, 2048, 64) == 0
    assert lib.tidas_beamform_workspace_bytes(11, 64, 2048, 64) == 0
    assert lib.tidas_beamform_workspace_bytes(1, 64, 2048, 8) == 2 * 4 * 64 * 2048 * 4
    assert lib.das_beamform_workspace_bytes(1, 0, 2048, 64) == 0
    assert lib.das_beamform_workspace_bytes(1, 64, 1, 64) == 0


def test_fixed_delay_beamform_rejects_invalid_arguments(lib):
    arr, tx, rx, g = _geom()
    ok = (ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(g))
    img = ctypes.c_void_p(0x2000)
    f = lib.tidas_beamform
    assert f(*ok, NUL, 2048, 1, NUL, NUL, img, NUL, 0, NUL) == _lib.TIDAS_EINVAL           # null rf
    assert f(*ok, FAKE, 2048, 1, NUL, NUL, NUL, NUL, 0, NUL) == _lib.TIDAS_EINVAL          # null image
    assert f(*ok, FAKE, 1, 1, NUL, NUL, img, NUL, 0, NUL) == _lib.TIDAS_EINVAL             # n_samples < 2
    assert f(*ok, FAKE, 2048, 0, NUL, NUL, img, NUL, 0, NUL) == _lib.TIDAS_EINVAL          # no frames
    assert f(*ok, FAKE, 2048, 1, NUL, NUL, FAKE, NUL, 0, NUL) == _lib.TIDAS_EINVAL         # image aliases rf
    assert f(*ok, FAKE, 2048, 1, img, NUL, img, NUL, 0, NUL) == _lib.TIDAS_EINVAL          # image aliases ref_row
    assert f(*ok, FAKE, 2048, 1, NUL, img, img, NUL, 0, NUL) == _lib.TIDAS_EINVAL          # image aliases theta
    badrx = _lib.make_rx(0.0)
    assert f(ok[0], ok[1], ctypes.byref(badrx), ok[3], FAKE, 2048, 1, NUL, NUL, img, NUL, 0, NUL) == _lib.TIDAS_EINVAL
    tx33 = _lib.make_tx([0.0] * 33, 40e6, 0, 5e6, 2)
    assert f(ok[0], ctypes.byref(tx33), *ok[2:], FAKE, 2048, 1, NUL, NUL, img, NUL, 0, NUL) == _lib.TIDAS_EUNSUPPORTED
    # the interleaved copy's workspace (one angle, eight frames or more): same rules as DAS
    assert f(*ok, FAKE, 2048, 8, NUL, NUL, img, NUL, 64, NUL) == _lib.TIDAS_EINVAL
    need = lib.tidas_beamform_workspace_bytes(1, 64, 2048, 8)
    assert need == lib.das_beamform_workspace_bytes(1, 64, 2048, 8) > 0
    assert f(*ok, FAKE, 2048, 8, NUL, NUL, img, ctypes.c_void_p(0x10040), need, NUL) == _lib.TIDAS_EINVAL
    assert f(*ok, FAKE, 2048, 8, NUL, NUL, img, ctypes.c_void_p(0x10000), need - 256, NUL) == _lib.TIDAS_EINVAL
    assert lib.tidas_last_error()


def test_build_kernels_rejects_invalid_arguments(lib):
    arr, tx, rx, g = _geom()
    ok = (ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(g))
    assert lib.tidas_build_kernels(*ok, 2048, 65, 0, None, NUL, NUL, NUL, 0, NUL) == -1       # null kernels
    assert lib.tidas_build_kernels(*ok, 2048, 64, 0, None, FAKE, NUL, NUL, 0, NUL) == -1      # even K
    assert lib.tidas_build_kernels(*ok, 2048, 65, 7, None, FAKE, NUL, NUL, 0, NUL) == -1      # bad mode
    assert lib.tidas_build_kernels(*ok, 1, 65, 0, None, FAKE, NUL, NUL, 0, NUL) == -1         # n_samples
    assert lib.tidas_build_kernels(*ok, 2048, 65, 0, None, FAKE, FAKE, NUL, 0, NUL) == -1     # theta aliases
    bad_ref = (ctypes.c_int32 * 256)(*([0] * 255 + [256]))
    assert lib.tidas_build_kernels(*ok, 2048, 65, 1, bad_ref, FAKE, NUL, NUL, 0, NUL) == -1   # ref out of range
    nopulse = _lib.make_tx([0.0], 40e6, 0, 0.0, 2)
    assert lib.tidas_build_kernels(ok[0], ctypes.byref(nopulse), *ok[2:], 2048, 65, 0, None, FAKE, NUL, NUL, 0,
                                   NUL) == -1


def test_simulate_rejects_invalid_arguments(lib):
    arr, tx, _, _ = _geom()
    assert lib.tidas_simulate_rf(ctypes.byref(arr), ctypes.byref(tx), NUL, 5, 2048, FAKE, NUL, 0, NUL) == -1
    assert lib.tidas_simulate_rf(ctypes.byref(arr), ctypes.byref(tx), FAKE, -1, 2048, FAKE, NUL, 0, NUL) == -1
    assert lib.tidas_simulate_rf(ctypes.byref(arr), ctypes.byref(tx), FAKE, 5, 0, FAKE, NUL, 0, NUL) == -1
    assert lib.tidas_simulate_rf(ctypes.byref(arr), ctypes.byref(tx), FAKE, 5, 2048, NUL, NUL, 0, NUL) == -1


def test_workspace_queries_and_checks(lib):
    """Every entry point that needs device scratch sizes it through a query and
    takes it from the caller (or allocates it itself when given NULL, 0):
    a short, misaligned or size-without-pointer workspace is EINVAL before
    anything is enqueued."""
    Z, K = 256, 65
    # kernel build: paper and line modes only, sized for every row its own reference
    assert lib.tidas_build_kernels_workspace_bytes(Z, K, _lib.MODE_EXACT) == 0
    assert lib.tidas_build_kernels_workspace_bytes(Z, K, _lib.MODE_LATERAL) == 0
    need = lib.tidas_build_kernels_workspace_bytes(Z, K, _lib.MODE_PAPER)
    assert need == 8 * Z * K + 16 * Z + 16 == lib.tidas_build_kernels_workspace_bytes(Z, K, _lib.MODE_LINE)
    arr, tx, rx, g = _geom()
    ok = (ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(g))
    ws = ctypes.c_void_p(0x100000)
    assert lib.tidas_build_kernels(*ok, 2048, K, 1, None, FAKE, NUL, ws, need - 1, NUL) == -1      # short
    assert lib.tidas_build_kernels(*ok, 2048, K, 1, None, FAKE, NUL, ctypes.c_void_p(0x100080), need,
                                   NUL) == -1                                                     # misaligned
    assert lib.tidas_build_kernels(*ok, 2048, K, 1, None, FAKE, NUL, NUL, need, NUL) == -1         # bytes, no pointer
    assert lib.tidas_last_error()
    # RF synthesis: the fixed-point accumulator and its scale
    assert lib.tidas_simulate_rf_workspace_bytes(2, 64, 2048) == 8 * (2 * 64 * 2048 + 1)
    assert lib.tidas_simulate_rf_workspace_bytes(0, 64, 2048) == 0
    need = lib.tidas_simulate_rf_workspace_bytes(1, arr.n_elem, 2048)
    assert lib.tidas_simulate_rf(ctypes.byref(arr), ctypes.byref(tx), FAKE, 5, 2048, ctypes.c_void_p(0x8000),
                                 ws, need - 8, NUL) == -1
    # kernel gradient: partial-sum slices (a whole number of Z x K slices)
    need = lib.tidas_kernel_grad_workspace_bytes(K, 4, Z, 64)
    assert need > 0 and need % (4 * Z * K) == 0
    assert lib.tidas_kernel_grad_workspace_bytes(64, 4, Z, 64) == 0
    assert lib.tidas_kernel_grad(K, FAKE, ctypes.c_void_p(0x2000), 4, Z, 64, ctypes.c_void_p(0x3000), ws, need - 4,
                                 NUL) == -1
    # deconvolution: step operators, band images, c and c2 (at least two frames)
    need = lib.tidas_deconvolve_workspace_bytes(K, 1, Z, 64)
    assert need >= 2 * 4 * Z * 64
    f = ctypes.c_float
    assert lib.tidas_deconvolve(FAKE, K, ctypes.c_void_p(0x4000), 1, Z, 64, f(1e-3), f(0.1), 10,
                                ctypes.c_void_p(0x3000), ctypes.c_void_p(0x2000), ws, need - 1, NUL) == -1
    # power iteration: the band images
    need = lib.tidas_operator_norm_sq_workspace_bytes(K, Z)
    assert need > 0 and lib.tidas_operator_norm_sq_workspace_bytes(K, 0) == 0
    out = ctypes.c_double(0)
    assert lib.tidas_operator_norm_sq(FAKE, K, Z, 10, ctypes.c_void_p(0x2000), ctypes.byref(out), ws, need - 1,
                                      NUL) == -1


def test_python_api_refuses_host_tensors():
    """The product path has no CPU fallback: host tensors are rejected."""
    torch = pytest.importorskip("torch")
    import paper_2507_15464_amd as td
    kb = torch.zeros((8, 3))
    x = torch.zeros((8, 4))
    for fn in (td.apply, td.adjoint):
        with pytest.raises(ValueError):
            fn(kb, x)
    with pytest.raises(ValueError):
        td.apply_ex(kb, x)
    with pytest.raises(ValueError):
        td.deconvolve(kb, x, 1e-3, eta=0.1)


def test_deconvolve_and_norm_reject_invalid_arguments(lib):
    ok = ctypes.c_void_p(0x1000)
    w = ctypes.c_void_p(0x2000)
    r = ctypes.c_void_p(0x3000)
    y = ctypes.c_void_p(0x4000)
    f = ctypes.c_float
    assert lib.tidas_deconvolve(ok, 65, y, 1, 16, 16, f(1e-3), f(0.1), 10, r, r, NUL, 0, NUL) == -1   # r aliases work
    assert lib.tidas_deconvolve(ok, 65, y, 1, 16, 16, f(1e-3), f(0.0), 10, r, w, NUL, 0, NUL) == -1   # eta = 0
    assert lib.tidas_deconvolve(ok, 65, y, 1, 16, 16, f(-1.0), f(0.1), 10, r, w, NUL, 0, NUL) == -1   # lam < 0
    assert lib.tidas_deconvolve(ok, 64, y, 1, 16, 16, f(1e-3), f(0.1), 10, r, w, NUL, 0, NUL) == -1   # even K
    assert lib.tidas_deconvolve(ok, 65, y, 1, 16, 16, f(1e-3), f(0.1), -1, r, w, NUL, 0, NUL) == -1   # iters < 0
    out = ctypes.c_double(0)
    assert lib.tidas_operator_norm_sq(ok, 65, 16, 0, w, ctypes.byref(out), NUL, 0, NUL) == -1
    assert lib.tidas_operator_norm_sq(ok, 65, 16, 10, w, None, NUL, 0, NUL) == -1
    assert lib.tidas_apply_ex(ok, 65, y, 1, 16, 16, f(1.0), f(1.0), y, r, NUL) == -1        # base aliases input
    assert lib.tidas_adjoint_ex(ok, 65, y, 1, 16, 16, f(float("inf")), f(1.0), None, r, NUL) == -1


def test_batch_entry_points_reject_invalid_arguments(lib):
    arr, tx, rx, g = _geom()
    frames = (_lib.Frame * 2)()
    for f in range(2):
        frames[f] = _lib.Frame(g, 0x1000, 0x2000, 0x3000, 0x4000 + 0x100 * f)
    need = lib.tidas_batch_workspace_bytes(2)
    assert need >= 2 * 72 and lib.tidas_batch_workspace_bytes(0) == 0
    ws = ctypes.c_void_p(0x10000)
    geo = (ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx))
    assert lib.das_beamform_batch(*geo, 2048, frames, 2, ws, need - 1, 0, NUL) == -1       # small workspace
    assert lib.das_beamform_batch(*geo, 2048, frames, 2, ws, need, _lib.DAS_BATCH_VARIANTS, NUL) == -1  # variant
    assert lib.das_beamform_batch(*geo, 2048, frames, 0, ws, need, 0, NUL) == -1           # no frames
    assert lib.das_beamform_batch(*geo, 2048, frames, 2, ctypes.c_void_p(0x10004), need, 0, NUL) == -1  # alignment
    assert lib.tidas_apply_batch(frames, 2, 64, ws, need, 0, NUL) == -1                     # even K
    assert lib.tidas_apply_batch(frames, 2, 65, ws, need, -1, NUL) == -1                    # variant
    bad = (_lib.Frame * 1)()
    bad[0] = _lib.Frame(_lib.make_grid(0, 4, 0, 1e-4, 0, 1e-4), 0x1000, 0x2000, 0x3000, 0x4000)
    assert lib.tidas_apply_batch(bad, 1, 65, ws, need, 0, NUL) == -1                        # empty grid
    bad[0] = _lib.Frame(g, 0x1000, 0x2000, 0x3000, 0)
    assert lib.das_beamform_batch(*geo, 2048, bad, 1, ws, need, 0, NUL) == -1              # null output


def test_kernel_grad_rejects_invalid_arguments(lib):
    out = ctypes.c_void_p(0x3000)
    f = lib.tidas_kernel_grad
    assert f(65, NUL, FAKE, 1, 16, 16, out, NUL, 0, NUL) == _lib.TIDAS_EINVAL      # null refl
    assert f(65, FAKE, NUL, 1, 16, 16, out, NUL, 0, NUL) == _lib.TIDAS_EINVAL      # null image_bar
    assert f(65, FAKE, ctypes.c_void_p(0x2000), 1, 16, 16, NUL, NUL, 0, NUL) == _lib.TIDAS_EINVAL  # null output
    assert f(64, FAKE, ctypes.c_void_p(0x2000), 1, 16, 16, out, NUL, 0, NUL) == _lib.TIDAS_EINVAL  # even K
    assert f(0, FAKE, ctypes.c_void_p(0x2000), 1, 16, 16, out, NUL, 0, NUL) == _lib.TIDAS_EINVAL   # K = 0
    assert f(5, FAKE, ctypes.c_void_p(0x2000), 0, 16, 16, out, NUL, 0, NUL) == _lib.TIDAS_EINVAL   # B = 0
    assert f(5, FAKE, ctypes.c_void_p(0x2000), 1, 0, 16, out, NUL, 0, NUL) == _lib.TIDAS_EINVAL    # Z = 0
    assert f(5, FAKE, ctypes.c_void_p(0x2000), 1, 16, -1, out, NUL, 0, NUL) == _lib.TIDAS_EINVAL   # X < 0
    assert f(5, FAKE, ctypes.c_void_p(0x2000), 1, 16, 16, FAKE, NUL, 0, NUL) == _lib.TIDAS_EINVAL  # output aliases refl
    # a frame whose 32-bit byte offsets would overflow
    assert f(5, FAKE, ctypes.c_void_p(0x2000), 1, 1 << 20, 1024, out, NUL, 0, NUL) == _lib.TIDAS_EUNSUPPORTED
    assert lib.tidas_last_error()


def test_kernel_grad_path_choice(lib):
    k = lib.tidas_kernel_grad_kernel
    assert k(16, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)) == _lib.KGRAD_SPLIT_BF16
    assert k(16, ctypes.c_void_p(0x1004), ctypes.c_void_p(0x2000)) == _lib.KGRAD_FP32   # refl not 16-byte aligned
    assert k(16, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2008)) == _lib.KGRAD_FP32   # image_bar not aligned
    assert k(18, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)) == _lib.KGRAD_FP32   # X % 4 != 0
    assert k(0, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)) == _lib.TIDAS_EINVAL


def test_line_kernel_rejects_invalid_sizes(lib):
    assert lib.tidas_line_kernel(64, 1, 64, 64) == _lib.TIDAS_EINVAL   # even K
    assert lib.tidas_line_kernel(0, 1, 64, 64) == _lib.TIDAS_EINVAL
    assert lib.tidas_line_kernel(65, 0, 64, 64) == _lib.TIDAS_EINVAL
    assert lib.tidas_line_kernel(65, 1, 0, 64) == _lib.TIDAS_EINVAL
    assert lib.tidas_line_kernel(65, 1, 64, 0) == _lib.TIDAS_EINVAL


def test_prepared_bank_size_and_invalid_arguments(lib):
    # two-block images: 16 tiles of 64 rows, two modes, three bf16 planes of
    # 64 x 200 (K = 129); four-block images: 8 tiles of 128 rows, two modes,
    # four blocks of three planes of 32 x 168 (ten 16-row window steps), each
    # block padded to a multiple of 8 KB
    two = 2 * 16 * 3 * 64 * 200 * 2
    block = -(-3 * 32 * 168 * 2 // 8192) * 8192
    assert block == 32768
    assert lib.tidas_prepared_bytes(129, 1024) == two + 2 * 8 * 4 * block
    # K = 163: a 32-row block's window spans 13 steps of 16 rows, more than the
    # four-block tile's 12: two-block images only (16 steps, planes 64 x 264)
    assert lib.tidas_prepared_bytes(163, 128) == 2 * 2 * 3 * 64 * 264 * 2
    assert lib.tidas_prepared_bytes(161, 128) == 2 * 2 * 3 * 64 * 264 * 2 + 2 * 1 * 4 * 40960
    assert lib.tidas_prepared_bytes(129, 1000) == lib.tidas_prepared_bytes(129, 1024)
    assert lib.tidas_prepared_bytes(64, 1024) == 0      # even K
    assert lib.tidas_prepared_bytes(0, 1024) == 0
    assert lib.tidas_prepared_bytes(129, 0) == 0
    assert lib.tidas_prepared_bytes(401, 1024) == 0     # band tile larger than LDS
    big = 1 << 30
    assert lib.tidas_prepare(NUL, 129, 1024, FAKE, big, NUL) == _lib.TIDAS_EINVAL
    assert lib.tidas_prepare(FAKE, 129, 1024, NUL, big, NUL) == _lib.TIDAS_EINVAL
    assert lib.tidas_prepare(FAKE, 128, 1024, ctypes.c_void_p(0x2000), big, NUL) == _lib.TIDAS_EINVAL
    assert lib.tidas_prepare(FAKE, 129, 1024, ctypes.c_void_p(0x2000), 1000, NUL) == _lib.TIDAS_EINVAL  # too small
    assert lib.tidas_prepare(FAKE, 129, 1024, ctypes.c_void_p(0x2008), big, NUL) == _lib.TIDAS_EINVAL  # misaligned
    assert lib.tidas_prepare(FAKE, 401, 1024, ctypes.c_void_p(0x2000), big, NUL) == _lib.TIDAS_EUNSUPPORTED
    f1, f0 = ctypes.c_float(1.0), ctypes.c_float(0.0)
    for fn in (lib.tidas_apply_prepared, lib.tidas_adjoint_prepared):
        assert fn(NUL, 129, FAKE, 1, 64, 64, f1, f0, NUL, ctypes.c_void_p(0x2000), NUL) == _lib.TIDAS_EINVAL
        assert fn(FAKE, 128, FAKE, 1, 64, 64, f1, f0, NUL, ctypes.c_void_p(0x2000), NUL) == _lib.TIDAS_EINVAL
        assert fn(FAKE, 129, FAKE, 1, 64, 64, f1, f0, NUL, FAKE, NUL) == _lib.TIDAS_EINVAL  # out aliases input
        assert fn(FAKE, 401, FAKE, 1, 64, 64, f1, f0, NUL, ctypes.c_void_p(0x2000), NUL) == _lib.TIDAS_EUNSUPPORTED


def test_point_study_rejects_invalid_arguments(lib):
    arr = _lib.make_array(33, 0.3e-3, 1540.0)
    tx = _lib.make_tx([0.0], 40e6, 0.0, 5e6, 2.0)
    rx = _lib.make_rx(1.0)
    f = lib.tidas_point_study
    need = lib.tidas_point_study_workspace_bytes(33, 10, 1400, 1000)
    assert need > 10 * 33 * 1400 * 8
    assert lib.tidas_point_study_workspace_bytes(33, 0, 1400, 1000) == 0
    T, Th, L, G, S, W, WS = (ctypes.c_void_p(a) for a in (0x1000, 0x2000, 0x3000, 0x4000, 0x5000, 0x6000, 0x7000))

    def call(arr_=arr, tx_=tx, rx_=rx, n_tx=9, ns=1400, P=10, z1=6e-3, dz=2e-3, fi=4, lh=1000, sh=100,
             th=Th, lo=L, gl=G, st=S, ws=WS, nb=need):
        return f(ctypes.byref(arr_), ctypes.byref(tx_), ctypes.byref(rx_), n_tx, ns, P, z1, dz, fi, lh, sh, th, lo,
                 gl, st, W, ws, nb, NUL)
    E = _lib.TIDAS_EINVAL
    assert call(n_tx=8) == E                                   # C - n_tx odd
    assert call(n_tx=0) == E and call(n_tx=35) == E
    assert call(tx_=_lib.make_tx([0.1], 40e6, 0.0, 5e6, 2.0)) == E      # steered
    assert call(tx_=_lib.make_tx([0.0, 0.0], 40e6, 0.0, 5e6, 2.0)) == E  # several angles
    assert call(ns=1) == E and call(P=0) == E
    assert call(z1=0.0) == E and call(dz=0.0) == E
    assert call(fi=10) == E and call(fi=-1) == E and call(lh=-1) == E
    assert call(sh=512) == E                                   # stats axis over 1023 samples
    assert call(th=NUL) == E and call(ws=NUL) == E
    assert call(lo=Th) == E and call(st=G) == E                 # overlapping outputs
    assert call(nb=need - 1) == E                               # short workspace
    big = _lib.make_array(514, 0.3e-3, 1540.0)
    assert call(arr_=big, n_tx=10) == _lib.TIDAS_EUNSUPPORTED
    assert call(tx_=_lib.make_tx([0.0], 40e6, 0.0, 0.2e6, 2.0)) == _lib.TIDAS_EUNSUPPORTED  # pulse too long
    assert lib.tidas_last_error()


def test_kossoff_count_matches_the_oracle_on_the_host(lib):
    from oracle import point_study as ps
    for C in (16, 17, 64, 127, 128, 192):
        for fc in (3e6, 5e6, 7e6, 9e6):
            for zf in (2e-3, 15e-3, 25e-3, 35e-3, 1.0):
                arr = _lib.make_array(C, 0.3e-3, 1540.0)
                assert lib.tidas_kossoff_tx_count(ctypes.byref(arr), fc, zf, 0.6) == \
                    ps.kossoff_tx_count(C, 0.3e-3, 1540.0, fc, zf)
    arr = _lib.make_array(16, 0.3e-3, 1540.0)
    assert lib.tidas_kossoff_tx_count(ctypes.byref(arr), 0.0, 25e-3, 0.6) == _lib.TIDAS_EINVAL
    assert lib.tidas_kossoff_tx_count(ctypes.byref(arr), 5e6, 25e-3, 0.0) == _lib.TIDAS_EINVAL
