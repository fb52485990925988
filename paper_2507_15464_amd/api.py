"""Python entry points of the tiDAS library: thin wrappers over the C ABI.

Geometry arguments are duck-typed: ``setup`` needs ``n_elem, pitch, c, fs, t0,
fc, cycles, angles, fnumber``; ``grid`` needs ``nz, nx, z0, dz, x0, dx`` (one
object may provide both).  Tensors must be float32, contiguous and on the
current HIP device; results are enqueued on torch's current stream.
"""
import ctypes

import torch

from . import _lib

__all__ = ["das_beamform", "tidas_beamform", "build_kernels", "apply", "adjoint", "apply_lateral", "kernel_grad", "kernel_grad_kernel", "point_study", "kossoff_tx_count",
           "simulate_rf", "version"]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _workspace(nbytes, dev):
    """Device scratch of a call and its size (None, 0 when it needs none), from
    torch's caching allocator, so that the library itself allocates nothing."""
    nbytes = int(nbytes)
    if nbytes == 0:
        return None, 0
    return torch.empty(nbytes, dtype=torch.uint8, device=dev), nbytes


def _check_tensor(t, name, dtype=torch.float32):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _descs(setup, grid=None):
    arr = _lib.make_array(setup.n_elem, setup.pitch, setup.c)
    tx = _lib.make_tx(list(setup.angles), setup.fs, setup.t0, setup.fc, setup.cycles)
    rx = _lib.make_rx(setup.fnumber)
    g = _lib.make_grid(grid.nz, grid.nx, grid.z0, grid.dz, grid.x0, grid.dx) if grid is not None else None
    return arr, tx, rx, g


def version():
    return _lib.load().tidas_version().decode()


def das_beamform(rf, setup, grid=None, out=None):
    """Exact DAS.  rf [B][A][C][T] (or [A][C][T]) -> image [B][Z][X] (or [Z][X])."""
    grid = grid or setup
    lib = _lib.load()
    _check_tensor(rf, "rf")
    squeeze = rf.dim() == 3
    r4 = rf.unsqueeze(0) if squeeze else rf
    if r4.dim() != 4 or r4.shape[1] != len(setup.angles) or r4.shape[2] != setup.n_elem:
        raise ValueError("rf must be [B][A][C][T] matching the setup")
    B, T = r4.shape[0], r4.shape[3]
    if out is None:
        out = torch.empty((B, grid.nz, grid.nx), device=rf.device, dtype=torch.float32)
    _check_tensor(out, "out")
    arr, tx, rx, g = _descs(setup, grid)
    ws, nws = _workspace(lib.das_beamform_workspace_bytes(len(setup.angles), setup.n_elem, T, B), rf.device)
    _lib.check(lib.das_beamform(ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(g),
                                _ptr(r4), T, B, _ptr(out), _ptr(ws), nws, _stream()))
    return out[0] if squeeze else out


def tidas_beamform(rf, setup, ref_row=None, theta=None, grid=None, out=None):
    """The time-invariant beamformer from RF: each row's receive law frozen at
    its reference row (ref_row: int32 device tensor [Z] or None = own row),
    scaled by theta (device [Z] or None = ones).  rf as in ``das_beamform``."""
    grid = grid or setup
    lib = _lib.load()
    _check_tensor(rf, "rf")
    squeeze = rf.dim() == 3
    r4 = rf.unsqueeze(0) if squeeze else rf
    if r4.dim() != 4 or r4.shape[1] != len(setup.angles) or r4.shape[2] != setup.n_elem:
        raise ValueError("rf must be [B][A][C][T] matching the setup")
    if ref_row is not None:
        _check_tensor(ref_row, "ref_row", torch.int32)
        if ref_row.shape != (grid.nz,):
            raise ValueError("ref_row must be [Z]")
    if theta is not None:
        _check_tensor(theta, "theta")
        if theta.shape != (grid.nz,):
            raise ValueError("theta must be [Z]")
    B, T = r4.shape[0], r4.shape[3]
    if out is None:
        out = torch.empty((B, grid.nz, grid.nx), device=rf.device, dtype=torch.float32)
    _check_tensor(out, "out")
    arr, tx, rx, g = _descs(setup, grid)
    ws, nws = _workspace(lib.tidas_beamform_workspace_bytes(len(setup.angles), setup.n_elem, T, B), rf.device)
    _lib.check(lib.tidas_beamform(ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(g),
                                  _ptr(r4), T, B, _ptr(ref_row), _ptr(theta), _ptr(out), _ptr(ws), nws, _stream()))
    return out[0] if squeeze else out


def build_kernels(setup, grid=None, K=None, mode="exact", ref_row=None, n_samples=None, with_theta=False):
    """Kernel bank [Z][K] (and theta [Z] when with_theta)."""
    grid = grid or setup
    lib = _lib.load()
    K = int(K if K is not None else setup.K)
    T = int(n_samples if n_samples is not None else setup.n_samples)
    m = {"exact": _lib.MODE_EXACT, "paper": _lib.MODE_PAPER, "line": _lib.MODE_LINE,
         "lateral": _lib.MODE_LATERAL}[mode]
    dev = torch.device("cuda", torch.cuda.current_device())
    kb = torch.empty((grid.nz, K), device=dev, dtype=torch.float32)
    th = torch.empty(grid.nz, device=dev, dtype=torch.float32) if with_theta else None
    ref = None
    if ref_row is not None:
        vals = [int(v) for v in ref_row]
        if len(vals) != grid.nz:
            raise ValueError("ref_row must have one entry per depth row")
        ref = (ctypes.c_int32 * len(vals))(*vals)
    arr, tx, rx, g = _descs(setup, grid)
    ws, nws = _workspace(lib.tidas_build_kernels_workspace_bytes(grid.nz, K, m), dev)
    _lib.check(lib.tidas_build_kernels(ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), ctypes.byref(g), T, K,
                                       m, ref, _ptr(kb), _ptr(th), _ptr(ws), nws, _stream()))
    return (kb, th) if with_theta else kb


class Prepared:
    """A kernel bank converted once by ``tidas_prepare`` (forward and adjoint
    band tiles in split-bfloat16 form).  Pass it wherever a kernel bank is
    taken; results equal those of the bank itself, bit for bit.  Valid while
    the bank it was made from is unchanged."""

    def __init__(self, kernels):
        lib = _lib.load()
        _check_tensor(kernels, "kernels")
        if kernels.dim() != 2:
            raise ValueError("kernels must be [Z][K]")
        self.Z, self.K = int(kernels.shape[0]), int(kernels.shape[1])
        nbytes = lib.tidas_prepared_bytes(self.K, self.Z)
        if nbytes == 0:
            raise _lib.TidasError(_lib.TIDAS_EUNSUPPORTED, f"no prepared form for K={self.K}")
        self.buffer = torch.empty(nbytes, device=kernels.device, dtype=torch.uint8)
        _lib.check(lib.tidas_prepare(_ptr(kernels), self.K, self.Z, _ptr(self.buffer), nbytes, _stream()))
        self.device = kernels.device
        self.shape = (self.Z, self.K)


def line_kernel(K, B, Z, X):
    """Which line-model kernel a launch of B frames of Z x X with K taps runs
    (``_lib.LINE_FOUR_BLOCK`` … ``_lib.LINE_VECTOR``)."""
    r = _lib.load().tidas_line_kernel(int(K), int(B), int(Z), int(X))
    _lib.check(r if r < 0 else 0)
    return r


def kernel_grad_kernel(refl, image_bar):
    """Which kernel ``kernel_grad`` runs for these inputs
    (``_lib.KGRAD_SPLIT_BF16`` or ``_lib.KGRAD_FP32``)."""
    r = _lib.load().tidas_kernel_grad_kernel(int(refl.shape[-1]), _ptr(refl), _ptr(image_bar))
    _lib.check(r if r < 0 else 0)
    return r


def prepare(kernels):
    """Convert a kernel bank [Z][K] once for repeated ``apply`` / ``adjoint``."""
    return Prepared(kernels)


def conv_ex(adj, kernels, x, alpha=1.0, beta=0.0, base=None, out=None):
    """alpha * A(x) + beta * base (adj: A^T); kernels a bank [Z][K] or a Prepared."""
    lib = _lib.load()
    _check_tensor(x, "input")
    x3 = x.unsqueeze(0) if x.dim() == 2 else x
    if x3.dim() != 3:
        raise ValueError("the input must be [B][Z][X] or [Z][X]")
    B, Z, X = x3.shape
    if base is not None:
        _check_tensor(base, "base")
        if base.numel() != x3.numel():
            raise ValueError("base must have the input's shape")
    if out is None:
        out = torch.empty_like(x3)
    _check_tensor(out, "out")
    if isinstance(kernels, Prepared):
        if kernels.Z != Z:
            raise ValueError("the prepared bank's Z differs from the input's")
        fn = "tidas_adjoint_prepared" if adj else "tidas_apply_prepared"
        ptr, K = _ptr(kernels.buffer), kernels.K
    else:
        _check_tensor(kernels, "kernels")
        if kernels.dim() != 2 or kernels.shape[0] != Z:
            raise ValueError("kernels must be [Z][K] with the input's Z")
        fn = "tidas_adjoint_ex" if adj else "tidas_apply_ex"
        ptr, K = _ptr(kernels), kernels.shape[1]
    _lib.check(getattr(lib, fn)(ptr, K, _ptr(x3), B, Z, X, ctypes.c_float(alpha), ctypes.c_float(beta), _ptr(base),
                                _ptr(out), _stream()))
    return out.view(x.shape)


def _conv(fn, kernels, x, out):
    if isinstance(kernels, Prepared):
        return conv_ex(fn == "tidas_adjoint", kernels, x, out=out)
    lib = _lib.load()
    _check_tensor(kernels, "kernels")
    _check_tensor(x, "input")
    squeeze = x.dim() == 2
    x3 = x.unsqueeze(0) if squeeze else x
    if x3.dim() != 3 or kernels.dim() != 2 or kernels.shape[0] != x3.shape[1]:
        raise ValueError("kernels must be [Z][K] and the input [B][Z][X] with the same Z")
    B, Z, X = x3.shape
    if out is None:
        out = torch.empty_like(x3)
    _check_tensor(out, "out")
    _lib.check(getattr(lib, fn)(_ptr(kernels), kernels.shape[1], _ptr(x3), B, Z, X, _ptr(out), _stream()))
    return out[0] if squeeze else out


def apply(kernels, refl, out=None):
    """tiDAS line model: image = A(refl), refl [B][Z][X] or [Z][X]."""
    return _conv("tidas_apply", kernels, refl, out)


def adjoint(kernels, image_bar, out=None):
    """Transpose of ``apply``."""
    return _conv("tidas_adjoint", kernels, image_bar, out)


def apply_lateral(kernels_x, x, out=None):
    """Lateral pass of the separable 2-D model: each row of x ([B][Z][X] or
    [Z][X]) convolved along X with its kernel kernels_x [Z][K]."""
    if isinstance(kernels_x, Prepared):
        raise TypeError("the lateral pass takes a kernel bank, not a prepared line-model bank")
    return _conv("tidas_apply_lateral", kernels_x, x, out)


def kernel_grad(refl, image_bar, K, out=None):
    """Gradient of the line model in its kernels: [Z][K] from refl and image_bar ([B][Z][X] or [Z][X])."""
    lib = _lib.load()
    _check_tensor(refl, "refl")
    _check_tensor(image_bar, "image_bar")
    if refl.shape != image_bar.shape or refl.dim() not in (2, 3):
        raise ValueError("refl and image_bar must share one [B][Z][X] or [Z][X] shape")
    B, Z, X = (1,) + tuple(refl.shape) if refl.dim() == 2 else tuple(refl.shape)
    if out is None:
        out = torch.empty((Z, int(K)), device=refl.device, dtype=torch.float32)
    _check_tensor(out, "out")
    if tuple(out.shape) != (Z, int(K)):
        raise ValueError("out must be [Z][K]")
    ws, nws = _workspace(lib.tidas_kernel_grad_workspace_bytes(int(K), B, Z, X), refl.device)
    _lib.check(lib.tidas_kernel_grad(int(K), _ptr(refl), _ptr(image_bar), B, Z, X, _ptr(out), _ptr(ws), nws,
                                     _stream()))
    return out


def simulate_rf(setup, scat, n_samples=None, out=None):
    """RF [A][C][T] of scatterers ``scat`` (float64 device tensor [S][3]: x, z, amplitude)."""
    lib = _lib.load()
    T = int(n_samples if n_samples is not None else setup.n_samples)
    _check_tensor(scat, "scat", torch.float64)
    if scat.dim() != 2 or scat.shape[1] != 3:
        raise ValueError("scat must be [S][3]")
    if out is None:
        out = torch.empty((len(setup.angles), setup.n_elem, T), device=scat.device, dtype=torch.float32)
    _check_tensor(out, "out")
    arr, tx, _, _ = _descs(setup)
    ws, nws = _workspace(lib.tidas_simulate_rf_workspace_bytes(len(setup.angles), setup.n_elem, T), scat.device)
    _lib.check(lib.tidas_simulate_rf(ctypes.byref(arr), ctypes.byref(tx), _ptr(scat), scat.shape[0], T, _ptr(out),
                                     _ptr(ws), nws, _stream()))
    return out


def kossoff_tx_count(setup, z_focus, ratio=0.6):
    """Transmit elements of the single-point study's focused beam (Kossoff's criterion)."""
    arr = _lib.make_array(setup.n_elem, setup.pitch, setup.c)
    r = _lib.load().tidas_kossoff_tx_count(ctypes.byref(arr), float(setup.fc), float(z_focus), float(ratio))
    _lib.check(r if r < 0 else 0)
    return r


def point_study(setup, n_tx, n_points, z_first, z_step, focal_index, line_half, stats_half=None):
    """The single-point study (``tidas_point_study``) on the current device.

    ``setup`` needs n_elem, pitch, c, fs, t0, fc, cycles, fnumber, n_samples
    and angles == (0.0,).  Returns a dict of float64 device tensors: theta,
    err_local, err_global ([P][P], entry [r][s]), stats ([P][4] or None) and
    window (W in metres, a 1-element tensor)."""
    lib = _lib.load()
    dev = torch.device("cuda", torch.cuda.current_device())
    P = int(n_points)
    nbytes = int(lib.tidas_point_study_workspace_bytes(int(setup.n_elem), P, int(setup.n_samples), int(line_half)))
    if nbytes == 0:
        raise ValueError("invalid study sizes")
    ws = torch.empty(nbytes, device=dev, dtype=torch.uint8)
    out = {k: torch.empty((P, P), device=dev, dtype=torch.float64) for k in ("theta", "err_local", "err_global")}
    out["stats"] = torch.empty((P, 4), device=dev, dtype=torch.float64) if stats_half is not None else None
    out["window"] = torch.empty(1, device=dev, dtype=torch.float64)
    arr, tx, rx, _ = _descs(setup)
    _lib.check(lib.tidas_point_study(ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), int(n_tx),
                                     int(setup.n_samples), P, float(z_first), float(z_step), int(focal_index),
                                     int(line_half), int(stats_half or 0), _ptr(out["theta"]),
                                     _ptr(out["err_local"]), _ptr(out["err_global"]), _ptr(out["stats"]),
                                     _ptr(out["window"]), _ptr(ws), nbytes, _stream()))
    out["_workspace"] = ws  # kept alive until the caller synchronises
    return out
