"""ctypes binding of ``libtidas.so`` (the C ABI declared in include/tidas.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  torch is imported before the library is loaded so that the
library binds to the HIP runtime torch already loaded (one runtime per
process).  A missing or stale library raises: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtidas.so")
DEBUG_LIB_PATH = os.path.join(HERE, "libtidas_debug.so")  # built with -DTIDAS_DEBUG

TIDAS_OK = 0
TIDAS_EINVAL = -1
TIDAS_EHIP = -2
TIDAS_ENOMEM = -3
TIDAS_EUNSUPPORTED = -4
MODE_EXACT = 0
MODE_PAPER = 1
MODE_LINE = 2
MODE_LATERAL = 3
LINE_FOUR_BLOCK, LINE_TWO_BLOCK, LINE_FP32_MATRIX, LINE_VECTOR = 1, 2, 3, 4
KGRAD_SPLIT_BF16, KGRAD_FP32 = 1, 2
DBG_NONFINITE_IN, DBG_STUDY_SPAN = 2, 4


class TidasError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tidas error {code}: {msg}")
        self.code = code


class Array(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int32), ("pitch", ctypes.c_double), ("c", ctypes.c_double)]


class Tx(ctypes.Structure):
    _fields_ = [("n_angles", ctypes.c_int32), ("angles", ctypes.POINTER(ctypes.c_double)),
                ("fs", ctypes.c_double), ("t0", ctypes.c_double), ("fc", ctypes.c_double),
                ("cycles", ctypes.c_double)]


class Rx(ctypes.Structure):
    _fields_ = [("fnumber", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32), ("z0", ctypes.c_double),
                ("dz", ctypes.c_double), ("x0", ctypes.c_double), ("dx", ctypes.c_double)]


class Frame(ctypes.Structure):
    _fields_ = [("grid", Grid), ("rf", ctypes.c_void_p), ("kernels", ctypes.c_void_p), ("in_", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]


DAS_BATCH_VARIANTS = 18
APPLY_BATCH_VARIANTS = 7
APPLY_BATCH_FOUR_BLOCK = 6


_P = ctypes.c_void_p
_I = ctypes.c_int32
_Z = ctypes.c_size_t
_SIGS = {
    "tidas_version": (ctypes.c_char_p, []),
    "tidas_last_error": (ctypes.c_char_p, []),
    "tidas_debug_flags": (_I, [ctypes.POINTER(ctypes.c_uint32), _I]),
    "das_beamform": (_I, [ctypes.POINTER(Array), ctypes.POINTER(Tx), ctypes.POINTER(Rx), ctypes.POINTER(Grid),
                          _P, _I, _I, _P, _P, _Z, _P]),
    "das_beamform_workspace_bytes": (_Z, [_I, _I, _I, _I]),
    "tidas_beamform": (_I, [ctypes.POINTER(Array), ctypes.POINTER(Tx), ctypes.POINTER(Rx), ctypes.POINTER(Grid),
                            _P, _I, _I, _P, _P, _P, _P, _Z, _P]),
    "tidas_beamform_workspace_bytes": (_Z, [_I, _I, _I, _I]),
    "tidas_build_kernels": (_I, [ctypes.POINTER(Array), ctypes.POINTER(Tx), ctypes.POINTER(Rx),
                                 ctypes.POINTER(Grid), _I, _I, _I, ctypes.POINTER(ctypes.c_int32), _P, _P, _P, _Z,
                                 _P]),
    "tidas_build_kernels_workspace_bytes": (_Z, [_I, _I, _I]),
    "tidas_apply": (_I, [_P, _I, _P, _I, _I, _I, _P, _P]),
    "tidas_adjoint": (_I, [_P, _I, _P, _I, _I, _I, _P, _P]),
    "tidas_apply_noalloc": (_I, [_P, _I, _P, _I, _I, _I, _P, _P]),
    "tidas_simulate_rf": (_I, [ctypes.POINTER(Array), ctypes.POINTER(Tx), _P, _I, _I, _P, _P, _Z, _P]),
    "tidas_simulate_rf_workspace_bytes": (_Z, [_I, _I, _I]),
    "tidas_apply_ex": (_I, [_P, _I, _P, _I, _I, _I, ctypes.c_float, ctypes.c_float, _P, _P, _P]),
    "tidas_adjoint_ex": (_I, [_P, _I, _P, _I, _I, _I, ctypes.c_float, ctypes.c_float, _P, _P, _P]),
    "tidas_line_kernel": (_I, [_I, _I, _I, _I]),
    "tidas_prepared_bytes": (ctypes.c_size_t, [_I, _I]),
    "tidas_prepare": (_I, [_P, _I, _I, _P, ctypes.c_size_t, _P]),
    "tidas_apply_prepared": (_I, [_P, _I, _P, _I, _I, _I, ctypes.c_float, ctypes.c_float, _P, _P, _P]),
    "tidas_adjoint_prepared": (_I, [_P, _I, _P, _I, _I, _I, ctypes.c_float, ctypes.c_float, _P, _P, _P]),
    "tidas_deconvolve": (_I, [_P, _I, _P, _I, _I, _I, ctypes.c_float, ctypes.c_float, _I, _P, _P, _P, _Z, _P]),
    "tidas_deconvolve_workspace_bytes": (_Z, [_I, _I, _I, _I]),
    "tidas_kernel_grad": (_I, [_I, _P, _P, _I, _I, _I, _P, _P, _Z, _P]),
    "tidas_kernel_grad_workspace_bytes": (_Z, [_I, _I, _I, _I]),
    "tidas_kernel_grad_kernel": (_I, [_I, _P, _P]),
    "tidas_point_study_workspace_bytes": (ctypes.c_size_t, [_I, _I, _I, _I]),
    "tidas_point_study": (_I, [ctypes.POINTER(Array), ctypes.POINTER(Tx), ctypes.POINTER(Rx), _I, _I, _I,
                               ctypes.c_double, ctypes.c_double, _I, _I, _I, _P, _P, _P, _P, _P, _P,
                               ctypes.c_size_t, _P]),
    "tidas_kossoff_tx_count": (_I, [ctypes.POINTER(Array), ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "tidas_apply_lateral": (_I, [_P, _I, _P, _I, _I, _I, _P, _P]),
    "tidas_operator_norm_sq": (_I, [_P, _I, _I, _I, _P, ctypes.POINTER(ctypes.c_double), _P, _Z, _P]),
    "tidas_operator_norm_sq_workspace_bytes": (_Z, [_I, _I]),
    "tidas_batch_workspace_bytes": (ctypes.c_size_t, [_I]),
    "das_beamform_batch": (_I, [ctypes.POINTER(Array), ctypes.POINTER(Tx), ctypes.POINTER(Rx), _I,
                                ctypes.POINTER(Frame), _I, _P, ctypes.c_size_t, _I, _P]),
    "tidas_apply_batch": (_I, [ctypes.POINTER(Frame), _I, _I, _P, ctypes.c_size_t, _I, _P]),
    "tidas_apply_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Frame), _I, _I]),
    "tidas_apply_batch_prepare": (_I, [ctypes.POINTER(Frame), _I, _I, _P, ctypes.c_size_t, _P]),
    "tidas_apply_batch_prepared": (_I, [ctypes.POINTER(Frame), _I, _I, _P, ctypes.c_size_t, _P]),
    "tidas_kernels_at": (_I, [ctypes.POINTER(Array), ctypes.c_double, ctypes.c_double, ctypes.c_double, _I,
                              ctypes.c_double, _P, _I, _I, _I, _P, _P, _P]),
    "tidas_mlp_param_count": (ctypes.c_int64, [ctypes.POINTER(ctypes.c_int32)]),
    "tidas_mlp_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(ctypes.c_int32), _I]),
    "tidas_mlp_features": (_I, [_P, _I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _P, _P]),
    "tidas_mlp_to_bf16": (_I, [_P, ctypes.c_int64, _P, _P]),
    "tidas_mlp_forward": (_I, [ctypes.POINTER(ctypes.c_int32), _P, _P, _P, _I, _P, _P, _P, ctypes.c_size_t, _P]),
    "tidas_mlp_train_step": (_I, [ctypes.POINTER(ctypes.c_int32), _P, _P, _P, _P, _I, _P, _I, _P, _P, _P,
                                  ctypes.c_size_t, _P]),
    "tidas_sq_norms": (_I, [_P, _P, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_double), _P]),
    "tidas_mlp_adam": (_I, [ctypes.POINTER(ctypes.c_int32), _P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, ctypes.c_float, _I, _P]),
}

_lib = None


def exported_symbols():
    """Names of the C entry points this binding expects."""
    return list(_SIGS)


def load(path=None):
    """Load the library once (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    import torch  # noqa: F401  -- binds the HIP runtime first
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with paper_2507_15464_amd.build.build()")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def check(code):
    if code != TIDAS_OK:
        msg = load().tidas_last_error().decode(errors="replace")
        raise TidasError(code, msg)


def make_array(n_elem, pitch, c):
    return Array(int(n_elem), float(pitch), float(c))


def make_tx(angles, fs, t0, fc, cycles):
    buf = (ctypes.c_double * max(1, len(angles)))(*[float(a) for a in angles])
    tx = Tx(len(angles), ctypes.cast(buf, ctypes.POINTER(ctypes.c_double)), float(fs), float(t0), float(fc),
            float(cycles))
    tx._keep = buf  # keep the HOST angle array alive with the descriptor
    return tx


def make_rx(fnumber):
    return Rx(float(fnumber))


def make_grid(nz, nx, z0, dz, x0, dx):
    return Grid(int(nz), int(nx), float(z0), float(dz), float(x0), float(dx))
