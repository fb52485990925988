"""MI355X-native tiDAS (arXiv 2507.15464): exact DAS, per-depth-row kernel
banks, the time-invariant line model and its adjoint, as hand-written HIP
kernels for gfx950 behind a C ABI (include/tidas.h)."""
from .api import (Prepared, adjoint, apply, apply_lateral, build_kernels, das_beamform, kernel_grad,  # noqa: F401
                  kernel_grad_kernel, kossoff_tx_count, line_kernel, point_study, prepare, simulate_rf, tidas_beamform, version)
from .autograd import TiDASFunction, adjoint_ex, apply_ex, deconvolve, operator_norm_sq, step_size, tidas  # noqa: F401,E402
from .batch import PreparedBatch, apply_batch, das_beamform_batch  # noqa: F401,E402
from . import autotune  # noqa: F401,E402
from . import surrogate  # noqa: F401,E402
