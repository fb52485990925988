"""torch.autograd integration and Tikhonov deconvolution through the line model.

``TiDASFunction``: forward = tidas_apply, backward = tidas_adjoint (the exact
transpose) for the reflectivity map and tidas_kernel_grad for a kernel bank
that requires a gradient, so any loss built on the line model's output
back-propagates through the library's own kernels to the map and to the
kernels (a prepared bank is a constant).

``deconvolve``: the library's native gradient loop for
1/2 ||A r - y||^2 + lam/2 ||r||^2 (two fused launches per step).
``operator_norm_sq``: largest eigenvalue of A^T A by power iteration on the
device, from which a safe step size 1 / (||A||^2 + lam) follows.
"""
import ctypes

import torch

from . import _lib
from .api import Prepared, _check_tensor, _ptr, _stream, _workspace, adjoint, apply, conv_ex, kernel_grad

__all__ = ["TiDASFunction", "tidas", "apply_ex", "adjoint_ex", "deconvolve", "operator_norm_sq", "step_size"]


class TiDASFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, refl, kernels):
        refl = refl.contiguous()
        if isinstance(kernels, Prepared):
            ctx.prepared = kernels
            ctx.save_for_backward(None, None)
        else:
            ctx.prepared = None
            ctx.save_for_backward(kernels, refl if ctx.needs_input_grad[1] else None)
        return apply(kernels, refl)

    @staticmethod
    def backward(ctx, grad_out):
        kernels, refl = ctx.saved_tensors
        if ctx.prepared is not None:
            kernels = ctx.prepared
        grad_out = grad_out.contiguous()
        g_refl = adjoint(kernels, grad_out) if ctx.needs_input_grad[0] else None
        g_k = None
        if ctx.prepared is None and ctx.needs_input_grad[1]:
            g_k = kernel_grad(refl, grad_out, kernels.shape[1])
        return g_refl, g_k


def tidas(refl, kernels):
    """Differentiable line model: image = A(refl)."""
    return TiDASFunction.apply(refl, kernels)


def apply_ex(kernels, refl, alpha=1.0, beta=0.0, base=None, out=None):
    """out = alpha * A(refl) + beta * base (base may be ``out`` itself); kernels a bank or a Prepared."""
    return conv_ex(False, kernels, refl, alpha, beta, base, out)


def adjoint_ex(kernels, image_bar, alpha=1.0, beta=0.0, base=None, out=None):
    """out = alpha * A^T(image_bar) + beta * base (base may be ``out`` itself); kernels a bank or a Prepared."""
    return conv_ex(True, kernels, image_bar, alpha, beta, base, out)


def operator_norm_sq(kernels, iters=100):
    """Largest eigenvalue of A^T A of the column operator (power iteration on the device)."""
    lib = _lib.load()
    _check_tensor(kernels, "kernels")
    Z, K = kernels.shape
    work = torch.empty(3 * Z + 4, device=kernels.device, dtype=torch.float32)
    out = ctypes.c_double(0.0)
    ws, nws = _workspace(lib.tidas_operator_norm_sq_workspace_bytes(K, Z), kernels.device)
    _lib.check(lib.tidas_operator_norm_sq(_ptr(kernels), K, Z, int(iters), _ptr(work), ctypes.byref(out), _ptr(ws),
                                          nws, _stream()))
    return out.value


def step_size(kernels, lam, iters=100):
    """eta = 1 / (||A||^2 + lam), the inverse Lipschitz constant of the gradient."""
    return 1.0 / (operator_norm_sq(kernels, iters) + lam)


def deconvolve(kernels, y, lam, eta=None, iters=200, out=None, work=None):
    """Gradient-descent Tikhonov deconvolution of y [B][Z][X] (or [Z][X]) from r_0 = 0."""
    lib = _lib.load()
    _check_tensor(kernels, "kernels")
    _check_tensor(y, "y")
    y3 = y.unsqueeze(0) if y.dim() == 2 else y
    B, Z, X = y3.shape
    if eta is None:
        eta = step_size(kernels, lam)
    r = torch.empty_like(y3) if out is None else out
    w = torch.empty_like(y3) if work is None else work
    _check_tensor(r, "out")
    _check_tensor(w, "work")
    ws, nws = _workspace(lib.tidas_deconvolve_workspace_bytes(kernels.shape[1], B, Z, X), y.device)
    _lib.check(lib.tidas_deconvolve(_ptr(kernels), kernels.shape[1], _ptr(y3), B, Z, X, ctypes.c_float(lam),
                                    ctypes.c_float(eta), int(iters), _ptr(r), _ptr(w), _ptr(ws), nws, _stream()))
    return r.view(y.shape)
