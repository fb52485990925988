"""Kernel surrogate: an MLP from (depth, F-number, steering angle, centre
frequency) to a normalised exact-mode row kernel, trained and run by the
library's own matrix-core kernels.

Not claimed by the paper (its conclusion calls the weights Theta learned).
The target of row i is K_i / s_i with s_i = max(sum_n w(-x_n, z_i), 1) the
aperture weight sum, so kernels of very different amplitude (aperture size
grows with depth) share one scale; inference multiplies the output back by
s_i.  Exact kernels (``tidas_kernels_at``) stay available as the fallback
and serve as the error judge.

All arithmetic runs in the C ABI (features, forward, loss and gradients,
Adam, data generation).  This module owns buffers and the step schedule.
"""
import ctypes
import math

import torch

from . import _lib
from .api import _check_tensor, _stream

__all__ = ["Surrogate", "kernels_at", "features", "aperture_scale", "rel_l2"]

WIDTHS = (4, 256, 256, 256, 129)


def _widths_arg(widths):
    return (ctypes.c_int32 * 5)(*[int(w) for w in widths])


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def kernels_at(array, fs, t0, cycles, n_samples, dz, params, K, normalise=False):
    """Exact-mode kernels [N][K] and aperture scales [N] for per-row draws
    ``params`` (float64 device tensor [N][4]: depth, F-number, angle, fc).
    ``array`` needs ``n_elem, pitch, c``."""
    lib = _lib.load()
    _check_tensor(params, "params", torch.float64)
    N = params.shape[0]
    out = torch.empty((N, K), device=params.device, dtype=torch.float32)
    scale = torch.empty(N, device=params.device, dtype=torch.float32)
    arr = _lib.make_array(array.n_elem, array.pitch, array.c)
    _lib.check(lib.tidas_kernels_at(ctypes.byref(arr), float(fs), float(t0), float(cycles), int(n_samples), float(dz),
                                    _ptr(params), N, int(K), int(bool(normalise)), _ptr(out), _ptr(scale), _stream()))
    return out, scale


def rel_l2(a, b):
    """||a - b|| / ||b|| over two float32 device tensors of equal size."""
    lib = _lib.load()
    _check_tensor(a, "a")
    _check_tensor(b, "b")
    if a.numel() != b.numel():
        raise ValueError("sizes differ")
    work = torch.empty(2, device=a.device, dtype=torch.float64)
    out = (ctypes.c_double * 2)()
    _lib.check(lib.tidas_sq_norms(_ptr(a), _ptr(b), a.numel(), _ptr(work), out, _stream()))
    return math.sqrt(out[0] / out[1]) if out[1] > 0 else math.sqrt(out[0])


def aperture_scale(array, params):
    """s_i = max(sum_n w(-x_n, z_i), 1) for each row draw (no kernel taps)."""
    _, s = kernels_at(array, 1.0, 0.0, 1.0, 2, 1.0, params, 1)
    return s


def features(params, lo, hi):
    """Normalised network inputs [N][4] in [-1, 1] from float64 draws [N][4]."""
    lib = _lib.load()
    _check_tensor(params, "params", torch.float64)
    N = params.shape[0]
    x = torch.empty((N, 4), device=params.device, dtype=torch.float32)
    dlo = (ctypes.c_double * 4)(*[float(v) for v in lo])
    dhi = (ctypes.c_double * 4)(*[float(v) for v in hi])
    _lib.check(lib.tidas_mlp_features(_ptr(params), N, dlo, dhi, _ptr(x), _stream()))
    return x


class Surrogate:
    """Flat float32 master parameters, their bfloat16 copy, Adam moments."""

    def __init__(self, widths=WIDTHS, device=None):
        self.lib = _lib.load()
        self.widths = tuple(int(w) for w in widths)
        self._w = _widths_arg(self.widths)
        self.P = int(self.lib.tidas_mlp_param_count(self._w))
        if self.P <= 0:
            raise ValueError("bad widths")
        dev = device or torch.device("cuda", torch.cuda.current_device())
        self.params = torch.zeros(self.P, device=dev, dtype=torch.float32)
        self.params16 = torch.zeros(self.P, device=dev, dtype=torch.bfloat16)
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, device=dev, dtype=torch.float32)
        self.step = 0
        self._work = {}

    # -- parameter exchange (host layout: list of (W [out][in], b [out])) --
    def load_layers(self, layers):
        flat = []
        for W, b in layers:
            flat.append(torch.as_tensor(W, dtype=torch.float32).reshape(-1))
            flat.append(torch.as_tensor(b, dtype=torch.float32).reshape(-1))
        p = torch.cat(flat)
        if p.numel() != self.P:
            raise ValueError("layer shapes do not match the widths")
        self.params.copy_(p.to(self.params.device))
        self.refresh_bf16()

    def layers(self):
        p = self.params.detach().cpu().double().numpy()
        out, off = [], 0
        for i, o in zip(self.widths[:-1], self.widths[1:]):
            W = p[off:off + o * i].reshape(o, i)
            off += o * i
            b = p[off:off + o]
            off += o
            out.append((W, b))
        return out

    def refresh_bf16(self):
        _lib.check(self.lib.tidas_mlp_to_bf16(_ptr(self.params), self.P, _ptr(self.params16), _stream()))

    def _workspace(self, N):
        w = self._work.get(N)
        if w is None:
            nbytes = int(self.lib.tidas_mlp_workspace_bytes(self._w, N))
            w = (torch.empty(nbytes + 256, dtype=torch.uint8, device=self.params.device), nbytes)
            self._work[N] = w
        buf, nbytes = w
        off = (-buf.data_ptr()) % 256
        return ctypes.c_void_p(buf.data_ptr() + off), nbytes

    # -- compute --
    def forward(self, x, scale=None, out=None):
        _check_tensor(x, "x")
        N = x.shape[0]
        y = out if out is not None else torch.empty((N, self.widths[-1]), device=x.device, dtype=torch.float32)
        ws, nb = self._workspace(N)
        _lib.check(self.lib.tidas_mlp_forward(self._w, _ptr(self.params16), _ptr(self.params), _ptr(x), N,
                                              _ptr(scale), _ptr(y), ws, nb, _stream()))
        return y

    def train_step(self, x, target, idx=None, batch=None):
        """Loss and gradient on rows idx of (x, target) (or the first ``batch`` rows)."""
        _check_tensor(x, "x")
        _check_tensor(target, "target")
        n_rows = x.shape[0]
        if idx is not None:
            _check_tensor(idx, "idx", torch.int32)
            N = idx.shape[0]
        else:
            N = batch or n_rows
        ws, nb = self._workspace(N)
        _lib.check(self.lib.tidas_mlp_train_step(self._w, _ptr(self.params16), _ptr(self.params), _ptr(x),
                                                 _ptr(target), n_rows, _ptr(idx), N, _ptr(self.grad),
                                                 _ptr(self.loss), ws, nb, _stream()))
        return self.loss

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _lib.check(self.lib.tidas_mlp_adam(self._w, _ptr(self.params), _ptr(self.grad), _ptr(self.m), _ptr(self.v),
                                           _ptr(self.params16), ctypes.c_float(lr), ctypes.c_float(beta1),
                                           ctypes.c_float(beta2), ctypes.c_float(eps), self.step, _stream()))

    @staticmethod
    def cosine_lr(step, total, lr0=1e-3, lr1=1e-5):
        f = min(max(step / float(total), 0.0), 1.0)
        return lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * f))

    def fit(self, x, target, batches, total_steps=None, lr0=1e-3, lr1=1e-5, log_every=0, log=None):
        """Run one Adam step per index batch (device int32 tensors), cosine
        schedule over ``total_steps`` (default: len(batches)) counted from the
        current step, so a resumed run continues the same schedule."""
        total = total_steps or (self.step + len(batches))
        for idx in batches:
            self.train_step(x, target, idx=idx)
            self.adam(self.cosine_lr(self.step, total, lr0, lr1))
            if log_every and log is not None and self.step % log_every == 0:
                log(self.step, float(self.loss))
        return float(self.loss)

    def kernel_bank(self, rig, params, lo, hi, judge_rows=16, tol=1e-2):
        """Kernel bank [N][K] for row draws ``params`` (float64 device [N][4]).

        The surrogate predicts every row; the exact kernels of ``judge_rows``
        evenly spaced rows judge it.  If their relative L2 error exceeds
        ``tol`` the bank falls back to exact kernels for all rows.  ``rig``
        needs ``n_elem, pitch, c, fs, t0, cycles, n_samples, dz``.
        Returns (bank, info)."""
        N = params.shape[0]
        K = self.widths[-1]
        x = features(params, lo, hi)
        s = aperture_scale(rig, params)
        bank = self.forward(x, scale=s)
        rows = torch.linspace(0, N - 1, min(judge_rows, N), device=params.device).round().long()
        exact_rows, _ = kernels_at(rig, rig.fs, rig.t0, rig.cycles, rig.n_samples, rig.dz, params[rows].contiguous(), K)
        err = rel_l2(bank[rows].contiguous(), exact_rows)
        info = {"judge_rel_l2": err, "fallback": False}
        if err > tol:
            bank, _ = kernels_at(rig, rig.fs, rig.t0, rig.cycles, rig.n_samples, rig.dz, params, K)
            info["fallback"] = True
        return bank, info

    # -- checkpoint / resume --
    def state_dict(self):
        return {"widths": list(self.widths), "params": self.params.detach().cpu(), "m": self.m.detach().cpu(),
                "v": self.v.detach().cpu(), "step": self.step}

    def load_state_dict(self, sd):
        if tuple(sd["widths"]) != self.widths:
            raise ValueError("checkpoint widths differ")
        self.params.copy_(sd["params"].to(self.params.device))
        self.m.copy_(sd["m"].to(self.m.device))
        self.v.copy_(sd["v"].to(self.v.device))
        self.step = int(sd["step"])
        self.refresh_bf16()

    def save(self, path):
        torch.save(self.state_dict(), path)

    def load(self, path):
        self.load_state_dict(torch.load(path, map_location="cpu", weights_only=True))
