"""Ragged multi-frame batches: one persistent launch per batch.

Each frame carries its own image grid and buffers; the array / transmit /
receive set-up (and the tap count K for the line model) are shared.  The
launch variant (wave tile and workgroup shape, workgroups per compute unit, prefetch depth)
is a parameter; ``autotune`` picks it by timing.
"""
import ctypes

import torch

from . import _lib
from .api import _check_tensor, _descs, _stream

__all__ = ["das_beamform_batch", "apply_batch", "PreparedBatch"]


def _grid_of(g):
    return _lib.make_grid(g.nz, g.nx, g.z0, g.dz, g.x0, g.dx)


def _workspace(n, device):
    nbytes = _lib.load().tidas_batch_workspace_bytes(n)
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def das_beamform_batch(setup, grids, rfs, outs=None, variant=0):
    """DAS of ragged frames: outs[f] = DAS(rfs[f]) on grids[f] (one launch).
    rfs[f]: float32 [A][C][T] device tensors with a common T."""
    lib = _lib.load()
    n = len(grids)
    if n < 1 or len(rfs) != n:
        raise ValueError("need one RF record per grid")
    T = rfs[0].shape[-1]
    if outs is None:
        outs = [torch.empty((g.nz, g.nx), device=rfs[0].device, dtype=torch.float32) for g in grids]
    frames = (_lib.Frame * n)()
    for f, (g, rf, out) in enumerate(zip(grids, rfs, outs)):
        _check_tensor(rf, "rf")
        _check_tensor(out, "out")
        if rf.shape != (len(setup.angles), setup.n_elem, T):
            raise ValueError("every rf must be [A][C][T] with the same T")
        if out.shape != (g.nz, g.nx):
            raise ValueError("out[f] must be [nz][nx] of its grid")
        frames[f] = _lib.Frame(_grid_of(g), rf.data_ptr(), 0, 0, out.data_ptr())
    ws, nbytes = _workspace(n, rfs[0].device)
    arr, tx, rx, _ = _descs(setup)
    _lib.check(lib.das_beamform_batch(ctypes.byref(arr), ctypes.byref(tx), ctypes.byref(rx), T, frames, n,
                                      ctypes.c_void_p(ws.data_ptr()), nbytes, int(variant), _stream()))
    return outs


def _line_frames(kernels, refls, outs):
    n = len(kernels)
    if n < 1 or len(refls) != n:
        raise ValueError("need one reflectivity map per kernel bank")
    K = kernels[0].shape[1]
    if outs is None:
        outs = [torch.empty_like(r) for r in refls]
    frames = (_lib.Frame * n)()
    for f, (kb, r, out) in enumerate(zip(kernels, refls, outs)):
        for t, name in ((kb, "kernels"), (r, "refl"), (out, "out")):
            _check_tensor(t, name)
        if kb.dim() != 2 or kb.shape[1] != K or r.dim() != 2 or kb.shape[0] != r.shape[0] or out.shape != r.shape:
            raise ValueError("frame f needs kernels [Z][K] (common K), refl and out [Z][X]")
        g = _lib.make_grid(r.shape[0], r.shape[1], 0.0, 1.0, 0.0, 1.0)
        frames[f] = _lib.Frame(g, 0, kb.data_ptr(), r.data_ptr(), out.data_ptr())
    return frames, K, outs


def _line_workspace(frames, n, K, device):
    nbytes = _lib.load().tidas_apply_batch_workspace_bytes(frames, n, K)
    if nbytes == 0:
        raise ValueError("invalid batch")
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def apply_batch(kernels, refls, outs=None, variant=0):
    """Line model of ragged frames: outs[f] = A_f(refls[f]) with bank kernels[f] [Z_f][K]."""
    lib = _lib.load()
    frames, K, outs = _line_frames(kernels, refls, outs)
    n = len(outs)
    ws, nbytes = _line_workspace(frames, n, K, refls[0].device)
    _lib.check(lib.tidas_apply_batch(frames, n, K, ctypes.c_void_p(ws.data_ptr()), nbytes, int(variant), _stream()))
    return outs


class PreparedBatch:
    """A ragged batch of the line model prepared once (frame table and every
    frame's band images, ``tidas_apply_batch_prepare``): ``apply()`` is then one
    launch over the batch (``tidas_apply_batch_prepared``), writing ``outs``.
    The banks, maps and outputs are held by reference; the banks must not
    change while the batch is in use (the maps may: they are read at each
    ``apply``)."""

    def __init__(self, kernels, refls, outs=None):
        self.lib = _lib.load()
        self.kernels, self.refls = list(kernels), list(refls)
        self.frames, self.K, self.outs = _line_frames(self.kernels, self.refls, outs)
        self.n = len(self.outs)
        self.ws, self.nbytes = _line_workspace(self.frames, self.n, self.K, self.refls[0].device)
        _lib.check(self.lib.tidas_apply_batch_prepare(self.frames, self.n, self.K, ctypes.c_void_p(self.ws.data_ptr()),
                                                      self.nbytes, _stream()))

    def apply(self):
        _lib.check(self.lib.tidas_apply_batch_prepared(self.frames, self.n, self.K,
                                                       ctypes.c_void_p(self.ws.data_ptr()), self.nbytes, _stream()))
        return self.outs
