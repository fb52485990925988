"""Kernel-surrogate MLP (oracle; test infrastructure only).

Not part of the paper: a small network mapping normalised (depth, F-number,
steering angle, centre frequency) to a row kernel of the line model.  The
paper's conclusion treats the weights Theta as learned quantities; this
network learns the whole row kernel instead.

Architecture: four linear layers 4 -> 256 -> 256 -> 256 -> K with GELU
G(u) = u/2 (1 + erf(u / sqrt 2)) after the first three.  Weights W_l are
[out][in] (row-major), biases b_l [out].  Loss: mean squared error over
batch and outputs.  Optimiser: Adam with bias correction.

Two arithmetic modes:
* ``bf16=False``: plain float64 throughout.
* ``bf16=True``: the GEMM operands are rounded to bfloat16 (round to nearest
  even) exactly where the device kernels round them -- the input x, every
  weight matrix, each hidden activation before the next GEMM, and each
  back-propagated gradient before its GEMMs -- while sums, biases, GELU and
  its derivative stay in float64 (the device accumulates in float32).
"""
import numpy as np
from scipy.special import erf

SQRT2 = np.sqrt(2.0)
INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)


def kernel_scale(z, fnumber, n_elem, pitch):
    """Normaliser of a row kernel: max(sum_n w(-x_n, z), 1), the aperture's
    Hann weight sum (the centre tap of an unsteered exact kernel is this sum
    times the pulse peak, up to interpolation), floored at 1."""
    from . import geometry
    w = geometry.hann_apod(-geometry.element_x(n_elem, pitch), z, fnumber)
    return max(float(np.sum(w)), 1.0)


def features(params, lo, hi):
    """Affine map of each parameter column onto [-1, 1]."""
    params = np.asarray(params, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    return 2.0 * (params - lo) / (hi - lo) - 1.0


def bf16(v):
    """Round to bfloat16 (8 significant bits, round to nearest even), returned
    as float64.  The value is first rounded to float32 (the device rounds
    float32 values)."""
    f = np.asarray(v, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def gelu(u):
    return 0.5 * u * (1.0 + erf(u / SQRT2))


def gelu_grad(u):
    return 0.5 * (1.0 + erf(u / SQRT2)) + u * INV_SQRT_2PI * np.exp(-0.5 * u * u)


def forward(params, x, bf16_mode=True):
    """params: list of (W, b) for the four layers.  x [N][4].
    Returns (y [N][K], cache for ``backward``)."""
    rnd = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    h = rnd(x)
    cache = {"h": [h], "z": [], "W": []}
    L = len(params)
    for l, (W, b) in enumerate(params):
        Wr = rnd(W)
        z = h @ Wr.T + np.asarray(b, np.float64)
        cache["W"].append(Wr)
        cache["z"].append(z)
        if l < L - 1:
            h = rnd(gelu(z))
            cache["h"].append(h)
        else:
            y = z
    return y, cache


def loss(y, t):
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(d * d))


def backward(cache, y, t, bf16_mode=True):
    """Gradients of ``loss`` w.r.t. every (W, b), as a list of (dW, db)."""
    rnd = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    y = np.asarray(y, np.float64)
    g = 2.0 * (y - np.asarray(t, np.float64)) / y.size
    L = len(cache["W"])
    grads = [None] * L
    for l in range(L - 1, -1, -1):
        gr = rnd(g)
        dW = gr.T @ cache["h"][l]
        db = g.sum(axis=0)
        grads[l] = (dW, db)
        if l > 0:
            gh = gr @ cache["W"][l]
            g = gh * gelu_grad(cache["z"][l - 1])
    return grads


def adam_step(params, grads, state, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected, step counted from 1) of FP64 master
    weights.  state: list of (mW, vW, mb, vb).  Returns new params and state."""
    new_p, new_s = [], []
    c1 = 1.0 - beta1 ** step
    c2 = 1.0 - beta2 ** step
    for (W, b), (dW, db), (mW, vW, mb, vb) in zip(params, grads, state):
        out = []
        for P, G, M, V in ((W, dW, mW, vW), (b, db, mb, vb)):
            M = beta1 * M + (1.0 - beta1) * G
            V = beta2 * V + (1.0 - beta2) * G * G
            P = P - lr * (M / c1) / (np.sqrt(V / c2) + eps)
            out.append((P, M, V))
        (W2, mW2, vW2), (b2, mb2, vb2) = out
        new_p.append((W2, b2))
        new_s.append((mW2, vW2, mb2, vb2))
    return new_p, new_s


def cosine_lr(step, total, lr0=1e-3, lr1=1e-5):
    """Cosine decay from lr0 at step 0 to lr1 at step ``total``."""
    f = min(max(step / float(total), 0.0), 1.0)
    return lr1 + 0.5 * (lr0 - lr1) * (1.0 + np.cos(np.pi * f))
