"""Delay-and-Sum beamforming (oracle; test infrastructure only).

Sec. 2, eqn:appF: g(r) = sum_{n in N} S_n * delta_{D_n(r)} -- every image
point gets its own delay profile (dynamic focusing).  With plane-wave
transmits, a Hann F-number receive aperture and linear interpolation of the
sampled channel data (readings recorded with the design), the image is

    I[i][j] = sum_a sum_n w(x_j - x_n, z_i) * L(RF[a][n], (tau_n(x_j, z_i; a) - t0) * fs)

with L the linear-interpolation read of ``lerp_read`` (zero outside the
record) and w the apodization of ``geometry.hann_apod``.

The time-invariant beamformer of the paper (Sec. 2.3 eqn:tDAS: the delays of
one point applied to a whole line; Sec. 2.4 eqn:line_conv: a convolution with
fixed parameters scaled by Theta) is the same read with the receive law frozen:
row i uses the delays D_n and the weights of its reference row r = r(i), in
every column, and is scaled by theta_i:

    I[i][j] = theta_i sum_a sum_n w(x_j - x_n, z_r) *
              L(RF[a][n], (tau_tx(x_j, z_i; a) + z_i / c - D_n(x_j, z_r) - t0) * fs)

with D_n(x, z) = (z - rho_n(x, z)) / c, the delay law of eqn:delay at lateral
position x.  With r(i) = i and theta = 1 it is DAS.
"""
import math

import numpy as np

from . import geometry


def lerp_read(S, u):
    """L(S, u) = (1 - f) S[q] + f S[q + 1], q = floor(u), f = u - q, with
    S[k] = 0 for k outside [0, T-1].  S is 1-D, u any shape."""
    S = np.asarray(S, np.float64)
    T = S.shape[-1]
    u = np.asarray(u, np.float64)
    q = np.floor(u)
    f = u - q
    q = q.astype(np.int64)
    s0 = np.where((q >= 0) & (q < T), S[np.clip(q, 0, T - 1)], 0.0)
    s1 = np.where((q + 1 >= 0) & (q + 1 < T), S[np.clip(q + 1, 0, T - 1)], 0.0)
    return (1.0 - f) * s0 + f * s1


def das(rf, xs, zs, n_elem, pitch, c, fs, t0, angles, fnumber):
    """Vectorised FP64 DAS.  rf [A][C][T]; xs [X], zs [Z] pixel centres.
    Returns the image [Z][X] (depth-row major)."""
    rf = np.asarray(rf, np.float64)
    xn_all = geometry.element_x(n_elem, pitch)
    X, Z = np.meshgrid(np.asarray(xs, np.float64), np.asarray(zs, np.float64))
    img = np.zeros(Z.shape, np.float64)
    for ai, alpha in enumerate(angles):
        ttx = geometry.tau_tx(X, Z, alpha, c)
        for n, xn in enumerate(xn_all):
            w = geometry.hann_apod(X - xn, Z, fnumber)
            u = (ttx + geometry.rho(X, Z, xn) / c - t0) * fs
            img += w * lerp_read(rf[ai, n], u)
    return img


def fixed_delay_das(rf, xs, zs, ref_rows, n_elem, pitch, c, fs, t0, angles, fnumber, theta=None):
    """FP64 fixed-delay (time-invariant) beamformer over the whole grid.
    rf [A][C][T]; xs [X], zs [Z]; ref_rows [Z] row indices; theta [Z] or None
    (ones).  Returns the image [Z][X]."""
    rf = np.asarray(rf, np.float64)
    xs = np.asarray(xs, np.float64)
    zs = np.asarray(zs, np.float64)
    ref_rows = np.asarray(ref_rows, np.int64)
    if ref_rows.shape != zs.shape or np.any(ref_rows < 0) or np.any(ref_rows >= zs.size):
        raise ValueError("ref_rows must hold one row index in [0, Z) per row")
    xn_all = geometry.element_x(n_elem, pitch)
    X, Zi = np.meshgrid(xs, zs)
    Zr = np.meshgrid(xs, zs[ref_rows])[1]
    img = np.zeros(Zi.shape, np.float64)
    for ai, alpha in enumerate(angles):
        t_line = geometry.tau_tx(X, Zi, alpha, c) + Zi / c
        for n, xn in enumerate(xn_all):
            w = geometry.hann_apod(X - xn, Zr, fnumber)
            u = (t_line - geometry.receive_delay(xn - X, Zr, c) - t0) * fs
            img += w * lerp_read(rf[ai, n], u)
    if theta is not None:
        img *= np.asarray(theta, np.float64)[:, None]
    return img


def das_bruteforce(rf, xs, zs, n_elem, pitch, c, fs, t0, angles, fnumber):
    """The same definition as four nested pure-Python loops with the math
    module, for tiny grids (used to pin ``das``)."""
    A, C, T = len(rf), len(rf[0]), len(rf[0][0])
    img = [[0.0] * len(xs) for _ in zs]
    for i, z in enumerate(zs):
        for j, x in enumerate(xs):
            acc = 0.0
            for a in range(A):
                alpha = angles[a]
                for n in range(C):
                    xn = (n - (C - 1) / 2.0) * pitch
                    half = z / (2.0 * fnumber)
                    d = x - xn
                    if half <= 0 or abs(d) > half:
                        continue
                    w = 0.5 * (1.0 + math.cos(math.pi * d / half))
                    tau = (x * math.sin(alpha) + z * math.cos(alpha)) / c + math.sqrt(d * d + z * z) / c
                    u = (tau - t0) * fs
                    q = math.floor(u)
                    f = u - q
                    s0 = float(rf[a][n][q]) if 0 <= q < T else 0.0
                    s1 = float(rf[a][n][q + 1]) if 0 <= q + 1 < T else 0.0
                    acc += w * ((1.0 - f) * s0 + f * s1)
            img[i][j] = acc
    return np.array(img, np.float64)
