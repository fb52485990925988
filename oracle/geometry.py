"""Geometry and delay law (oracle; test infrastructure only).

Linear probe with element centres (x_n, 0) on a set N symmetric about the
probe centre (Sec. 2, definition of N; Sec. 2.1, element centres).  Image
points are r = (x, z) with z the depth.  All values SI (m, s), float64.
"""
import numpy as np


def element_x(n_elem, pitch):
    """Element centres x_n = (n - (C-1)/2) * pitch, n = 0..C-1.

    The active set of Sec. 2 is symmetric about the probe centre; element n of
    the C elements sits at that lateral coordinate.
    """
    n = np.arange(n_elem, dtype=np.float64)
    return (n - (n_elem - 1) / 2.0) * float(pitch)


def axis(n, start, step):
    """Pixel-centre coordinates start + k * step, k = 0..n-1."""
    return float(start) + np.arange(n, dtype=np.float64) * float(step)


def tau_tx(x, z, alpha, c):
    """Plane-wave transmit time: the front crosses (0, 0) at t = 0 and travels
    along direction angle alpha, so it reaches (x, z) at (x sin a + z cos a)/c.

    The paper analyses a focused, unsteered transmit (Sec. 2.1); the
    workloads here use plane waves, the reading recorded with the design.
    """
    return (np.asarray(x, np.float64) * np.sin(alpha) + np.asarray(z, np.float64) * np.cos(alpha)) / c


def rho(x, z, xn):
    """Receive path length from (x, z) back to the element centre (x_n, 0)."""
    x = np.asarray(x, np.float64)
    z = np.asarray(z, np.float64)
    return np.sqrt((x - xn) ** 2 + z ** 2)


def arrival_time(x, z, xn, alpha, c):
    """Two-way time of flight tau_n(x, z; alpha) = tau_tx + rho_n / c."""
    return tau_tx(x, z, alpha, c) + rho(x, z, xn) / c


def receive_delay(xn, z, c):
    """Receive delay law on the centre line, Sec. 2.1 eqn:delay:
    D_n(z) = (z - sqrt(x_n^2 + z^2)) / c.  At lateral position x the same law
    with x_n - x in place of x_n."""
    z = np.asarray(z, np.float64)
    return (z - np.sqrt(np.asarray(xn, np.float64) ** 2 + z ** 2)) / c


def hann_apod(d, z, fnumber):
    """Receive apodization: Hann window over the F-number aperture.

    The receive aperture keeps a fixed F-number (Sec. 3.1), i.e. a half width
    a_z = z / (2 F) at depth z.  Weight 0.5 (1 + cos(pi d / a_z)) for
    |d| <= a_z, zero outside and zero where a_z <= 0.  Not normalised.
    """
    d = np.asarray(d, np.float64)
    z = np.asarray(z, np.float64)
    a = z / (2.0 * fnumber)
    safe = np.where(a > 0, a, 1.0)
    w = 0.5 * (1.0 + np.cos(np.pi * d / safe))
    return np.where((a > 0) & (np.abs(d) <= a), w, 0.0)
