"""Born-approximation RF synthesis (oracle; test infrastructure only).

Sec. 2, eqn:SRX: the echo of a scatterer at r recorded by element n is its
reflectivity times the transmitted signal, convolved with the element
response.  Under the Born approximation (Sec. 2, multiple scattering
neglected) the echoes of many scatterers add linearly.  Point elements, no
attenuation or spreading (the element response H_n is left unspecified in
the paper), so

    RF[a][n][k] = sum_s A_s * p(t0 + k / fs - tau_n(x_s, z_s; a))

with tau_n the two-way time of flight of ``geometry.arrival_time``.
"""
import numpy as np

from . import geometry, pulse as pulse_mod


def simulate_rf(sx, sz, amp, n_elem, pitch, c, fs, t0, fc, sigma, n_samples, angles):
    """FP64 RF channel data, shape [A][C][T].

    sx, sz, amp: scatterer lateral position, depth and amplitude (1-D arrays).
    """
    sx = np.asarray(sx, np.float64).ravel()
    sz = np.asarray(sz, np.float64).ravel()
    amp = np.asarray(amp, np.float64).ravel()
    xn_all = geometry.element_x(n_elem, pitch)
    T = int(n_samples)
    out = np.zeros((len(angles), n_elem, T), np.float64)
    half = pulse_mod.TRUNC_SIGMAS * sigma
    width = int(np.ceil(2.0 * half * fs)) + 2
    offs = np.arange(width)
    chunk = max(1, 2_000_000 // width)
    for ai, alpha in enumerate(angles):
        for n, xn in enumerate(xn_all):
            acc = np.zeros(T, np.float64)
            for s0 in range(0, sx.size, chunk):
                tau = geometry.arrival_time(sx[s0:s0 + chunk], sz[s0:s0 + chunk], xn, alpha, c)
                k_lo = np.ceil((tau - half - t0) * fs).astype(np.int64)
                k = k_lo[:, None] + offs[None, :]
                t = t0 + k / fs - tau[:, None]
                val = amp[s0:s0 + chunk, None] * pulse_mod.pulse(t, fc, sigma)
                keep = (k >= 0) & (k < T)
                acc += np.bincount(k[keep], weights=val[keep], minlength=T)[:T]
            out[ai, n] = acc
    return out


def to_fp32(rf):
    """Round FP64 RF to FP32 (round to nearest even), the stored sample format."""
    return np.asarray(rf, np.float64).astype(np.float32)
