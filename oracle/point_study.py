"""The paper's single-point study (oracle; test infrastructure only).

Sec. 2.1 analyses an unsteered beam focused on the probe axis; Sec. 3.1 sets
up the study: an axial line of points, a transmit aperture sized by
Kossoff's criterion, a receive aperture of fixed F-number, one of the points
taken as the transmit focus, and the FWHM of the DAS PSF at that focus as the
correction window.  Sec. 3.3 then reconstructs a unit scatterer at every
point s with DAS and with the fixed delay curve of every point r, giving the
weight matrix Theta[r][s] (eqn:theta) and the local (near the peak) and
global (whole line) squared errors; Sec. 3.2 compares peak heights and FWHMs
of DAS and tiDAS along the line for the focal point's delay curve.

Readings (the paper leaves these open):
* Transmit: the n_tx centremost elements fire with focusing delays
  T_m = (z_f - sqrt(x_m^2 + z_f^2)) / c, so every element's wave reaches the
  focus (0, z_f) at z_f / c; uniform transmit weights.  On the axis the
  beamformer takes the transmit arrival as z / c (a virtual source at the
  focus, exact at the focus).
* Kossoff's criterion with parameter 0.6: the aperture width D for which the
  focal depth is 0.6 of the aperture's near-field length D^2 / (4 lambda),
  D = sqrt(4 lambda z_f / 0.6), lambda = c / fc; n_tx = D / pitch rounded to
  the nearest count with the parity of C (so the set is symmetric), clamped
  to [1 or 2, C].
* Receive: the library's Hann aperture of half width z / (2 F).
* Lines: the fine axis z_s + q dzf (dzf = c / (2 fs), one RF sample of
  two-way time), q in [-Ql, Ql], centred on the scatterer; the window B is
  |q| <= floor(W / (2 dzf)) with W the FWHM of the envelope of the DAS line
  of the focal point's scatterer on |q| <= Qf (as for the paper-mode
  kernels); the global error runs over the whole line |q| <= Ql.
* Errors: ||theta a - b||^2 / ||b||^2 over B (local) and over the line
  (global), 0 where ||b|| = 0; peak heights are envelope maxima, FWHMs those
  of the envelopes, both on |q| <= Qh.

The echo of a unit scatterer at (0, z_s) is synthesised in float64 on the RF
sample grid (never rounded):
  RF_s[n][k] = sum_{m in TX} p(t0 + k/fs - T_m - rho_m(z_s)/c - rho_n(z_s)/c),
zero outside 0 <= k < T, and read with the library's linear interpolation.
"""
import numpy as np

from . import geometry, kernels as kern_mod, pulse as pulse_mod
from .das import lerp_read

KOSSOFF_RATIO = 0.6


def kossoff_tx_count(n_elem, pitch, c, fc, z_focus, ratio=KOSSOFF_RATIO):
    """Transmit element count for focal depth z_focus (Sec. 3.1, Kossoff's
    criterion read as z_f = ratio * D^2 / (4 lambda))."""
    lam = c / fc
    width = np.sqrt(4.0 * lam * z_focus / ratio)
    par = int(n_elem) % 2
    n = par + 2 * int(np.floor((width / pitch - par) / 2.0 + 0.5))
    smallest = 1 if par else 2
    return int(min(max(n, smallest), int(n_elem)))


def tx_elements(n_elem, pitch, n_tx):
    """Lateral positions of the n_tx centremost elements (a set symmetric
    about the probe centre; n_elem - n_tx must be even)."""
    if (int(n_elem) - int(n_tx)) % 2:
        raise ValueError("n_elem - n_tx must be even")
    x = geometry.element_x(n_elem, pitch)
    first = (int(n_elem) - int(n_tx)) // 2
    return x[first:first + int(n_tx)]


def tx_fire_times(x_tx, z_focus, c):
    """Focusing delays: element m fires at T_m so that its wave reaches the
    focus at z_f / c (Sec. 2.1: a beam focused on the axis)."""
    x_tx = np.asarray(x_tx, np.float64)
    return (z_focus - np.sqrt(x_tx ** 2 + z_focus ** 2)) / c


def focused_echo(z_s, *, n_elem, pitch, c, fs, t0, fc, sigma, n_samples, z_focus, n_tx):
    """RF [C][T] of a unit scatterer at (0, z_s) under the focused transmit."""
    xn = geometry.element_x(n_elem, pitch)
    xm = tx_elements(n_elem, pitch, n_tx)
    Tm = tx_fire_times(xm, z_focus, c)
    t = t0 + np.arange(int(n_samples), dtype=np.float64) / fs
    rx = np.sqrt(xn ** 2 + z_s ** 2) / c                      # [C]
    tx = Tm + np.sqrt(xm ** 2 + z_s ** 2) / c                  # [M]
    rf = np.zeros((xn.size, t.size), np.float64)
    for m in range(xm.size):
        rf += pulse_mod.pulse(t[None, :] - tx[m] - rx[:, None], fc, sigma)
    return rf


def das_line(rf, z, *, n_elem, pitch, c, fs, t0, fnumber):
    """DAS (Sec. 2, eqn:appF) of RF [C][T] on the probe axis at depths z:
    transmit arrival z / c, dynamic receive delays and aperture."""
    z = np.asarray(z, np.float64)
    out = np.zeros(z.shape, np.float64)
    for n, xn in enumerate(geometry.element_x(n_elem, pitch)):
        w = geometry.hann_apod(-xn, z, fnumber)
        u = (z / c + geometry.rho(0.0, z, xn) / c - t0) * fs
        out += w * lerp_read(rf[n], u)
    return out


def fixed_delay_line(rf, z, z_ref, *, n_elem, pitch, c, fs, t0, fnumber):
    """The time-invariant line of Sec. 2.3 (eqn:tDAS) on the probe axis: the
    receive delays D_n(z_ref) (eqn:delay) and the aperture of depth z_ref
    serve every depth z; read time 2 z / c - D_n(z_ref)."""
    z = np.asarray(z, np.float64)
    out = np.zeros(z.shape, np.float64)
    for n, xn in enumerate(geometry.element_x(n_elem, pitch)):
        w = geometry.hann_apod(-xn, z_ref, fnumber)
        u = (2.0 * z / c - geometry.receive_delay(xn, z_ref, c) - t0) * fs
        out += w * lerp_read(rf[n], u)
    return out


def _rel_sq(u, v):
    den = float(np.sum(v * v))
    return float(np.sum((u - v) ** 2)) / den if den > 0 else 0.0


def study_axis(n_points, z_first, z_step):
    return float(z_first) + np.arange(int(n_points), dtype=np.float64) * float(z_step)


def window_width(setup, z_points, focal_index):
    """W: FWHM of the envelope of the focal point's DAS PSF (Sec. 3.1-3.2)."""
    c, fs = setup["c"], setup["fs"]
    dzf = c / (2.0 * fs)
    Qf = kern_mod.fine_half_length(fs, setup["sigma"])
    zf = z_points[focal_index]
    rf = focused_echo(zf, z_focus=zf, **_echo_args(setup))
    b = das_line(rf, zf + np.arange(-Qf, Qf + 1) * dzf, **_line_args(setup))
    return kern_mod.fwhm(kern_mod.envelope(b), dzf)


def _echo_args(setup):
    keys = ("n_elem", "pitch", "c", "fs", "t0", "fc", "sigma", "n_samples", "n_tx")
    return {k: setup[k] for k in keys}


def _line_args(setup):
    keys = ("n_elem", "pitch", "c", "fs", "t0", "fnumber")
    return {k: setup[k] for k in keys}


def study(setup, n_points, z_first, z_step, focal_index, line_half, refs=None, points=None, stats_half=None):
    """Theta[r][s], local and global squared errors [r][s] (Sec. 3.3) for the
    delay curves of points ``refs`` and the scatterers at points ``points``
    (default: all), the window width W, and (stats_half given) per scatterer
    the peak heights and FWHMs of DAS and of tiDAS with the focal point's
    delay curve (Sec. 3.2), each [4] = (DAS peak, tiDAS peak, DAS FWHM,
    tiDAS FWHM).  ``setup`` holds n_elem, pitch, c, fs, t0, fc, sigma,
    n_samples, fnumber and n_tx."""
    zp = study_axis(n_points, z_first, z_step)
    refs = list(range(n_points)) if refs is None else list(refs)
    points = list(range(n_points)) if points is None else list(points)
    c, fs = setup["c"], setup["fs"]
    dzf = c / (2.0 * fs)
    zf = zp[focal_index]
    W = window_width(setup, zp, focal_index)
    Qw = int(np.floor(0.5 * W / dzf))
    q = np.arange(-int(line_half), int(line_half) + 1, dtype=np.float64)
    in_B = np.abs(q) <= Qw
    theta = np.zeros((len(refs), len(points)))
    local = np.zeros_like(theta)
    glob = np.zeros_like(theta)
    stats = np.zeros((len(points), 4)) if stats_half is not None else None
    for j, s in enumerate(points):
        rf = focused_echo(zp[s], z_focus=zf, **_echo_args(setup))
        z = zp[s] + q * dzf
        b = das_line(rf, z, **_line_args(setup))
        for i, r in enumerate(refs):
            a = fixed_delay_line(rf, z, zp[r], **_line_args(setup))
            th = kern_mod.theta_ls(a[in_B], b[in_B])
            theta[i, j] = th
            local[i, j] = _rel_sq(th * a[in_B], b[in_B])
            glob[i, j] = _rel_sq(th * a, b)
        if stats is not None:
            Qh = int(stats_half)
            qh = np.arange(-Qh, Qh + 1, dtype=np.float64)
            zh = zp[s] + qh * dzf
            bh = das_line(rf, zh, **_line_args(setup))
            ah = fixed_delay_line(rf, zh, zf, **_line_args(setup))
            zB = zp[s] + q[in_B] * dzf
            th = kern_mod.theta_ls(fixed_delay_line(rf, zB, zf, **_line_args(setup)),
                                   das_line(rf, zB, **_line_args(setup)))
            eb, ea = kern_mod.envelope(bh), kern_mod.envelope(th * ah)
            stats[j] = (eb.max(), ea.max(), kern_mod.fwhm(eb, dzf), kern_mod.fwhm(ea, dzf))
    return theta, local, glob, W, stats
