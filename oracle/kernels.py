"""Per-depth-row kernels of the line model (oracle; test infrastructure only).

Two constructions, both evaluated on the centre line x = 0 from the echo of a
unit scatterer.  The echo is used analytically (FP64, never rounded):
RF1[a][n][k] = p(t0 + k/fs - tau_n(x_s, z_s; a)) for 0 <= k < T, zero
outside, which is exactly what ``simulate.simulate_rf`` returns for one
scatterer of amplitude 1 before its FP32 rounding.

* exact mode (Sec. 2.2, eq:PSF): row i's kernel is the DAS point-spread
  function of a unit scatterer at (0, z_i), sampled at the output depths
  z_i + m dz, m = -h..h:  K[i][m+h] = DAS(RF1_i)(0, z_i + m dz).

* paper mode (Sec. 2.3, eqn:tDAS, eqn:diff, eq:norma, eqn:theta; Sec. 3.1-3.2):
  the receive law (delays and apodization) is frozen at a reference depth
  z_r.  With t(z; a) = tau_tx(0, z; a) + z / c the arrival time at the probe
  centre and D_n(z_r) the delay law of eqn:delay, the fixed-delay line reads

      F_r[S](z) = sum_a sum_n w(-x_n, z_r) * L(S[a][n], (t(z; a) - D_n(z_r) - t0) fs).

  h_r[m] = F_r[RF1 at z_r](z_r + m dz) is the time-invariant kernel; on a fine
  depth axis of spacing dzf = c / (2 fs) (one sample of two-way time)
  a_i = F_r[RF1 at z_i] and b_i = DAS(RF1 at z_i) along x = 0; the window B_i
  is centred on z_i and as wide as the FWHM W_r of the envelope of b_r
  (Sec. 3.1-3.2: the width of the reference PSF at half its maximum); the weight is the least
  squares solution of the first line of eqn:theta,
  theta_i = sum_B a_i b_i / sum_B a_i^2 (its time-domain form, Plancherel);
  finally K[i] = theta_i * h_{r(i)}.

* lateral mode (the separable 2-D extension the conclusion, Sec. 4, leaves
  for future work): row i's lateral kernel is the DAS response of the same
  unit scatterer at (0, z_i) along its own row, normalised by its centre,
      Kx[i][m+h] = DAS(RF1_i)(m dx, z_i) / DAS(RF1_i)(0, z_i)   (0 if the centre is 0),
  so that a depth pass with exact kernels followed by a lateral pass with
  these kernels reproduces DAS along an on-axis scatterer's own row.

* line mode (Sec. 2.4, eqn:line_conv taken literally): the line model is
  Theta times the fixed-delay beamformer of the RF.  By Born linearity its
  exact form on a reflectivity map has, for output row i and source row
  i - m, the kernel K[i][m+h] = theta_i * F_r[RF1 at z_{i-m}](z_i): the
  fixed-delay response of the source scatterer read at the output depth,
  scaled by the output row's weight.  theta_i and r(i) as in paper mode.
"""
import numpy as np

from . import geometry, pulse as pulse_mod


def unit_echo_read(u, tau, t0, fs, fc, sigma, n_samples):
    """L(RF1, u) for the analytic unit echo RF1[k] = p(t0 + k/fs - tau),
    0 <= k < T (zero outside the record); linear interpolation as in DAS."""
    u = np.asarray(u, np.float64)
    q = np.floor(u)
    f = u - q
    T = int(n_samples)
    s0 = np.where((q >= 0) & (q < T), pulse_mod.pulse(t0 + q / fs - tau, fc, sigma), 0.0)
    s1 = np.where((q + 1 >= 0) & (q + 1 < T), pulse_mod.pulse(t0 + (q + 1) / fs - tau, fc, sigma), 0.0)
    return (1.0 - f) * s0 + f * s1


def unit_das(x_pix, z_pix, x_s, z_s, *, n_elem, pitch, c, fs, t0, fc, sigma, n_samples, angles, fnumber):
    """DAS (Sec. 2, eqn:appF) at pixels (x_pix, z_pix) of the RF of a unit
    scatterer at (x_s, z_s) (Sec. 2.2, eq:PSF).  Arguments broadcast."""
    x_pix, z_pix, x_s, z_s = np.broadcast_arrays(*(np.asarray(v, np.float64) for v in (x_pix, z_pix, x_s, z_s)))
    out = np.zeros(x_pix.shape, np.float64)
    for alpha in angles:
        for xn in geometry.element_x(n_elem, pitch):
            w = geometry.hann_apod(x_pix - xn, z_pix, fnumber)
            u = (geometry.arrival_time(x_pix, z_pix, xn, alpha, c) - t0) * fs
            tau = geometry.arrival_time(x_s, z_s, xn, alpha, c)
            out += w * unit_echo_read(u, tau, t0, fs, fc, sigma, n_samples)
    return out


def fixed_delay_line(z_eval, z_ref, z_s, *, n_elem, pitch, c, fs, t0, fc, sigma, n_samples, angles, fnumber):
    """F_r[RF1 at (0, z_s)](z_eval) with the receive law frozen at depth z_ref
    (Sec. 2.3, eqn:tDAS: delays D_n of one point s; Sec. 2.4 fixed delay set D).
    Arguments broadcast."""
    z_eval, z_ref, z_s = np.broadcast_arrays(*(np.asarray(v, np.float64) for v in (z_eval, z_ref, z_s)))
    out = np.zeros(z_eval.shape, np.float64)
    for alpha in angles:
        t_centre = geometry.tau_tx(0.0, z_eval, alpha, c) + z_eval / c
        for xn in geometry.element_x(n_elem, pitch):
            w = geometry.hann_apod(-xn, z_ref, fnumber)
            u = (t_centre - geometry.receive_delay(xn, z_ref, c) - t0) * fs
            tau = geometry.arrival_time(0.0, z_s, xn, alpha, c)
            out += w * unit_echo_read(u, tau, t0, fs, fc, sigma, n_samples)
    return out


def exact_kernels(z_rows, dz, K, **setup):
    """Exact-mode kernel bank [Z][K]: K[i][m+h] = DAS(RF1_i)(0, z_i + m dz)."""
    h = (K - 1) // 2
    z = np.asarray(z_rows, np.float64)[:, None]
    m = np.arange(-h, h + 1, dtype=np.float64)[None, :]
    return unit_das(0.0, z + m * dz, 0.0, z, **setup)


def envelope(x):
    """|analytic signal| of a real sequence: FFT, zero-padded to the first power
    of two >= 2 len(x); keep DC and Nyquist, double positive frequencies,
    drop negative ones; inverse FFT."""
    x = np.asarray(x, np.float64)
    L = x.size
    N = 1
    while N < 2 * L:
        N *= 2
    X = np.fft.fft(x, N)
    H = np.zeros(N)
    H[0] = 1.0
    H[1:N // 2] = 2.0
    H[N // 2] = 1.0
    return np.abs(np.fft.ifft(X * H)[:L])


def fwhm(env, step):
    """Full width at half maximum of a sampled envelope: from the (first)
    maximum walk outwards to the first samples below half the maximum and
    interpolate the crossings linearly; an axis end with no crossing counts
    as the crossing.  Returned in units of ``step``."""
    env = np.asarray(env, np.float64)
    L = env.size
    p = int(np.argmax(env))
    half = 0.5 * env[p]
    lo = p
    while lo > 0 and env[lo - 1] >= half:
        lo -= 1
    x_left = float(lo) if lo == 0 else (lo - 1) + (half - env[lo - 1]) / (env[lo] - env[lo - 1])
    hi = p
    while hi < L - 1 and env[hi + 1] >= half:
        hi += 1
    x_right = float(hi) if hi == L - 1 else hi + (env[hi] - half) / (env[hi] - env[hi + 1])
    return (x_right - x_left) * step


def theta_ls(a, b):
    """Least-squares weight of eqn:theta (first line) in the time domain:
    argmin_t ||t a - b||^2 = <a, b> / <a, a>, and 0 when <a, a> = 0."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = float(np.dot(a, a))
    return float(np.dot(a, b)) / den if den > 0 else 0.0


def theta_frequency(a, b):
    """eqn:theta first line evaluated literally in the frequency domain:
    int (conj(a) b + a conj(b)) df / (2 int |a|^2 df), on zero-padded DFTs."""
    n = 2 * max(len(a), len(b))
    A = np.fft.fft(np.asarray(a, np.float64), n)
    B = np.fft.fft(np.asarray(b, np.float64), n)
    num = np.sum(np.conj(A) * B + A * np.conj(B)).real
    den = 2.0 * np.sum(np.abs(A) ** 2)
    return float(num / den) if den > 0 else 0.0


def lateral_kernels(z_rows, dx, K, **setup):
    """Lateral-mode kernel bank [Z][K]: Kx[i][m+h] = DAS(RF1_i)(m dx, z_i) / DAS(RF1_i)(0, z_i)."""
    h = (K - 1) // 2
    z = np.asarray(z_rows, np.float64)[:, None]
    m = np.arange(-h, h + 1, dtype=np.float64)[None, :]
    prof = unit_das(m * dx, z, 0.0, z, **setup)
    centre = prof[:, h:h + 1]
    safe = np.where(centre != 0.0, centre, 1.0)
    return np.where(centre != 0.0, prof / safe, 0.0)


def fine_half_length(fs, sigma):
    """Half length Qf (in fine-axis samples) of the axis on which the envelope
    FWHM is measured: twice the pulse support, ceil(8 sigma fs)."""
    return int(np.ceil(2.0 * pulse_mod.TRUNC_SIGMAS * sigma * fs))


def fixed_delay_beamform(rf, z_eval, z_ref, *, n_elem, pitch, c, fs, t0, angles, fnumber):
    """The fixed-delay line of Sec. 2.3 / 2.4 applied to sampled RF [A][C][T]
    on the centre line: sum_a sum_n w(-x_n, z_ref) L(RF[a][n], (t(z; a) - D_n(z_ref) - t0) fs)."""
    rf = np.asarray(rf, np.float64)
    z_eval = np.asarray(z_eval, np.float64)
    out = np.zeros(z_eval.shape, np.float64)
    from .das import lerp_read
    for ai, alpha in enumerate(angles):
        t_centre = geometry.tau_tx(0.0, z_eval, alpha, c) + z_eval / c
        for n, xn in enumerate(geometry.element_x(n_elem, pitch)):
            w = geometry.hann_apod(-xn, z_ref, fnumber)
            u = (t_centre - geometry.receive_delay(xn, z_ref, c) - t0) * fs
            out += w * lerp_read(rf[ai, n], u)
    return out


def paper_kernels(z_rows, dz, K, ref_rows=None, line=False, **setup):
    """Paper-mode kernel bank [Z][K] and weights theta [Z].

    ref_rows[i] is the row whose depth supplies the frozen receive law for
    row i (default: the row itself).  line=True gives the line-mode bank
    (theta_i times the fixed-delay response of each source row at row i)
    instead of theta_i times the reference response h_r.  Returns
    (kernels, theta, widths) with widths[i] = W_{r(i)} the FWHM window width
    in metres.
    """
    z_rows = np.asarray(z_rows, np.float64)
    Z = z_rows.size
    h = (K - 1) // 2
    c, fs = setup["c"], setup["fs"]
    ref_rows = np.arange(Z) if ref_rows is None else np.asarray(ref_rows, np.int64)
    dzf = c / (2.0 * fs)
    Qf = fine_half_length(fs, setup["sigma"])
    q_axis = np.arange(-Qf, Qf + 1, dtype=np.float64)
    m_axis = np.arange(-h, h + 1, dtype=np.float64)

    h_ref, w_ref = {}, {}
    for r in np.unique(ref_rows):
        zr = z_rows[r]
        h_ref[r] = fixed_delay_line(zr + m_axis * dz, zr, zr, **setup)
        b_r = unit_das(0.0, zr + q_axis * dzf, 0.0, zr, **setup)
        w_ref[r] = fwhm(envelope(b_r), dzf)

    kernels = np.zeros((Z, K), np.float64)
    theta = np.zeros(Z, np.float64)
    widths = np.zeros(Z, np.float64)
    for i in range(Z):
        r = int(ref_rows[i])
        W = w_ref[r]
        qmax = int(np.floor(0.5 * W / dzf))
        zq = z_rows[i] + np.arange(-qmax, qmax + 1, dtype=np.float64) * dzf
        a = fixed_delay_line(zq, z_rows[r], z_rows[i], **setup)
        b = unit_das(0.0, zq, 0.0, z_rows[i], **setup)
        theta[i] = theta_ls(a, b)
        if line:
            kernels[i] = theta[i] * fixed_delay_line(z_rows[i], z_rows[r], z_rows[i] - m_axis * dz, **setup)
        else:
            kernels[i] = theta[i] * h_ref[r]
        widths[i] = W
    return kernels, theta, widths
