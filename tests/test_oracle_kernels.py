"""Pins of the oracle's kernel construction: exact DAS PSF kernels
(Sec. 2.2 eq:PSF), paper-mode fixed-delay + theta kernels (Sec. 2.3
eqn:tDAS, eqn:theta; Sec. 3.1-3.2 FWHM window) and the lateral kernels of the
separable 2-D extension, with its lateral pass."""
import numpy as np
import pytest

from oracle import das, kernels, pulse, simulate, tidas
from workloads import config
from tests.helpers import das_kw, sim_kw, oracle_kw

C1 = config(1)


def test_exact_kernel_rows_equal_das_of_materialised_echo():
    """The analytic unit-echo path equals RF synthesis (FP64) followed by DAS at
    the pixels (0, z_i + m dz)."""
    s = C1.replace(n_samples=1500, angles=(-0.06, 0.0, 0.1))
    K = 9
    h = (K - 1) // 2
    zr = np.array([4.1e-3, 11.37e-3, 17.9e-3])
    kb = kernels.exact_kernels(zr, s.dz, K, **oracle_kw(s))
    for i, z in enumerate(zr):
        rf = simulate.simulate_rf([0.0], [z], [1.0], **sim_kw(s))
        col = das.das(rf, [0.0], z + np.arange(-h, h + 1) * s.dz, **das_kw(s))[:, 0]
        assert np.max(np.abs(kb[i] - col)) <= 1e-13 * np.max(np.abs(col))
        # centre tap = DAS value at the scatterer's own pixel
        assert abs(kb[i, h] - col[h]) <= 1e-13 * abs(col[h])


def test_exact_kernel_single_element_sample_aligned_is_sampled_pulse():
    """C = 1, unsteered, dz and z_i on the sample grid: every read falls on a
    sample, so K[i][m+h] = p(2 m dz / c)."""
    s = C1.replace(n_elem=1, n_samples=4000)
    dz = 3 * s.c / (2 * s.fs)
    K = 21
    h = 10
    zr = np.array([200, 517, 1300]) * s.c / (2 * s.fs)
    kb = kernels.exact_kernels(zr, dz, K, **oracle_kw(s))
    ref = pulse.pulse(2 * np.arange(-h, h + 1) * dz / s.c, s.fc, s.sigma)
    assert np.max(np.abs(kb - ref[None, :])) < 1e-13


def pythagorean_setup():
    """Two elements at x = +-30 l with l = c / fs; at reference depths 40 l and
    72 l the receive distances are 50 l and 78 l (Pythagorean triples), so
    every fractional sample index is an integer."""
    s = C1.replace(n_elem=2, n_samples=4000, fnumber=0.5)
    ell = s.c / s.fs
    s = s.replace(pitch=60 * ell)
    return s, ell


def test_paper_kernel_fixed_delay_response_is_pure_pulse_exact_case():
    s, ell = pythagorean_setup()
    dz = ell / 2                           # one sample of two-way time
    K = 15
    h = 7
    for zr in (40 * ell, 72 * ell):
        hr = kernels.fixed_delay_line(zr + np.arange(-h, h + 1) * dz, zr, zr, **oracle_kw(s))
        from oracle import geometry
        wsum = np.sum(geometry.hann_apod(-geometry.element_x(2, s.pitch), zr, s.fnumber))
        ref = wsum * pulse.pulse(2 * np.arange(-h, h + 1) * dz / s.c, s.fc, s.sigma)
        assert wsum > 0
        assert np.max(np.abs(hr - ref)) < 1e-13


def test_paper_kernel_general_case_pulse_up_to_lerp_error():
    """With arbitrary phases the fixed-delay response of the reference
    scatterer is the pulse up to the linear-interpolation error
    (bounded by (pi fc / fs)^2 / 2 relative to the peak)."""
    s = C1
    K = 65
    h = 32
    zr = 21.3e-3
    hr = kernels.fixed_delay_line(zr + np.arange(-h, h + 1) * s.dz, zr, zr, **oracle_kw(s))
    from oracle import geometry
    wsum = np.sum(geometry.hann_apod(-geometry.element_x(s.n_elem, s.pitch), zr, s.fnumber))
    ref = wsum * pulse.pulse(2 * np.arange(-h, h + 1) * s.dz / s.c, s.fc, s.sigma)
    bound = 0.5 * (np.pi * s.fc / s.fs) ** 2
    assert np.max(np.abs(hr - ref)) <= bound * wsum
    assert np.max(np.abs(hr - ref)) > 0


def test_theta_time_domain_equals_frequency_domain():
    """Plancherel (Sec. 2.3): the time-domain least-squares weight equals the
    first line of eqn:theta evaluated on DFTs."""
    rng = np.random.default_rng(5)
    for n in (1, 7, 64, 101):
        a = rng.standard_normal(n)
        b = rng.standard_normal(n) + 0.7 * a
        assert abs(kernels.theta_ls(a, b) - kernels.theta_frequency(a, b)) < 1e-12 * max(1, abs(kernels.theta_ls(a, b)))


def test_theta_properties():
    rng = np.random.default_rng(6)
    a = rng.standard_normal(33)
    b = rng.standard_normal(33)
    t = kernels.theta_ls(a, b)
    assert abs(kernels.theta_ls(a, 3.5 * b) - 3.5 * t) < 1e-12
    assert abs(kernels.theta_ls(a, a) - 1.0) < 1e-15
    assert kernels.theta_ls(np.zeros(5), b[:5]) == 0.0

    def J(th):
        return np.sum((th * a - b) ** 2)
    for d in (1e-3, 0.1, 1.0):
        assert J(t + d) >= J(t) and J(t - d) >= J(t)


def test_fwhm_exact_on_triangle_and_gaussian_envelope():
    # triangle of height 1 (peak on a sample) and half base 10.6: FWHM = 10.6
    # exactly, the crossings fall between samples on the linear pieces
    x = np.arange(-30, 31, dtype=float)
    tri = np.maximum(0.0, 1.0 - np.abs(x) / 10.6)
    assert abs(kernels.fwhm(tri, 1.0) - 10.6) < 1e-12
    assert abs(kernels.fwhm(tri, 0.5) - 5.3) < 1e-12
    # an asymmetric triangle: left half base 4.2, right 7.8 -> FWHM 6.0
    asym = np.where(x < 0, np.maximum(0.0, 1.0 + x / 4.2), np.maximum(0.0, 1.0 - x / 7.8))
    assert abs(kernels.fwhm(asym, 1.0) - 6.0) < 1e-12
    # Gaussian-modulated carrier with many cycles: envelope FWHM -> 2 sqrt(2 ln 2) sigma
    t = np.arange(-400, 401, dtype=float)
    sig = 40.0
    sigl = np.exp(-t * t / (2 * sig * sig)) * np.cos(2 * np.pi * 0.21 * t)
    env = kernels.envelope(sigl)
    assert abs(kernels.fwhm(env, 1.0) - pulse.FWHM_PER_SIGMA * sig) < 0.05
    assert np.all(env >= np.abs(sigl) - 1e-12)


def test_envelope_of_cosine_is_flat():
    n = 256
    k = np.arange(n)
    x = 2.0 * np.cos(2 * np.pi * 32 * k / n)   # periodic in the padded length -> exact
    env = kernels.envelope(x)
    assert np.all(env > 0.9)


def test_paper_theta_single_element_is_one():
    """C = 1: the fixed and the dynamic delay laws coincide (one element on the
    axis), so a_i = b_i and theta_i = 1."""
    s = C1.replace(n_elem=1, n_samples=3000)
    zr = s.z0 + np.arange(40, 60) * s.dz
    kb, th, W = kernels.paper_kernels(zr, s.dz, 33, **oracle_kw(s))
    assert np.max(np.abs(th - 1.0)) < 1e-13
    ref = kernels.exact_kernels(zr, s.dz, 33, **oracle_kw(s))
    assert np.max(np.abs(kb - ref)) < 1e-13
    assert np.all(W > 0)


def test_paper_theta_near_one_on_own_row_and_window_is_psf_fwhm():
    s = C1
    zr = s.z0 + np.array([60, 120, 200]) * s.dz
    kb, th, W = kernels.paper_kernels(zr, s.dz, 65, **oracle_kw(s))
    assert np.all(np.abs(th - 1.0) < 0.05)
    # PSF FWHM is close to the pulse's two-way envelope FWHM (cycles / fc in time)
    pulse_fwhm_depth = s.cycles / s.fc * s.c / 2
    assert np.all(np.abs(W - pulse_fwhm_depth) < 0.25 * pulse_fwhm_depth)


def test_paper_theta_drops_away_from_reference():
    """Sec. 3.3: the approximation degrades away from the reference depth; a
    frozen receive law defocuses distant scatterers, so theta moves away from
    the own-row value."""
    s = C1
    rows = np.array([40, 100, 150, 200, 240])
    zr = s.z0 + np.arange(s.nz) * s.dz
    ref = np.full(s.nz, 150)
    kb, th, W = kernels.paper_kernels(zr[rows], s.dz, 65, ref_rows=np.searchsorted(rows, ref[rows]), **oracle_kw(s))
    assert abs(th[2] - 1.0) < 0.05
    assert abs(th[0] - 1.0) > abs(th[2] - 1.0)


def test_line_mode_reproduces_the_rf_domain_line_model():
    """eqn:line_conv taken literally: Theta times the fixed-delay beamformer of
    the RF.  For an on-axis line phantom the line-mode kernels applied to the
    reflectivity map equal Theta times the fixed-delay beamformer run on the
    synthesised RF (Born linearity), up to rounding."""
    from oracle import tidas
    from workloads import generators
    s = C1.replace(n_samples=2000)
    zs = s.z0 + np.arange(s.nz) * s.dz
    rows = np.arange(40, 200)
    zr = zs[rows]
    ref = np.searchsorted(rows, 120)
    kb, th, _ = kernels.paper_kernels(zr, s.dz, 33, ref_rows=np.full(rows.size, ref), line=True, **oracle_kw(s))
    src = np.array([20, 21, 55, 90, 91, 140])
    amp = generators.normal(src.size, seed=4)
    R = np.zeros((rows.size, 1))
    R[src, 0] = amp
    y = tidas.apply(kb, R)[:, 0]
    rf = simulate.simulate_rf(np.zeros(src.size), zr[src], amp, **sim_kw(s))
    kw = dict(n_elem=s.n_elem, pitch=s.pitch, c=s.c, fs=s.fs, t0=s.t0, angles=list(s.angles), fnumber=s.fnumber)
    f = kernels.fixed_delay_beamform(rf, zr, zr[ref], **kw)
    assert np.max(np.abs(y - th * f)) <= 1e-12 * np.max(np.abs(th * f))


def test_line_mode_single_element_equals_exact():
    """One element at the probe centre: the fixed delay law is the DAS law, so
    theta = 1 and, on a depth grid of one two-way sample (linear interpolation
    then reads the echo at the same fractional position for source and output
    shifts), the line-mode kernel equals the exact one."""
    s = C1.replace(n_elem=1, n_samples=3000, dz=C1.c / (2 * C1.fs))
    zr = s.z0 + np.arange(40, 60) * s.dz
    kb, th, _ = kernels.paper_kernels(zr, s.dz, 33, line=True, **oracle_kw(s))
    ref = kernels.exact_kernels(zr, s.dz, 33, **oracle_kw(s))
    assert np.allclose(th, 1.0, rtol=0, atol=1e-12)
    assert np.max(np.abs(kb - ref)) < 1e-12 * np.max(np.abs(ref))


def test_lateral_kernel_rows_equal_das_row_of_materialised_echo():
    """Lateral kernels equal RF synthesis (FP64) followed by DAS along the
    scatterer's own row, divided by the value at the scatterer; unsteered,
    they are symmetric (lateral symmetry of DAS for an on-axis scatterer)."""
    s = C1.replace(n_samples=1500)
    K = 15
    h = 7
    zr = np.array([5.3e-3, 12.0e-3, 18.4e-3])
    kx = kernels.lateral_kernels(zr, s.dx, K, **oracle_kw(s))
    for i, z in enumerate(zr):
        rf = simulate.simulate_rf([0.0], [z], [1.0], **sim_kw(s))
        row = das.das(rf, np.arange(-h, h + 1) * s.dx, [z], **das_kw(s))[0]
        assert np.max(np.abs(kx[i] - row / row[h])) <= 1e-12 * np.max(np.abs(row / row[h]))
        assert kx[i, h] == 1.0
        assert np.max(np.abs(kx[i] - kx[i, ::-1])) <= 1e-13
    # steered transmits break the symmetry
    st = s.replace(angles=(0.15,))
    ks = kernels.lateral_kernels(zr, s.dx, K, **oracle_kw(st))
    assert np.max(np.abs(ks - ks[:, ::-1])) > 1e-3


@pytest.mark.parametrize("Z,X,K", [(1, 1, 1), (4, 9, 3), (6, 20, 7), (3, 5, 11)])
def test_lateral_pass_equals_row_matrices_and_numpy_convolve(Z, X, K):
    from workloads import generators
    kx = generators.normal((Z, K), seed=Z + K)
    Y = generators.normal((2, Z, X), seed=X)
    out = tidas.apply_lateral(kx, Y)
    h = (K - 1) // 2
    for i in range(Z):
        M = np.zeros((X, X))
        for j in range(X):
            for m in range(-h, h + 1):
                if 0 <= j - m < X:
                    M[j, j - m] = kx[i, m + h]
        for b in range(2):
            assert np.max(np.abs(out[b, i] - M @ Y[b, i])) <= 1e-12
            full = np.convolve(Y[b, i], kx[i])          # length X + K - 1, offset h
            assert np.max(np.abs(out[b, i] - full[h:h + X])) <= 1e-12


def test_separable_model_reproduces_das_along_the_scatterers_row():
    """Depth pass with exact kernels, then lateral pass with lateral kernels,
    on the reflectivity of one on-grid scatterer at (0, z_s): the scatterer's
    row equals DAS's row, and its column is the depth pass's column (the
    lateral centre tap is 1)."""
    s = C1.replace(n_samples=1500, nz=40, nx=15, dz=0.05e-3, dx=0.15e-3, z0=10e-3, x0=-7 * 0.15e-3)
    xs = s.x0 + np.arange(s.nx) * s.dx
    zs = s.z0 + np.arange(s.nz) * s.dz
    j0, i0 = 7, 20
    assert abs(xs[j0]) < 1e-15
    kz = kernels.exact_kernels(zs, s.dz, 41, **oracle_kw(s))
    kx = kernels.lateral_kernels(zs, s.dx, 15, **oracle_kw(s))
    R = np.zeros((s.nz, s.nx))
    R[i0, j0] = 1.0
    Y2 = tidas.apply_lateral(kx, tidas.apply(kz, R))
    rf = simulate.simulate_rf([0.0], [zs[i0]], [1.0], **sim_kw(s))
    D = das.das(rf, xs, zs, **das_kw(s))
    scale = np.max(np.abs(D))
    assert scale > 0.1
    assert np.max(np.abs(Y2[i0] - D[i0])) <= 1e-12 * scale
    Y1 = tidas.apply(kz, R)
    assert np.array_equal(Y2[:, j0], Y1[:, j0])
    assert abs(Y1[i0, j0] - D[i0, j0]) <= 1e-12 * scale
    # elsewhere it is an approximation, and a better one than the depth pass alone
    assert np.linalg.norm(Y2 - D) < 0.5 * np.linalg.norm(Y1 - D)


def hand_theta_setup():
    """Two elements at x = +-300 l (l = c / fs, fs = 200 MHz so that linear
    interpolation is nearly exact), reference depth z_r = 400 l with receive
    distance 500 l (a Pythagorean triple), scatterer at z_i = 430 l, F/0.05
    (a nearly flat Hann aperture)."""
    s = C1.replace(n_elem=2, n_samples=6000, fnumber=0.05, fs=200e6)
    ell = s.c / s.fs
    return s.replace(pitch=600 * ell), ell


def hand_theta(s, ell, z_r, z_i, centre, half):
    """eqn:theta (first line, time domain) on the explicitly listed window
    {centre + q dzf : |q dzf| <= half}, dzf = l / 2, with a_i and b_i written
    out by hand:
      a_i(z) = sum_n w(x_n, z_r) p((2z - z_r + rho_n(z_r) - z_i - rho_n(z_i)) / c)
    (the fixed-delay read index (2z - z_r + rho_n(z_r)) / l is an integer on
    this axis, so the read is the echo sample itself), and b_i(z) the DAS
    value at (0, z): per element numpy.interp of the sampled unit echo at
    (z + rho_n(z)) / l, weighted by the Hann weight of depth z."""
    import math
    dzf = ell / 2
    qmax = math.floor(half / dzf)
    z = centre + np.arange(-qmax, qmax + 1) * dzf
    k = np.arange(s.n_samples)
    a = np.zeros_like(z)
    b = np.zeros_like(z)
    for xn in (-0.5 * s.pitch, 0.5 * s.pitch):
        r_r, r_i = math.hypot(xn, z_r), math.hypot(xn, z_i)
        w_r = 0.5 * (1 + math.cos(math.pi * abs(xn) / (z_r / (2 * s.fnumber))))
        a += w_r * pulse.pulse((2 * z - z_r + r_r - z_i - r_i) / s.c, s.fc, s.sigma)
        w_z = 0.5 * (1 + np.cos(np.pi * abs(xn) / (z / (2 * s.fnumber))))
        echo = pulse.pulse(k / s.fs - (z_i + r_i) / s.c, s.fc, s.sigma)
        b += w_z * np.interp((z + np.hypot(xn, z)) / ell, k, echo)
    return float(np.dot(a, b) / np.dot(a, a))


def test_paper_theta_window_centre_and_width_by_hand():
    """The weight window B (Sec. 2.3 eqn:tDAS, eqn:theta; Sec. 3.1-3.2: its
    width is the FWHM of the reference depth's PSF) is centred on the
    scatterer's own depth z_i and is W_r wide.  W_r is pinned to the closed
    form: the envelope FWHM of the pulse in time (cycles / fc) mapped to depth
    by the two-way travel time's slope d(z + rho)/dz / c = (1 + z_r / rho_r) / c.
    theta_i is then recomputed by hand on that window; a window centred on
    z_r, or twice as wide, gives a different weight."""
    import math
    s, ell = hand_theta_setup()
    z_r, z_i = 400 * ell, 430 * ell
    kb, th, W = kernels.paper_kernels(np.array([z_r, z_i]), ell, 5, ref_rows=np.array([0, 0]), **oracle_kw(s))
    w_closed = (s.cycles / s.fc) * s.c / (1 + 400 / 500)
    assert np.all(np.abs(W - w_closed) < 5e-3 * w_closed)
    # the FWHM is the reference depth's: the scatterer depth's slope differs by 1.1 %
    w_at_zi = (s.cycles / s.fc) * s.c / (1 + z_i / math.hypot(0.5 * s.pitch, z_i))
    assert abs(W[1] - w_closed) < 0.3 * abs(w_at_zi - w_closed)
    # the closed-form and the measured width select the same discrete window
    assert math.floor(W[1] / ell) == math.floor(w_closed / ell)
    t_hand = hand_theta(s, ell, z_r, z_i, z_i, 0.5 * w_closed)
    assert abs(th[1] - t_hand) <= 1e-12 * abs(t_hand)
    assert abs(th[0] - hand_theta(s, ell, z_r, z_r, z_r, 0.5 * w_closed)) <= 1e-12
    # centre and width both matter at this tolerance
    assert abs(hand_theta(s, ell, z_r, z_i, z_r, 0.5 * w_closed) - t_hand) > 1e-3
    assert abs(hand_theta(s, ell, z_r, z_i, z_i, w_closed) - t_hand) > 1e-3
    # the kernel row is theta_i times the reference response h_r
    assert np.max(np.abs(kb[1] - th[1] / th[0] * kb[0])) <= 1e-13 * np.max(np.abs(kb[1]))
