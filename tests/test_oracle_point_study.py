"""Pins of the single-point study oracle (Sec. 3.1-3.3) against closed forms,
the independently written DAS and fixed-delay oracles, and the paper-mode
weights of the line model."""
import numpy as np
import pytest

from oracle import das as o_das, kernels as o_k, point_study as ps, pulse

C0 = 1540.0


def setup(n_elem=33, pitch=0.3e-3, fc=5e6, fs=40e6, n_samples=1400, fnumber=1.0, n_tx=9, t0=0.0, cycles=2.0):
    return dict(n_elem=n_elem, pitch=pitch, c=C0, fs=fs, t0=t0, fc=fc, sigma=pulse.pulse_sigma(fc, cycles),
                n_samples=n_samples, fnumber=fnumber, n_tx=n_tx)


def test_kossoff_count_closed_form():
    # lambda = 0.308 mm; D = sqrt(4 lambda z_f / 0.6) = 7.1647 mm at z_f = 25 mm: 23.88 pitches
    assert ps.kossoff_tx_count(192, 0.3e-3, C0, 5e6, 25e-3) == 24     # nearest even count
    assert ps.kossoff_tx_count(191, 0.3e-3, C0, 5e6, 25e-3) == 23     # nearest odd count
    # 15 mm at 7 MHz: D = sqrt(4 * 0.22 mm * 15 mm / 0.6) = 4.690 mm = 15.63 pitches
    assert ps.kossoff_tx_count(128, 0.3e-3, C0, 7e6, 15e-3) == 16
    assert ps.kossoff_tx_count(127, 0.3e-3, C0, 7e6, 15e-3) == 15
    # the focal depth is 0.6 of the near-field length of the unrounded aperture
    lam = C0 / 5e6
    D = np.sqrt(4 * lam * 25e-3 / 0.6)
    assert abs(0.6 * D * D / (4 * lam) - 25e-3) < 1e-15
    assert ps.kossoff_tx_count(16, 0.3e-3, C0, 5e6, 1.0) == 16        # clamped to the array
    assert ps.kossoff_tx_count(16, 0.3e-3, C0, 5e6, 1e-6) == 2        # at least one symmetric pair
    assert ps.kossoff_tx_count(15, 0.3e-3, C0, 5e6, 1e-6) == 1


def test_tx_elements_are_the_centremost():
    x = ps.tx_elements(8, 1.0, 4)
    assert np.allclose(x, [-1.5, -0.5, 0.5, 1.5])
    assert np.allclose(ps.tx_elements(7, 1.0, 3), [-1.0, 0.0, 1.0])
    with pytest.raises(ValueError):
        ps.tx_elements(8, 1.0, 3)


def test_fire_times_focus_every_element_at_the_focal_depth():
    """Each element's wave reaches the focus at z_f / c (the centre element,
    if any, fires at t = 0; outer elements fire earlier)."""
    x = ps.tx_elements(9, 0.3e-3, 9)
    zf = 20e-3
    T = ps.tx_fire_times(x, zf, C0)
    arrival = T + np.sqrt(x ** 2 + zf ** 2) / C0
    assert np.allclose(arrival, zf / C0, rtol=0, atol=1e-18)
    assert T[4] == 0.0 and np.all(T[:4] < 0) and np.allclose(T, T[::-1])


def test_echo_at_the_focus_is_n_tx_aligned_pulses():
    """A scatterer at the focus receives every transmit wave at once: the echo
    on element n is n_tx times the pulse delayed by z_f / c + rho_n / c."""
    s = setup(n_tx=9)
    zf = 17.3e-3
    rf = ps.focused_echo(zf, z_focus=zf, **ps._echo_args(s))
    t = np.arange(s["n_samples"]) / s["fs"]
    xn = (np.arange(s["n_elem"]) - (s["n_elem"] - 1) / 2) * s["pitch"]
    for n in (0, 7, 16, 32):
        want = 9 * pulse.pulse(t - zf / C0 - np.sqrt(xn[n] ** 2 + zf ** 2) / C0, s["fc"], s["sigma"])
        assert np.allclose(rf[n], want, rtol=0, atol=1e-12)


def test_echo_away_from_the_focus_spreads_the_transmit():
    """Off focus the outer transmit elements arrive later than z/c (shallower
    than the focus) or earlier (deeper): the echo is a sum of shifted pulses,
    not n_tx aligned ones."""
    s = setup(n_tx=9, fc=5e6, fs=40e6)
    zf = 20e-3
    zs = 8e-3
    rf = ps.focused_echo(zs, z_focus=zf, **ps._echo_args(s))
    t = np.arange(s["n_samples"]) / s["fs"]
    xm = ps.tx_elements(s["n_elem"], s["pitch"], 9)
    tx = ps.tx_fire_times(xm, zf, C0) + np.sqrt(xm ** 2 + zs ** 2) / C0
    want = sum(pulse.pulse(t - tm - zs / C0, s["fc"], s["sigma"]) for tm in tx)   # element at x = 0
    assert np.allclose(rf[16], want, rtol=0, atol=1e-12)
    assert tx.max() - tx.min() > 0.1 / s["fc"]


def test_single_centre_transmitter_is_the_plane_wave_echo():
    s = setup(n_tx=1)
    zs = 11.1e-3
    rf = ps.focused_echo(zs, z_focus=25e-3, **ps._echo_args(s))
    t = np.arange(s["n_samples"]) / s["fs"]
    xn = (np.arange(s["n_elem"]) - 16) * s["pitch"]
    want = pulse.pulse(t[None, :] - zs / C0 - np.sqrt(xn[:, None] ** 2 + zs ** 2) / C0, s["fc"], s["sigma"])
    assert np.allclose(rf, want, rtol=0, atol=1e-13)


def test_das_line_equals_the_das_oracle_on_the_axis():
    s = setup()
    zf = 15e-3
    rf = ps.focused_echo(12e-3, z_focus=zf, **ps._echo_args(s))
    z = 12e-3 + np.arange(-60, 61) * (C0 / (2 * s["fs"])) * 0.77
    got = ps.das_line(rf, z, **ps._line_args(s))
    want = o_das.das(rf[None], np.array([0.0]), z, n_elem=s["n_elem"], pitch=s["pitch"], c=C0, fs=s["fs"],
                     t0=s["t0"], angles=[0.0], fnumber=s["fnumber"])[:, 0]
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    assert np.max(np.abs(want)) > 1.0


def test_fixed_delay_line_equals_the_fixed_delay_oracle_and_das_at_its_depth():
    s = setup(t0=0.3e-6)
    rf = ps.focused_echo(14e-3, z_focus=20e-3, **ps._echo_args(s))
    z = 14e-3 + np.arange(-80, 81) * (C0 / (2 * s["fs"]))
    zr = 16.5e-3
    got = ps.fixed_delay_line(rf, z, zr, **ps._line_args(s))
    want = o_k.fixed_delay_beamform(rf[None], z, zr, n_elem=s["n_elem"], pitch=s["pitch"], c=C0, fs=s["fs"],
                                    t0=s["t0"], angles=[0.0], fnumber=s["fnumber"])
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    # at the reference depth the frozen law is DAS's own law
    at = ps.fixed_delay_line(rf, np.array([zr]), zr, **ps._line_args(s))
    assert abs(at[0] - ps.das_line(rf, np.array([zr]), **ps._line_args(s))[0]) <= 1e-13


def test_one_element_line_is_the_sampled_pulse():
    """C = 1 at x = 0, one transmitter, scatterer on the sample grid: both
    lines read the echo at integer indices and equal p(q / fs)."""
    fs = 40e6
    dzf = C0 / (2 * fs)
    s = setup(n_elem=1, n_tx=1, fs=fs, n_samples=900)
    zs = 300 * dzf
    rf = ps.focused_echo(zs, z_focus=10e-3, **ps._echo_args(s))
    q = np.arange(-20, 21)
    b = ps.das_line(rf, zs + q * dzf, **ps._line_args(s))
    a = ps.fixed_delay_line(rf, zs + q * dzf, 10e-3, **ps._line_args(s))
    want = pulse.pulse(q / fs, s["fc"], s["sigma"])
    assert np.allclose(b, want, rtol=0, atol=1e-12)
    assert np.allclose(a, want, rtol=0, atol=1e-12)


def test_study_theta_row_of_the_focus_equals_paper_mode_weights():
    """With one transmitter at the probe centre the study's transmit is the
    0-degree plane wave on the axis, so the study's weights for the focal
    point's delay curve are the paper-mode weights (Sec. 2.3 eqn:theta) of a
    depth grid on the study axis with that point as every row's reference:
    two independently written constructions of the same definition."""
    s = setup(n_elem=33, n_tx=1, fs=40e6, n_samples=1400)
    P, z_first, z_step, f = 9, 8e-3, 1.3e-3, 5
    Ql = 900
    th, loc, glo, W, _ = ps.study(s, P, z_first, z_step, f, Ql, refs=[f, 2])
    zs = z_first + np.arange(P) * z_step
    kw = dict(n_elem=s["n_elem"], pitch=s["pitch"], c=C0, fs=s["fs"], t0=s["t0"], fc=s["fc"], sigma=s["sigma"],
              n_samples=s["n_samples"], angles=[0.0], fnumber=s["fnumber"])
    _, th_p, widths = o_k.paper_kernels(zs, z_step, 5, ref_rows=[f] * P, **kw)
    assert abs(W - widths[0]) <= 1e-15
    assert np.allclose(th[0], th_p, rtol=1e-12, atol=0)
    # the diagonal entry is the own-row weight: near 1, with a small error
    assert abs(th[0, f] - 1.0) < 0.05 and loc[0, f] < 1e-2
    # a delay curve far from the scatterer fits worse than the scatterer's own
    assert loc[1, 8] > loc[0, 8] or loc[1, 8] > 1e-3


def test_study_errors_by_definition_and_theta_minimises_the_local_error():
    s = setup(n_elem=17, n_tx=5, fs=40e6, n_samples=1200)
    P, z_first, z_step, f = 6, 9e-3, 2.0e-3, 3
    Ql = 700
    th, loc, glo, W, _ = ps.study(s, P, z_first, z_step, f, Ql, refs=[1, 4], points=[0, 3, 5])
    zp = ps.study_axis(P, z_first, z_step)
    dzf = C0 / (2 * s["fs"])
    Qw = int(np.floor(0.5 * W / dzf))
    # recompute one pair by hand: the window is |q| <= Qw around the scatterer
    r, sc = 4, 5
    rf = ps.focused_echo(zp[sc], z_focus=zp[f], **ps._echo_args(s))
    q = np.arange(-Ql, Ql + 1)
    z = zp[sc] + q * dzf
    a = ps.fixed_delay_line(rf, z, zp[r], **ps._line_args(s))
    b = ps.das_line(rf, z, **ps._line_args(s))
    B = slice(Ql - Qw, Ql + Qw + 1)
    t = np.dot(a[B], b[B]) / np.dot(a[B], a[B])
    assert abs(th[1, 2] - t) <= 1e-12 * abs(t)
    assert abs(loc[1, 2] - np.sum((t * a[B] - b[B]) ** 2) / np.sum(b[B] ** 2)) <= 1e-12
    assert abs(glo[1, 2] - np.sum((t * a - b) ** 2) / np.sum(b ** 2)) <= 1e-12
    for d in (1e-3, -1e-3):
        assert np.sum(((t + d) * a[B] - b[B]) ** 2) >= np.sum((t * a[B] - b[B]) ** 2)
    assert np.all(loc >= 0) and np.all(glo >= 0)


def test_one_element_study_is_exact():
    """C = 1: the fixed and dynamic laws coincide (D = 0), so theta = 1 and both
    errors vanish; DAS and tiDAS have equal peaks and FWHMs, the FWHM being the
    pulse envelope's two periods mapped to depth (c / 2 per second)."""
    fs = 80e6
    s = setup(n_elem=1, n_tx=1, fs=fs, n_samples=2400, fc=5e6)
    dzf = C0 / (2 * fs)
    th, loc, glo, W, st = ps.study(s, 4, 400 * dzf, 300 * dzf, 1, 400, stats_half=120)
    assert np.allclose(th, 1.0, rtol=0, atol=1e-12)
    assert np.all(loc <= 1e-24) and np.all(glo <= 1e-24)
    assert np.allclose(st[:, 0], st[:, 1], rtol=1e-12) and np.allclose(st[:, 2], st[:, 3], rtol=1e-12)
    fwhm_depth = 2.0 / s["fc"] * C0 / 2
    assert np.all(np.abs(st[:, 2] - fwhm_depth) < 0.05 * fwhm_depth)
    assert abs(W - st[1, 2]) < 1e-12


def test_stats_at_the_focus_use_the_focal_delay_curve():
    """For the scatterer at the focus, the focal point's delay curve is its own
    law: the tiDAS peak matches the DAS peak within the small fixed-law
    error, while a distant point's curve would not."""
    s = setup(n_elem=33, n_tx=9, fs=40e6, n_samples=1400)
    P, z_first, z_step, f = 7, 6e-3, 2.0e-3, 4
    _, _, _, _, st = ps.study(s, P, z_first, z_step, f, 500, refs=[f], points=[f, 0], stats_half=150)
    assert abs(st[0, 1] / st[0, 0] - 1.0) < 0.02
    assert abs(st[0, 3] - st[0, 2]) < 0.05 * st[0, 2]
    # the shallow scatterer read with the deep focal curve: the fitted tiDAS
    # peak is lower than DAS's (energy spread along the line)
    assert st[1, 1] < st[1, 0]
