"""Pins of the oracle's geometry, delay law, apodization and pulse
(Sec. 2.1 eqn:delay / eqn:taylor / eqn:relTaylor)."""
import os

import numpy as np
import pytest

from oracle import geometry, pulse

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_delay_law_pythagorean_golden():
    """c * D_n(z) is an exact integer at Pythagorean geometries (hand-written fixture)."""
    rows = np.loadtxt(os.path.join(GOLD, "delay_law_pythagorean.txt"))
    c = 1540.0
    for xn, z, cd in rows:
        D = geometry.receive_delay(xn * 1e-3, z * 1e-3, c)
        assert abs(D * c - cd * 1e-3) <= 1e-17


def test_arrival_time_matches_delay_law():
    """On the centre line with an unsteered plane wave, the aligned read time
    2z/c - D_n(z) is the two-way flight time of the echo (eqn:delay)."""
    c = 1540.0
    xn = geometry.element_x(64, 0.3e-3)
    for z in (2e-3, 17.3e-3, 42e-3):
        tau = geometry.arrival_time(0.0, z, xn, 0.0, c)
        assert np.allclose(tau - 2 * z / c, -geometry.receive_delay(xn, z, c), rtol=0, atol=1e-20)


def test_relative_delay_variation_taylor_slope():
    """eqn:relTaylor: (D(z) - D(z0)) / D(z0) = -(z - z0) / sqrt(x_n^2 + z0^2) + O((z - z0)^2)."""
    c = 1540.0
    for xn in (0.45e-3, 3e-3, 9.45e-3):
        for z0 in (5e-3, 25e-3, 40e-3):
            rho0 = np.hypot(xn, z0)
            errs = []
            for dz in (1e-4, 5e-5, 2.5e-5):
                rel = (geometry.receive_delay(xn, z0 + dz, c) - geometry.receive_delay(xn, z0, c)) / \
                    geometry.receive_delay(xn, z0, c)
                errs.append(abs(rel + dz / rho0))
            # residual is second order in the step: it falls ~4x per halving
            assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0
            # the next Taylor term is D''/(2 D) dz^2 = -(rho0 + z0)/(2 rho0^2) dz * (dz/rho0) relative
            assert errs[0] < 1.01 * (rho0 + z0) / (2 * rho0) * (1e-4 / rho0) ** 2


def test_relative_variation_shrinks_with_depth_and_tails():
    """Sec. 2.1: the relative variation decreases with depth and towards the
    tails of the curve (larger |x_n|)."""
    c, dz = 1540.0, 1e-5

    def relvar(xn, z0):
        return abs((geometry.receive_delay(xn, z0 + dz, c) - geometry.receive_delay(xn, z0, c))
                   / geometry.receive_delay(xn, z0, c))
    zs = [5e-3, 10e-3, 20e-3, 40e-3]
    v = [relvar(3e-3, z) for z in zs]
    assert all(a > b for a, b in zip(v, v[1:]))
    xs = [0.5e-3, 2e-3, 6e-3, 12e-3]
    v = [relvar(x, 20e-3) for x in xs]
    assert all(a > b for a, b in zip(v, v[1:]))


def test_element_positions_symmetric():
    for C in (1, 2, 7, 64, 128):
        x = geometry.element_x(C, 0.3e-3)
        assert np.allclose(x, -x[::-1], atol=1e-18)
        if C > 1:
            assert np.allclose(np.diff(x), 0.3e-3, atol=1e-18)
    assert geometry.element_x(1, 0.3e-3)[0] == 0.0


def test_hann_apodization_values():
    z, F = 30e-3, 1.5
    a = z / (2 * F)
    assert geometry.hann_apod(0.0, z, F) == 1.0
    assert abs(geometry.hann_apod(0.5 * a, z, F) - 0.5) < 1e-15
    assert abs(geometry.hann_apod(-0.5 * a, z, F) - 0.5) < 1e-15
    assert abs(geometry.hann_apod(a, z, F)) < 1e-15
    assert geometry.hann_apod(1.0001 * a, z, F) == 0.0
    assert geometry.hann_apod(0.0, 0.0, F) == 0.0
    assert geometry.hann_apod(0.0, -1e-3, F) == 0.0


def test_pulse_closed_form_properties():
    fc, cycles = 5e6, 2.0
    s = pulse.pulse_sigma(fc, cycles)
    assert pulse.pulse(0.0, fc, s) == 1.0
    # envelope is exactly 1/2 at +- FWHM/2 = cycles / (2 fc); there cos(2 pi fc t) = cos(pi cycles)
    t = cycles / (2 * fc)
    assert abs(pulse.pulse(t, fc, s) - 0.5 * np.cos(np.pi * cycles)) < 1e-15
    assert abs(pulse.pulse(t, fc, s) - pulse.pulse(-t, fc, s)) == 0.0
    assert pulse.pulse(4.0001 * s, fc, s) == 0.0
    assert pulse.pulse(3.9999 * s, fc, s) != 0.0


@pytest.mark.parametrize("alpha", [0.0, 0.1, -0.17])
def test_plane_wave_transmit_time(alpha):
    """The front through (0, 0) at t = 0 is the line x sin a + z cos a = 0; a
    point at distance L along the propagation direction is reached at L / c."""
    c = 1540.0
    L = 12e-3
    assert abs(geometry.tau_tx(L * np.sin(alpha), L * np.cos(alpha), alpha, c) - L / c) < 1e-18
    assert abs(geometry.tau_tx(np.cos(alpha), -np.sin(alpha), alpha, c)) < 1e-18
