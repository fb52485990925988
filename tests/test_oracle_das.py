"""Pins of the oracle's RF synthesis (Sec. 2 eqn:SRX, Born superposition),
DAS (Sec. 2 eqn:appF): brute force, a textbook interpolation routine, the PSF
peak position, lateral symmetry and linearity; and of the fixed-delay
(time-invariant) beamformer of Sec. 2.3-2.4: DAS where every row is its own
reference, the centre-line fixed-delay line, the closed-form depth of its
shifted peak, symmetry and linearity."""
import numpy as np
import pytest

from oracle import das, geometry, kernels, pulse, simulate
from workloads import config, generators
from tests.helpers import das_kw, sim_kw, axes

C1 = config(1)


def tiny_setup(C, nz, nx, angles=(0.0,), T=160):
    s = C1.replace(n_elem=C, n_samples=T, angles=tuple(angles))
    # a small field whose echoes fit in T samples at 40 MHz
    return s.replace(**dict(nz=nz, nx=nx, dz=0.11e-3, dx=0.23e-3, z0=0.6e-3,
                            x0=-(nx - 1) / 2 * 0.23e-3))


@pytest.mark.parametrize("C,nz,nx,angles", [(1, 9, 3, (0.0,)), (4, 12, 5, (0.0,)),
                                            (8, 16, 8, (-0.1, 0.0, 0.13)), (3, 7, 2, (0.2,))])
def test_das_equals_bruteforce(C, nz, nx, angles):
    s = tiny_setup(C, nz, nx, angles)
    rf = generators.normal((len(angles), C, s.n_samples), seed=7 + C).astype(np.float32)
    xs, zs = axes(s)
    a = das.das(rf, xs, zs, **das_kw(s))
    b = das.das_bruteforce(rf.tolist(), xs.tolist(), zs.tolist(), **das_kw(s))
    assert np.max(np.abs(a - b)) <= 1e-13 * max(1.0, np.max(np.abs(b)))
    assert np.any(a != 0)


def test_das_single_element_is_textbook_interpolation():
    """C = 1 at x = 0, unsteered: the pixel (0, z) reads the channel at the
    two-way time 2z/c, i.e. numpy.interp of the zero-extended record."""
    s = tiny_setup(1, 40, 1, T=300).replace(x0=0.0)
    rf = generators.normal((1, 1, s.n_samples), seed=3)
    xs, zs = axes(s)
    img = das.das(rf, xs, zs, **das_kw(s))
    u = (2 * zs / s.c - s.t0) * s.fs
    padded = np.concatenate([[0.0], rf[0, 0], [0.0]])
    ref = np.interp(u, np.arange(-1, s.n_samples + 1), padded)
    assert np.max(np.abs(img[:, 0] - ref)) < 1e-13


def test_lerp_read_edges():
    S = np.array([1.0, 2.0, 4.0])
    assert das.lerp_read(S, -1.0) == 0.0
    assert das.lerp_read(S, -0.5) == 0.5
    assert das.lerp_read(S, 0.0) == 1.0
    assert das.lerp_read(S, 1.25) == 2.5
    assert das.lerp_read(S, 2.0) == 4.0
    assert das.lerp_read(S, 2.5) == 2.0
    assert das.lerp_read(S, 3.0) == 0.0


def test_rf_synthesis_linear_in_amplitudes_and_superposition():
    s = C1.replace(n_elem=16, n_samples=1200)
    x, z, a = generators.point_scatterers(6, 4e-3, 14e-3, seed=1)
    z = z + 1e-3
    kw = sim_kw(s)
    rf_all = simulate.simulate_rf(x, z, a, **kw)
    rf_a = simulate.simulate_rf(x[:3], z[:3], a[:3], **kw)
    rf_b = simulate.simulate_rf(x[3:], z[3:], a[3:], **kw)
    assert np.max(np.abs(rf_all - rf_a - rf_b)) < 1e-13
    rf_2 = simulate.simulate_rf(x, z, 2.5 * a, **kw)
    assert np.max(np.abs(rf_2 - 2.5 * rf_all)) < 1e-13


def test_rf_single_scatterer_peak_and_support():
    """A scatterer whose flight time is an integer number of samples puts its
    pulse peak (p(0) = 1) times the amplitude on that sample; the echo is even
    about it and zero beyond the pulse support."""
    s = C1.replace(n_elem=1, n_samples=800)
    k_star = 400
    z = k_star * s.c / (2 * s.fs)          # tau = 2 z / c = k_star / fs on the single element at x = 0
    rf = simulate.simulate_rf([0.0], [z], [1.7], **sim_kw(s))[0, 0]
    assert abs(rf[k_star] - 1.7) < 1e-12
    half = int(np.floor(pulse.TRUNC_SIGMAS * s.sigma * s.fs))
    assert np.max(np.abs(rf[k_star - half:k_star] - rf[k_star + half:k_star:-1])) < 1e-12
    assert np.all(rf[:k_star - half - 1] == 0) and np.all(rf[k_star + half + 2:] == 0)


def test_rf_on_axis_scatterer_mirror_symmetric():
    s = C1.replace(n_samples=1500)
    rf = simulate.simulate_rf([0.0], [13.1e-3], [1.0], **sim_kw(s))
    assert np.max(np.abs(rf[0] - rf[0, ::-1])) < 1e-13


def finer_grid_case():
    """Config-1 array with a pixel grid fine enough to resolve the 5 MHz
    oscillation (dz = lambda/8), one on-grid scatterer well inside."""
    s = C1.replace(n_samples=1400)
    lam = s.c / s.fc
    s = s.replace(nz=120, nx=41, dz=lam / 8, dx=0.1e-3, z0=12e-3, x0=-20 * 0.1e-3)
    return s


def test_psf_peak_at_scatterer_pixel():
    s = finer_grid_case()
    xs, zs = axes(s)
    for (ii, jj) in ((60, 20), (45, 27), (80, 9)):
        rf = simulate.simulate_rf([xs[jj]], [zs[ii]], [1.0], **sim_kw(s))
        img = das.das(rf, xs, zs, **das_kw(s))
        assert np.unravel_index(np.argmax(np.abs(img)), img.shape) == (ii, jj)


def test_lateral_symmetry_on_axis_scatterer():
    s = finer_grid_case()
    xs, zs = axes(s)
    assert np.allclose(xs, -xs[::-1], atol=1e-18)
    rf = simulate.simulate_rf([0.0], [zs[60]], [1.0], **sim_kw(s))
    img = das.das(rf, xs, zs, **das_kw(s))
    assert np.max(np.abs(img - img[:, ::-1])) <= 1e-13 * np.max(np.abs(img))
    # steered: I_alpha[i][j] = I_{-alpha}[i][X-1-j]
    a = 0.12
    sp, sm = s.replace(angles=(a,)), s.replace(angles=(-a,))
    ip = das.das(simulate.simulate_rf([0.0], [zs[60]], [1.0], **sim_kw(sp)), xs, zs, **das_kw(sp))
    im = das.das(simulate.simulate_rf([0.0], [zs[60]], [1.0], **sim_kw(sm)), xs, zs, **das_kw(sm))
    assert np.max(np.abs(ip - im[:, ::-1])) <= 1e-13 * np.max(np.abs(ip))
    assert np.max(np.abs(ip - ip[:, ::-1])) > 1e-3 * np.max(np.abs(ip))


def test_das_linear_under_superposition():
    s = C1.replace(n_samples=1500, angles=(-0.05, 0.0, 0.08))
    s = s.with_grid(64, 32)
    xs, zs = axes(s)
    r1 = generators.normal((3, s.n_elem, s.n_samples), seed=11)
    r2 = generators.normal((3, s.n_elem, s.n_samples), seed=12)
    a = das.das(r1 + 0.3 * r2, xs, zs, **das_kw(s))
    b = das.das(r1, xs, zs, **das_kw(s)) + 0.3 * das.das(r2, xs, zs, **das_kw(s))
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_das_config1_speckle_finite_and_nonzero():
    s = C1
    x, z, a = generators.point_scatterers(20, s.field_w, s.field_d, seed=0)
    rf = simulate.to_fp32(simulate.simulate_rf(x, z, a, **sim_kw(s)))
    xs, zs = axes(s)
    img = das.das(rf, xs, zs, **das_kw(s))
    assert img.shape == (256, 128) and np.all(np.isfinite(img)) and np.max(np.abs(img)) > 1.0


@pytest.mark.parametrize("C,nz,nx,angles", [(1, 9, 3, (0.0,)), (8, 16, 8, (-0.1, 0.0, 0.13)), (5, 12, 6, (0.2,))])
def test_fixed_delay_das_with_own_rows_is_das(C, nz, nx, angles):
    s = tiny_setup(C, nz, nx, angles)
    rf = generators.normal((len(angles), C, s.n_samples), seed=3 + C)
    xs, zs = axes(s)
    ref = das.das(rf, xs, zs, **das_kw(s))
    got = das.fixed_delay_das(rf, xs, zs, np.arange(nz), **das_kw(s))
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    # rows that are their own reference stay DAS rows when the others are not
    refs = np.arange(nz)
    refs[1::2] = nz // 2
    got = das.fixed_delay_das(rf, xs, zs, refs, **das_kw(s))
    own = refs == np.arange(nz)
    assert np.max(np.abs(got[own] - ref[own])) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(got[~own] - ref[~own])) > 1e-3 * np.max(np.abs(ref))
    # theta scales rows
    th = np.linspace(0.5, 2.0, nz)
    got_t = das.fixed_delay_das(rf, xs, zs, refs, **das_kw(s), theta=th)
    assert np.max(np.abs(got_t - th[:, None] * got)) <= 1e-13 * max(1.0, np.max(np.abs(got_t)))


def test_fixed_delay_das_centre_column_is_the_fixed_delay_line():
    s = finer_grid_case()
    xs, zs = axes(s)
    x_c = np.array([0.0])
    rf = simulate.simulate_rf([0.7e-3, -1.1e-3], [zs[40], zs[70]], [1.0, -0.6], **sim_kw(s))
    refs = np.clip((np.arange(s.nz) // 16) * 16 + 8, 0, s.nz - 1)
    got = das.fixed_delay_das(rf, x_c, zs, refs, **das_kw(s))[:, 0]
    line = kernels.fixed_delay_beamform(rf, zs, zs[refs], **das_kw(s))
    assert np.max(np.abs(got - line)) <= 1e-12 * np.max(np.abs(line))


def test_fixed_delay_peak_moves_to_the_closed_form_depth():
    """One element at x = 0, unsteered, a unit scatterer at (x_s, z_s) and every
    row frozen at depth z_r: along the column x = x_s the read time equals the
    echo's arrival time at 2 z/c = (z_s + rho_s + z_r - rho_r) / c, so the
    peak sits at z* = (z_s + rho_s + z_r - rho_r) / 2 (rho at lateral offset x_s)."""
    s = C1.replace(n_elem=1, n_samples=4000, angles=(0.0,), fs=100e6)
    x_s, z_s = 3.0e-3, 20.0e-3
    dzf = s.c / (2 * s.fs) / 8
    zs = z_s - 2e-3 + np.arange(int(4e-3 / dzf)) * dzf
    rf = simulate.simulate_rf([x_s], [z_s], [1.0], **sim_kw(s))
    for z_r in (17.0e-3, 20.0e-3, 24.0e-3):
        r = int(np.argmin(np.abs(zs - z_r))) if zs[0] <= z_r <= zs[-1] else 0
        zs_r = zs.copy()
        refs = np.full(zs.size, r)
        if not (zs[0] <= z_r <= zs[-1]):
            zs_r = np.concatenate([zs, [z_r]])
            refs = np.full(zs_r.size, zs_r.size - 1)
        img = das.fixed_delay_das(rf, [x_s], zs_r, refs, **das_kw(s))[:zs.size, 0]
        zr = zs_r[refs[0]]
        rho_s, rho_r = np.hypot(x_s, z_s), np.hypot(x_s, zr)
        z_star = (z_s + rho_s + zr - rho_r) / 2
        assert abs(zs[np.argmax(np.abs(img))] - z_star) <= 1.5 * dzf


def test_fixed_delay_das_symmetric_and_linear():
    s = finer_grid_case()
    xs, zs = axes(s)
    refs = np.full(s.nz, 60)
    rf = simulate.simulate_rf([0.0], [zs[50]], [1.0], **sim_kw(s))
    img = das.fixed_delay_das(rf, xs, zs, refs, **das_kw(s))
    assert np.max(np.abs(img - img[:, ::-1])) <= 1e-13 * np.max(np.abs(img))
    rf2 = simulate.simulate_rf([1.3e-3], [zs[80]], [-0.7], **sim_kw(s))
    both = das.fixed_delay_das(rf + 2.0 * rf2, xs, zs, refs, **das_kw(s))
    sep = img + 2.0 * das.fixed_delay_das(rf2, xs, zs, refs, **das_kw(s))
    assert np.max(np.abs(both - sep)) <= 1e-13 * np.max(np.abs(both))
