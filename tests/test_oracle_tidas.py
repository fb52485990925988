"""Pins of the oracle's line model (Sec. 2.4 eqn:line_conv), its adjoint, its
gradient in the kernels, the deconvolution built on it, and the tiDAS = DAS identity where the PSF is
truly row-invariant."""
import numpy as np
import pytest

from oracle import das, deconv, kernels, simulate, tidas
from workloads import config, generators
from tests.helpers import das_kw, sim_kw, oracle_kw

C1 = config(1)


@pytest.mark.parametrize("Z,X,K", [(1, 1, 1), (5, 3, 3), (17, 4, 7), (40, 6, 65), (64, 2, 129)])
def test_apply_equals_explicit_banded_matrix(Z, X, K):
    kb = generators.normal((Z, K), seed=Z + K)
    R = generators.normal((Z, X), seed=X)
    M = tidas.matrix(kb)
    assert np.max(np.abs(tidas.apply(kb, R) - M @ R)) < 1e-13 * max(1, np.max(np.abs(M @ R)))
    # band structure: nothing outside |i - s| <= h
    h = (K - 1) // 2
    i, s = np.nonzero(M)
    assert np.all(np.abs(i - s) <= h)


def test_shared_kernel_is_toeplitz_numpy_convolve():
    Z, X, K = 50, 5, 13
    k = generators.normal(K, seed=2)
    kb = np.tile(k, (Z, 1))
    R = generators.normal((Z, X), seed=3)
    Y = tidas.apply(kb, R)
    for j in range(X):
        assert np.max(np.abs(Y[:, j] - np.convolve(R[:, j], k, mode="same"))) < 1e-13
    M = tidas.matrix(kb)
    # Toeplitz: constant along diagonals
    for d in range(-(K // 2), K // 2 + 1):
        assert np.ptp(np.diagonal(M, d)) == 0.0
    Rb = tidas.adjoint(kb, Y)
    for j in range(X):
        assert np.max(np.abs(Rb[:, j] - np.correlate(Y[:, j], k, mode="same"))) < 1e-12


def test_impulse_response_reads_kernel_rows():
    Z, K = 30, 9
    h = 4
    kb = generators.normal((Z, K), seed=4)
    for s in (0, 3, 15, 29):
        R = np.zeros((Z, 1))
        R[s, 0] = 1.0
        Y = tidas.apply(kb, R)[:, 0]
        for i in range(Z):
            m = i - s
            expect = kb[i, m + h] if abs(m) <= h else 0.0
            assert Y[i] == expect


@pytest.mark.parametrize("Z,X,K,B", [(7, 3, 5, 1), (33, 8, 17, 2), (64, 5, 65, 3)])
def test_adjoint_is_transpose_and_dot_product_test(Z, X, K, B):
    kb = generators.normal((Z, K), seed=K)
    R = generators.normal((B, Z, X), seed=1)
    Yb = generators.normal((B, Z, X), seed=2)
    lhs = np.sum(tidas.apply(kb, R) * Yb)
    rhs = np.sum(R * tidas.adjoint(kb, Yb))
    assert abs(lhs - rhs) < 1e-12 * max(1, abs(lhs))
    M = tidas.matrix(kb)
    for b in range(B):
        assert np.max(np.abs(tidas.adjoint(kb, Yb[b]) - M.T @ Yb[b])) < 1e-12


def test_gradient_matches_central_finite_differences_32x64():
    """FP64 central differences of 1/2 ||A R - y||^2 at 32 x 64 (kernels of the
    config-1 kind: exact DAS PSFs, K = 65 on 32 rows)."""
    s = C1.with_grid(32, 64)
    zs = s.z0 + np.arange(32) * s.dz
    kb = kernels.exact_kernels(zs + 15e-3, s.dz, 65, **oracle_kw(s))
    R = generators.normal((32, 64), seed=8)
    y = generators.normal((32, 64), seed=9)

    def f(r):
        res = tidas.apply(kb, r) - y
        return 0.5 * np.sum(res * res)
    g = tidas.adjoint(kb, tidas.apply(kb, R) - y)
    rng = np.random.default_rng(10)
    eps = 1e-5
    for _ in range(25):
        i, j = rng.integers(32), rng.integers(64)
        e = np.zeros_like(R)
        e[i, j] = eps
        fd = (f(R + e) - f(R - e)) / (2 * eps)
        assert abs(fd - g[i, j]) <= 1e-7 * max(1.0, abs(g[i, j]))
    # and directional derivatives along random directions
    for k in range(5):
        d = generators.normal((32, 64), seed=100 + k)
        fd = (f(R + eps * d) - f(R - eps * d)) / (2 * eps)
        assert abs(fd - np.sum(g * d)) <= 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("Z,X,K,B", [(1, 1, 1, 1), (9, 3, 5, 2), (40, 7, 17, 1), (33, 4, 65, 3)])
def test_kernel_grad_is_the_band_of_ybar_times_r_transposed(Z, X, K, B):
    """Kbar[i][m+h] is entry (i, i - m) of sum_b Ybar_b R_b^T (a matrix
    product), and zero where i - m leaves the image."""
    R = generators.normal((B, Z, X), seed=Z + 1)
    Yb = generators.normal((B, Z, X), seed=Z + 2)
    G = tidas.kernel_grad(R, Yb, K)
    P = sum(Yb[b] @ R[b].T for b in range(B))
    h = (K - 1) // 2
    for i in range(Z):
        for m in range(-h, h + 1):
            expect = P[i, i - m] if 0 <= i - m < Z else 0.0
            assert abs(G[i, m + h] - expect) <= 1e-12 * max(1.0, abs(expect))


@pytest.mark.parametrize("Z,X,K,B", [(8, 2, 3, 1), (30, 5, 9, 2), (64, 3, 65, 2)])
def test_kernel_grad_dot_product_test(Z, X, K, B):
    """<dK, Kbar(R, Ybar)> = <A_dK R, Ybar> for any direction dK: the gradient
    is the line model's derivative in its kernels (the model is linear in K)."""
    R = generators.normal((B, Z, X), seed=11)
    Yb = generators.normal((B, Z, X), seed=12)
    dK = generators.normal((Z, K), seed=13)
    lhs = np.sum(dK * tidas.kernel_grad(R, Yb, K))
    rhs = np.sum(tidas.apply(dK, R) * Yb)
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))


def test_kernel_grad_matches_central_finite_differences_32x64():
    """FP64 central differences of 1/2 ||A_K R - y||^2 in single taps and along
    random directions of the kernel bank, at 32 x 64 with K = 65."""
    Z, X, K = 32, 64, 65
    kb = generators.normal((Z, K), seed=20) * 0.1
    R = generators.normal((2, Z, X), seed=21)
    y = generators.normal((2, Z, X), seed=22)

    def f(k):
        res = tidas.apply(k, R) - y
        return 0.5 * np.sum(res * res)
    g = tidas.kernel_grad(R, tidas.apply(kb, R) - y, K)
    rng = np.random.default_rng(23)
    eps = 1e-5
    for _ in range(25):
        i, t = rng.integers(Z), rng.integers(K)
        e = np.zeros_like(kb)
        e[i, t] = eps
        fd = (f(kb + e) - f(kb - e)) / (2 * eps)
        assert abs(fd - g[i, t]) <= 1e-7 * max(1.0, abs(g[i, t]))
    for k in range(5):
        d = generators.normal((Z, K), seed=200 + k)
        fd = (f(kb + eps * d) - f(kb - eps * d)) / (2 * eps)
        assert abs(fd - np.sum(g * d)) <= 1e-7 * max(1.0, abs(fd))


def test_kernel_grad_impulses_read_single_products():
    """R and Ybar single impulses: only the tap that joins them is non-zero."""
    Z, X, K = 20, 3, 7
    h = 3
    for (i, s, j) in [(5, 5, 0), (10, 8, 2), (0, 3, 1), (19, 16, 0), (4, 12, 1)]:
        R = np.zeros((Z, X))
        Yb = np.zeros((Z, X))
        R[s, j] = 2.0
        Yb[i, j] = -3.0
        G = tidas.kernel_grad(R, Yb, K)
        expect = np.zeros((Z, K))
        if abs(i - s) <= h:
            expect[i, i - s + h] = -6.0
        assert np.array_equal(G, expect)


def test_tidas_equals_das_where_psf_is_row_invariant():
    """One element at x = 0, unsteered, one column at x = 0, dz a multiple of
    c/(2 fs), z0 on the sample grid, scatterers on grid rows: every DAS read
    falls on a sample and the PSF is the same pulse at every depth, so the
    exact-kernel line model reproduces DAS (Sec. 2.4)."""
    s = C1.replace(n_elem=1, n_samples=3000)
    unit = s.c / (2 * s.fs)
    s = s.replace(nz=200, nx=1, dz=2 * unit, z0=300 * unit, x0=0.0)
    zs = s.z0 + np.arange(s.nz) * s.dz
    K = 33
    kb = kernels.exact_kernels(zs, s.dz, K, **oracle_kw(s))
    rows = np.array([20, 37, 38, 90, 150, 175])
    amp = generators.normal(rows.size, seed=13)
    R = generators.reflectivity_map(rows, np.zeros_like(rows), amp, s.nz, 1)
    rf = simulate.simulate_rf(np.zeros(rows.size), zs[rows], amp, **sim_kw(s))
    d = das.das(rf, [0.0], zs, **das_kw(s))
    y = tidas.apply(kb, R)
    assert np.max(np.abs(y - d)) < 1e-13 * np.max(np.abs(d))


def test_tidas_not_das_for_wide_aperture():
    """Sanity of the previous pin: with the full config-1 array the PSF varies
    with depth, and the line model is an approximation (nonzero error)."""
    s = C1
    zs = s.z0 + np.arange(s.nz) * s.dz
    kb = kernels.exact_kernels(zs, s.dz, s.K, **oracle_kw(s))
    rows = np.array([60, 130, 200])
    R = generators.reflectivity_map(rows, np.zeros(3, int), np.ones(3), s.nz, 1)
    rf = simulate.simulate_rf(np.zeros(3), zs[rows], np.ones(3), **sim_kw(s))
    d = das.das(rf, [0.0], zs, **das_kw(s))
    y = tidas.apply(kb, R)
    err = np.linalg.norm(y - d) / np.linalg.norm(d)
    assert 1e-6 < err < 0.5
    # the exact kernels put the correct peak on each scatterer's own row
    for r in rows:
        assert abs(y[r, 0] - d[r, 0]) < 1e-12 * abs(d[r, 0])


def test_deconvolution_monotone_and_converging_to_closed_form():
    s = C1.with_grid(48, 6)
    zs = s.z0 + np.arange(48) * s.dz + 10e-3
    kb = kernels.exact_kernels(zs, s.dz, 17, **oracle_kw(s))
    kb = kb / np.max(np.abs(kb))
    rtrue = generators.spikes(48, 6, 12, seed=3)
    y = tidas.apply(kb, rtrue) + 0.01 * generators.normal((48, 6), seed=4)
    lam = 1e-3
    eta = deconv.step_size(kb, lam)
    r, hist = deconv.gradient_descent(kb, y, lam, eta, 300, record=True)
    J = [deconv.objective(kb, h, y, lam) for h in hist]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(J, J[1:]))
    rstar = deconv.closed_form(kb, y, lam)
    g = deconv.gradient(kb, rstar, y, lam)
    assert np.max(np.abs(g)) < 1e-10
    dist = [np.linalg.norm(h - rstar) for h in hist[::50]]
    assert all(b < a for a, b in zip(dist, dist[1:]))
    assert deconv.objective(kb, r, y, lam) >= deconv.objective(kb, rstar, y, lam) - 1e-12


def test_matrix_form_gradient_descent_equals_operator_form():
    Z, X, K = 40, 5, 9
    kb = generators.normal((Z, K), seed=21) / 4
    y = generators.normal((Z, X), seed=22)
    lam = 1e-2
    eta = deconv.step_size(kb, lam)
    r_op, hist = deconv.gradient_descent(kb, y, lam, eta, 25, record=True)
    r_m, rec = deconv.gradient_descent_matrix(tidas.matrix(kb), y, lam, eta, 25, record_at=(1, 7, 25))
    assert np.max(np.abs(r_op - r_m)) < 1e-12
    for t in (1, 7):
        assert np.max(np.abs(hist[t] - rec[t])) < 1e-12
