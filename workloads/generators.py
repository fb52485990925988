"""Seeded random draws (numpy ``default_rng``; the draw order is fixed here).

Nothing in this module implements the method: it only draws positions,
amplitudes, sizes, noise and parameter samples.
"""
import numpy as np


def point_scatterers(n, width, depth, seed):
    """n scatterers uniform in [-W/2, W/2] x [0, D] with N(0, 1) amplitudes.
    Draw order: x, z, amplitude."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-0.5 * width, 0.5 * width, n)
    z = rng.uniform(0.0, depth, n)
    a = rng.standard_normal(n)
    return x, z, a


def speckle_with_cysts(n, width, depth, n_cysts, r_lo, r_hi, seed):
    """Speckle phantom: ``point_scatterers`` then ``n_cysts`` anechoic disks
    (radius U[r_lo, r_hi], centre uniform with a one-radius margin) from which
    every scatterer is removed.  Returns x, z, amplitude, cysts [(cx, cz, r)]."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-0.5 * width, 0.5 * width, n)
    z = rng.uniform(0.0, depth, n)
    a = rng.standard_normal(n)
    cysts = []
    keep = np.ones(n, bool)
    for _ in range(n_cysts):
        r = rng.uniform(r_lo, r_hi)
        cx = rng.uniform(-0.5 * width + r, 0.5 * width - r)
        cz = rng.uniform(r, depth - r)
        cysts.append((cx, cz, r))
        keep &= (x - cx) ** 2 + (z - cz) ** 2 > r * r
    return x[keep], z[keep], a[keep], cysts


def snap_to_grid(x, z, x0, dx, nx, z0, dz, nz):
    """Nearest pixel indices (clipped to the grid) and the snapped coordinates."""
    j = np.clip(np.rint((np.asarray(x) - x0) / dx), 0, nx - 1).astype(np.int64)
    i = np.clip(np.rint((np.asarray(z) - z0) / dz), 0, nz - 1).astype(np.int64)
    return i, j, z0 + i * dz, x0 + j * dx


def reflectivity_map(i, j, amp, nz, nx):
    """Dense [Z][X] map with the (summed) amplitudes at pixel indices (i, j)."""
    R = np.zeros((nz, nx), np.float64)
    np.add.at(R, (np.asarray(i), np.asarray(j)), np.asarray(amp, np.float64))
    return R


def spikes(nz, nx, n, seed):
    """n spikes at distinct uniformly drawn pixels, N(0, 1) amplitudes."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(nz * nx, size=n, replace=False)
    amp = rng.standard_normal(n)
    R = np.zeros(nz * nx, np.float64)
    R[flat] = amp
    return R.reshape(nz, nx)


def normal(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def uniform(shape, lo, hi, seed):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


def ragged_sizes(n_frames, x_lo, x_hi, z_lo, z_hi, seed):
    """Per-frame (nz, nx), both drawn uniformly over the inclusive ranges."""
    rng = np.random.default_rng(seed)
    nx = rng.integers(x_lo, x_hi + 1, n_frames)
    nz = rng.integers(z_lo, z_hi + 1, n_frames)
    return [(int(a), int(b)) for a, b in zip(nz, nx)]


def kernel_params(n, depth_lo, depth_hi, fnumber, angle_deg, fc, seed):
    """Columns (depth [m], F-number, angle [rad], centre frequency [Hz]), each
    uniform over its range.  Draw order: depth, F-number, angle, fc."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(depth_lo, depth_hi, n)
    f = rng.uniform(fnumber[0], fnumber[1], n)
    a = np.radians(rng.uniform(angle_deg[0], angle_deg[1], n))
    c = rng.uniform(fc[0], fc[1], n)
    return np.stack([d, f, a, c], axis=1)


def mlp_init(widths, seed):
    """Initial parameters: W_l [out][in] and b_l [out] uniform on
    [-1/sqrt(fan_in), 1/sqrt(fan_in)].  The nonzero first-layer biases spread
    the GELU kinks of the 4-input layer over the input box (zero biases put
    them all through the origin); on the 200k-kernel surrogate data this
    trains to half the held-out error of N(0, 2/fan_in) weights with zero
    biases."""
    rng = np.random.default_rng(seed)
    params = []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        bound = 1.0 / np.sqrt(fan_in)
        W = rng.uniform(-bound, bound, (fan_out, fan_in))
        b = rng.uniform(-bound, bound, fan_out)
        params.append((W, b))
    return params


def batch_indices(n_items, batch, n_steps, seed):
    """[n_steps][batch] row indices: a fresh permutation per epoch, cut into
    consecutive batches."""
    rng = np.random.default_rng(seed)
    out = []
    perm = rng.permutation(n_items)
    pos = 0
    for _ in range(n_steps):
        if pos + batch > n_items:
            perm = rng.permutation(n_items)
            pos = 0
        out.append(perm[pos:pos + batch])
        pos += batch
    return np.stack(out)
