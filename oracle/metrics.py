"""Error measures (oracle; test infrastructure only)."""
import numpy as np


def rel_l2(u, v):
    """||u - v||_2 / ||v||_2 (v the reference)."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    nv = float(np.linalg.norm(v.ravel()))
    return float(np.linalg.norm((u - v).ravel())) / nv if nv > 0 else float(np.linalg.norm(u.ravel()))


def squared_error(u, v, mask=None):
    """Relative squared l2 error ||u - v||^2 / ||v||^2, optionally restricted to
    a window (Sec. 3.3: local error near the peak, global error over the whole
    signal; the paper does not state the normalisation, the reference norm is
    used)."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    if mask is not None:
        u, v = u[mask], v[mask]
    nv = float(np.sum(v * v))
    return float(np.sum((u - v) ** 2)) / nv if nv > 0 else 0.0
