"""Tikhonov-regularised deconvolution through the line model (oracle; test
infrastructure only).

The paper motivates the convolutional form as a foundation for deconvolution
(abstract; Sec. 1; Sec. 4).  Objective, with A the operator of
``tidas.apply`` and lam > 0:

    J(r) = 1/2 ||A r - y||^2 + lam/2 ||r||^2

Gradient descent from r_0 = 0 with a fixed step eta:

    r_{t+1} = r_t - eta * (A^T (A r_t - y) + lam r_t)

and the closed-form minimiser per column, (M^T M + lam I)^-1 M^T y.
"""
import numpy as np

from . import tidas


def objective(K, r, y, lam):
    res = tidas.apply(K, r) - y
    return 0.5 * float(np.sum(res * res)) + 0.5 * lam * float(np.sum(np.asarray(r) ** 2))


def gradient(K, r, y, lam):
    return tidas.adjoint(K, tidas.apply(K, r) - y) + lam * np.asarray(r, np.float64)


def step_size(K, lam):
    """eta = 1 / (s_max(M)^2 + lam): the inverse Lipschitz constant of grad J."""
    s = np.linalg.svd(tidas.matrix(K), compute_uv=False)
    return 1.0 / (float(s[0]) ** 2 + lam)


def gradient_descent(K, y, lam, eta, iters, record=False):
    """Returns the final iterate (and, with record=True, every iterate)."""
    y = np.asarray(y, np.float64)
    r = np.zeros_like(y)
    hist = [r.copy()] if record else None
    for _ in range(int(iters)):
        r = r - eta * gradient(K, r, y, lam)
        if record:
            hist.append(r.copy())
    return (r, hist) if record else r


def closed_form(K, y, lam):
    """Exact minimiser of J for each lateral column."""
    M = tidas.matrix(K)
    Z = M.shape[0]
    lhs = M.T @ M + lam * np.eye(Z)
    y = np.asarray(y, np.float64)
    return np.linalg.solve(lhs, M.T @ y)


def gradient_descent_matrix(M, y, lam, eta, iters, record_at=()):
    """The same iteration with the operator given as its explicit column
    matrix M (``tidas.matrix``): A r = M @ r per column.  Returns the final
    iterate and a dict {t: r_t} for t in ``record_at``."""
    M = np.asarray(M, np.float64)
    y = np.asarray(y, np.float64)
    r = np.zeros_like(y)
    rec = {0: r.copy()} if 0 in record_at else {}
    for t in range(1, int(iters) + 1):
        r = r - eta * (M.T @ (M @ r - y) + lam * r)
        if t in record_at:
            rec[t] = r.copy()
    return r, rec
