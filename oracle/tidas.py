"""The tiDAS line model as an operator on a reflectivity map (oracle; test
infrastructure only).

Sec. 2.4, eqn:line_conv: along an image line the reconstruction is a
convolution with fixed parameters, scaled per output point by the weight set
Theta.  Written against the reflectivity map R (Born linearity, Sec. 2), each
lateral column is convolved along depth, and the kernel is chosen by the
OUTPUT row (gather form: Theta multiplies the output):

    Y[b][i][j] = sum_{m=-h..h} K[i][m+h] * R[b][i-m][j],   R = 0 outside [0, Z)

The adjoint (transpose) is

    Rbar[b][s][j] = sum_{m=-h..h} K[s+m][m+h] * Ybar[b][s+m][j],

terms with s + m outside [0, Z) dropped.  The gradient of a loss L with
respect to the kernels, given Ybar = dL/dY, follows from differentiating the
sum above term by term (the conclusion, Sec. 4, treats the weights as
learnable):

    Kbar[i][m+h] = sum_b sum_j Ybar[b][i][j] * R[b][i-m][j],   R = 0 outside [0, Z).

All three are written as plain loops over the tap index m.

The lateral pass of the separable 2-D extension (future work in Sec. 4)
convolves each depth row along the lateral axis with that row's kernel:

    Y2[b][i][j] = sum_{m=-h..h} Kx[i][m+h] * Y[b][i][j-m],   Y = 0 outside [0, X).
"""
import numpy as np


def _check(K):
    K = np.asarray(K, np.float64)
    if K.ndim != 2 or K.shape[1] % 2 != 1:
        raise ValueError("kernel bank must be [Z][K] with K odd")
    return K, (K.shape[1] - 1) // 2


def apply(K, R):
    """Y = A R.  K [Z][K]; R [Z][X] or [B][Z][X]."""
    K, h = _check(K)
    R = np.asarray(R, np.float64)
    squeeze = R.ndim == 2
    R3 = R[None] if squeeze else R
    B, Z, X = R3.shape
    if K.shape[0] != Z:
        raise ValueError("kernel bank rows must equal image rows")
    Y = np.zeros_like(R3)
    for m in range(-h, h + 1):
        for i in range(Z):
            s = i - m
            if 0 <= s < Z:
                Y[:, i, :] += K[i, m + h] * R3[:, s, :]
    return Y[0] if squeeze else Y


def adjoint(K, Yb):
    """Rbar = A^T Ybar.  Same shapes as ``apply``."""
    K, h = _check(K)
    Yb = np.asarray(Yb, np.float64)
    squeeze = Yb.ndim == 2
    Y3 = Yb[None] if squeeze else Yb
    B, Z, X = Y3.shape
    if K.shape[0] != Z:
        raise ValueError("kernel bank rows must equal image rows")
    Rb = np.zeros_like(Y3)
    for m in range(-h, h + 1):
        for s in range(Z):
            i = s + m
            if 0 <= i < Z:
                Rb[:, s, :] += K[i, m + h] * Y3[:, i, :]
    return Rb[0] if squeeze else Rb


def kernel_grad(R, Yb, K):
    """Kbar = dL/dK for Ybar = dL/dY: [Z][K] from R, Ybar ([Z][X] or [B][Z][X]) and the tap count K."""
    R = np.asarray(R, np.float64)
    Yb = np.asarray(Yb, np.float64)
    if R.shape != Yb.shape or R.ndim not in (2, 3):
        raise ValueError("R and Ybar must have the same [Z][X] or [B][Z][X] shape")
    if K < 1 or K % 2 != 1:
        raise ValueError("K must be odd")
    R3 = R[None] if R.ndim == 2 else R
    Y3 = Yb[None] if Yb.ndim == 2 else Yb
    Z = R3.shape[1]
    h = (K - 1) // 2
    G = np.zeros((Z, K), np.float64)
    for m in range(-h, h + 1):
        for i in range(Z):
            s = i - m
            if 0 <= s < Z:
                G[i, m + h] = np.sum(Y3[:, i, :] * R3[:, s, :])
    return G


def apply_lateral(Kx, Y):
    """Y2 = lateral pass of Y ([Z][X] or [B][Z][X]) with the row kernels Kx [Z][K]."""
    Kx, h = _check(Kx)
    Y = np.asarray(Y, np.float64)
    squeeze = Y.ndim == 2
    Y3 = Y[None] if squeeze else Y
    B, Z, X = Y3.shape
    if Kx.shape[0] != Z:
        raise ValueError("kernel bank rows must equal image rows")
    out = np.zeros_like(Y3)
    for m in range(-h, h + 1):
        for j in range(X):
            s = j - m
            if 0 <= s < X:
                out[:, :, j] += Kx[None, :, m + h] * Y3[:, :, s]
    return out[0] if squeeze else out


def matrix(K):
    """The banded Z x Z matrix M of the column operator: M[i][i-m] = K[i][m+h]."""
    K, h = _check(K)
    Z = K.shape[0]
    M = np.zeros((Z, Z), np.float64)
    for i in range(Z):
        for m in range(-h, h + 1):
            if 0 <= i - m < Z:
                M[i, i - m] = K[i, m + h]
    return M
