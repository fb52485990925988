"""Transmitted pulse (oracle; test infrastructure only).

The paper leaves the pulse S^F unspecified (Sec. 2, eqn:SRX).  The workloads
use a Gaussian-modulated cosine whose envelope FWHM spans ``cycles`` periods
of the centre frequency, peaking at t = 0 and truncated to zero beyond four
standard deviations of the envelope.
"""
import numpy as np

# FWHM of a Gaussian = 2 sqrt(2 ln 2) sigma
FWHM_PER_SIGMA = 2.0 * np.sqrt(2.0 * np.log(2.0))
TRUNC_SIGMAS = 4.0


def pulse_sigma(fc, cycles):
    """Envelope standard deviation for an envelope FWHM of ``cycles`` periods."""
    return (float(cycles) / float(fc)) / FWHM_PER_SIGMA


def pulse(t, fc, sigma):
    """p(t) = exp(-t^2 / (2 sigma^2)) cos(2 pi fc t), zero for |t| > 4 sigma."""
    t = np.asarray(t, np.float64)
    v = np.exp(-t * t / (2.0 * sigma * sigma)) * np.cos(2.0 * np.pi * fc * t)
    return np.where(np.abs(t) <= TRUNC_SIGMAS * sigma, v, 0.0)
