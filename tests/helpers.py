"""Shared test helpers: turning a workload Setup into oracle arguments and
into pixel axes.  No arithmetic of the method lives here."""
import numpy as np


def oracle_kw(s, **over):
    kw = dict(n_elem=s.n_elem, pitch=s.pitch, c=s.c, fs=s.fs, t0=s.t0, fc=s.fc, sigma=s.sigma,
              n_samples=s.n_samples, angles=list(s.angles), fnumber=s.fnumber)
    kw.update(over)
    return kw


def das_kw(s):
    return dict(n_elem=s.n_elem, pitch=s.pitch, c=s.c, fs=s.fs, t0=s.t0, angles=list(s.angles),
                fnumber=s.fnumber)


def sim_kw(s):
    return dict(n_elem=s.n_elem, pitch=s.pitch, c=s.c, fs=s.fs, t0=s.t0, fc=s.fc, sigma=s.sigma,
                n_samples=s.n_samples, angles=list(s.angles))


def axes(s):
    xs = s.x0 + np.arange(s.nx) * s.dx
    zs = s.z0 + np.arange(s.nz) * s.dz
    return xs, zs
