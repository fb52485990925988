"""Parameter sets of the five workloads (SI units).

1. small plain case: 64 elements, 0.3 mm pitch, 5 MHz 2-cycle pulse, 40 MHz
   sampling, 2048 samples, one 0-degree plane wave, 20 point scatterers in a
   19 x 40 mm field, image 128 lateral x 256 depth, Hann F/1.5, 65 taps.
2. clinical plain case: 128 elements, 7.5 MHz, 50 MHz, 4096 samples, speckle
   of 100k scatterers in 38 x 60 mm with 5 anechoic cysts (radius 2-4 mm),
   image 256 x 1024, 129 taps.
3. batching: 64 frames of ragged sizes (256..512 lateral x 512..2048 depth),
   11 plane waves from -10 to +10 degrees compounded, array of case 1.
4. differentiation: 256 x 1024 image with case-1 geometry, 65 taps, 500
   spikes + 40 dB noise, lambda 1e-3, 200 gradient iterations.
5. learned kernels: array of case 2, rows of a 512 x 2048 image over
   38 x 60 mm, 129 taps; draws of depth, F-number in [1, 3], angle in
   [-15, 15] degrees, centre frequency in [3, 10] MHz.

The single-point study (the paper's Sec. 3.1-3.3 set-up, its open
parameters read as stated here): 192 elements at 0.3 mm pitch, 50 MHz
sampling, 3200 samples, 2-cycle pulse, receive F-number 1, 600 points
from 2 to 42 mm on the axis, transmit focus at 15, 25 or 35 mm with a
Kossoff aperture (parameter 0.6), centre frequencies 3 to 9 MHz.
"""
from dataclasses import dataclass, replace
import math


@dataclass(frozen=True)
class Setup:
    n_elem: int
    pitch: float
    c: float
    fs: float
    t0: float
    fc: float
    cycles: float
    n_samples: int
    angles: tuple
    fnumber: float
    nz: int
    nx: int
    z0: float
    dz: float
    x0: float
    dx: float
    K: int
    field_w: float
    field_d: float

    @property
    def sigma(self):
        """Envelope standard deviation of a pulse whose envelope FWHM spans
        ``cycles`` periods (FWHM = 2 sqrt(2 ln 2) sigma)."""
        return (self.cycles / self.fc) / (2.0 * math.sqrt(2.0 * math.log(2.0)))

    def with_grid(self, nz, nx):
        return replace(self, **field_grid(self.field_w, self.field_d, nz, nx))

    def replace(self, **kw):
        return replace(self, **kw)


def field_grid(width, depth, nz, nx):
    """Pixel centres filling the field: x in [-W/2, W/2], z in (0, D]."""
    dx = width / nx
    dz = depth / nz
    return dict(nz=nz, nx=nx, dz=dz, dx=dx, z0=0.5 * dz, x0=-0.5 * width + 0.5 * dx)


def _setup(n_elem, fc, fs, n_samples, width, depth, nz, nx, K, angles=(0.0,)):
    return Setup(n_elem=n_elem, pitch=0.3e-3, c=1540.0, fs=fs, t0=0.0, fc=fc, cycles=2.0,
                 n_samples=n_samples, angles=tuple(angles), fnumber=1.5, K=K,
                 field_w=width, field_d=depth, **field_grid(width, depth, nz, nx))


ANGLES_11 = tuple(math.radians(a) for a in range(-10, 11, 2))

CONFIGS = {
    1: _setup(64, 5e6, 40e6, 2048, 19e-3, 40e-3, 256, 128, 65),
    2: _setup(128, 7.5e6, 50e6, 4096, 38e-3, 60e-3, 1024, 256, 129),
    3: _setup(64, 5e6, 40e6, 2048, 19e-3, 40e-3, 512, 256, 65, angles=ANGLES_11),
    4: _setup(64, 5e6, 40e6, 2048, 19e-3, 40e-3, 1024, 256, 65),
    5: _setup(128, 7.5e6, 50e6, 4096, 38e-3, 60e-3, 2048, 512, 129),
}

# workload constants that are not geometry
N_SCATTERERS = {1: 20, 2: 100_000, 3: 20}
CYSTS = dict(n=5, r_lo=2e-3, r_hi=4e-3)
RAGGED = dict(n_frames=64, x_lo=256, x_hi=512, z_lo=512, z_hi=2048)
DECONV = dict(n_spikes=500, snr_db=40.0, lam=1e-3, iters=200)
SURROGATE = dict(n_train=200_000, fnumber=(1.0, 3.0), angle_deg=(-15.0, 15.0), fc=(3e6, 10e6),
                 widths=(4, 256, 256, 256, 129), batch=1024)


def config(k):
    return CONFIGS[int(k)]


STUDY = dict(n_elem=192, pitch=0.3e-3, fs=50e6, n_samples=3200, fnumber=1.0, n_points=600, z_first=2e-3,
             z_last=42e-3, foci=(15e-3, 25e-3, 35e-3), fcs=(3e6, 5e6, 7e6, 9e6), kossoff=0.6)


def study_setup(fc, **over):
    """Setup of the single-point study at centre frequency fc (one 0-degree
    angle: the focused beam is unsteered; the grid fields describe the
    axial line of points)."""
    p = dict(STUDY, **over)
    n = p["n_points"]
    dz = (p["z_last"] - p["z_first"]) / (n - 1)
    return Setup(n_elem=p["n_elem"], pitch=p["pitch"], c=1540.0, fs=p["fs"], t0=0.0, fc=fc, cycles=2.0,
                 n_samples=p["n_samples"], angles=(0.0,), fnumber=p["fnumber"], nz=n, nx=1, z0=p["z_first"], dz=dz,
                 x0=0.0, dx=p["pitch"], K=1, field_w=p["n_elem"] * p["pitch"], field_d=p["z_last"])


def study_line_half(setup):
    """Half length of the whole line in fine samples: the span of the points."""
    return int(math.ceil((setup.nz - 1) * setup.dz / (setup.c / (2.0 * setup.fs))))


def study_focal_index(setup, z_focus):
    """The point nearest the requested focal depth."""
    return int(round((z_focus - setup.z0) / setup.dz))
