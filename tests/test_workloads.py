"""The seeded workload generators produce the shapes and ranges the workloads state."""
import numpy as np

from workloads import config, generators
from workloads.configs import CYSTS, RAGGED, SURROGATE


def test_ragged_sizes_match_workload_ranges():
    sizes = generators.ragged_sizes(RAGGED["n_frames"], RAGGED["x_lo"], RAGGED["x_hi"], RAGGED["z_lo"],
                                    RAGGED["z_hi"], seed=0)
    assert len(sizes) == 64
    assert all(512 <= nz <= 2048 and 256 <= nx <= 512 for nz, nx in sizes)
    assert sizes == generators.ragged_sizes(64, 256, 512, 512, 2048, seed=0)


def test_speckle_phantom_cysts_are_empty_and_inside_the_field():
    s = config(2)
    x, z, a, cysts = generators.speckle_with_cysts(20000, s.field_w, s.field_d, CYSTS["n"], CYSTS["r_lo"],
                                                   CYSTS["r_hi"], seed=3)
    assert len(cysts) == 5
    for cx, cz, r in cysts:
        assert 2e-3 <= r <= 4e-3
        assert -0.5 * s.field_w + r <= cx <= 0.5 * s.field_w - r and r <= cz <= s.field_d - r
        assert np.all((x - cx) ** 2 + (z - cz) ** 2 > r * r)
    assert np.all(np.abs(x) <= 0.5 * s.field_w) and np.all((z >= 0) & (z <= s.field_d))


def test_spikes_distinct_and_counted():
    R = generators.spikes(64, 32, 100, seed=1)
    assert np.count_nonzero(R) == 100


def test_kernel_param_draw_ranges():
    P = generators.kernel_params(5000, 1e-3, 60e-3, SURROGATE["fnumber"], SURROGATE["angle_deg"], SURROGATE["fc"], 0)
    assert P.shape == (5000, 4)
    assert np.all((P[:, 1] >= 1) & (P[:, 1] <= 3))
    assert np.all(np.abs(P[:, 2]) <= np.radians(15) + 1e-12)
    assert np.all((P[:, 3] >= 3e6) & (P[:, 3] <= 10e6))


def test_grid_fills_the_field():
    for k in (1, 2, 4, 5):
        s = config(k)
        assert abs(s.x0 - (-0.5 * s.field_w + 0.5 * s.dx)) < 1e-15
        assert abs(s.z0 + (s.nz - 1) * s.dz - (s.field_d - 0.5 * s.dz)) < 1e-12
