"""What the trained surrogate gains over the method without it.

Without the network, a kernel bank for a new (depth, F-number, angle, fc)
configuration comes from the paper's own cheap strategy -- a small set of
predefined delay profiles, each row taking the fixed-delay kernel of its
nearest reference depth scaled by its least-squares weight theta (Sec. 2.3
eqn:theta; Sec. 3.3-3.4 and Sec. 4: a few representative profiles serve a
whole line) -- or from the exact derivation (DAS of a unit echo per row and
tap).  The test trains a surrogate briefly on the device and shows, on
held-out configurations, that its bank is closer to the exact bank than the
paper-mode bank of equal or lower build time (one delay curve per line),
reporting the banks from 16 and 64 profiles beside it, and that it is closer
than a nearest-neighbour table holding as many numbers as the network has
parameters; it also exercises the exact-kernel fallback driven by the error
judge.  Build times are measured by bench.py (surrogate workload), not
asserted here.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2507_15464_amd import surrogate as sg  # noqa: E402
from workloads import config, generators  # noqa: E402
from workloads.configs import SURROGATE  # noqa: E402

pytestmark = pytest.mark.gpu
S5 = config(5)
LO = (S5.z0, SURROGATE["fnumber"][0], np.radians(SURROGATE["angle_deg"][0]), SURROGATE["fc"][0])
HI = (S5.z0 + (S5.nz - 1) * S5.dz, SURROGATE["fnumber"][1], np.radians(SURROGATE["angle_deg"][1]), SURROGATE["fc"][1])


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def draws(n, seed, dev):
    P = generators.kernel_params(n, LO[0], HI[0], SURROGATE["fnumber"], SURROGATE["angle_deg"], SURROGATE["fc"], seed)
    return torch.from_numpy(P).to(dev)


@pytest.fixture(scope="module")
def trained(dev):
    n, steps = 65536, 3000
    P = draws(n, 0, dev)
    x = sg.features(P, LO, HI)
    t, _ = sg.kernels_at(S5, S5.fs, S5.t0, S5.cycles, S5.n_samples, S5.dz, P, S5.K, normalise=True)
    m = sg.Surrogate()
    m.load_layers([(W, b) for W, b in generators.mlp_init(SURROGATE["widths"], 0)])
    idx = torch.from_numpy(generators.batch_indices(n, 1024, steps, seed=2).astype(np.int32)).to(dev)
    m.fit(x, t, [idx[i] for i in range(steps)], total_steps=steps)
    return m


def test_surrogate_beats_equal_memory_table_on_heldout_draws(dev, trained):
    K = S5.K
    P_te = draws(2048, 1, dev)
    ex, s = sg.kernels_at(S5, S5.fs, S5.t0, S5.cycles, S5.n_samples, S5.dz, P_te, K)
    pred = trained.forward(sg.features(P_te, LO, HI), scale=s)
    err_net = sg.rel_l2(pred, ex)
    # table of exact normalised kernels with as many numbers as the network has parameters
    n_tab = trained.P // K
    P_tab = draws(n_tab, 4, dev)
    tab, _ = sg.kernels_at(S5, S5.fs, S5.t0, S5.cycles, S5.n_samples, S5.dz, P_tab, K, normalise=True)
    xt = sg.features(P_tab, LO, HI).cpu().numpy().astype(np.float64)
    xq = sg.features(P_te, LO, HI).cpu().numpy().astype(np.float64)
    nn = np.argmin(((xq[:, None, :] - xt[None, :, :]) ** 2).sum(-1), axis=1)
    table_pred = tab.cpu().numpy()[nn] * s.cpu().numpy()[:, None]
    exn = ex.cpu().numpy().astype(np.float64)
    err_tab = np.linalg.norm(table_pred - exn) / np.linalg.norm(exn)
    print(f"held-out rel-L2: surrogate {err_net:.3e}, nearest-of-{n_tab} table {err_tab:.3e}")
    assert err_net < err_tab


# held-out image configurations (F-number, angle in degrees, fc): none of them
# is a training draw (those are continuous uniform draws of another seed)
HELD_OUT_CONFIGS = [(1.5, 0.0, 7.5e6), (2.3, -7.0, 4.2e6), (1.2, 11.0, 9.1e6)]


@pytest.mark.parametrize("fnum,angle_deg,fc", HELD_OUT_CONFIGS)
def test_surrogate_beats_paper_mode_profiles(dev, trained, fnum, angle_deg, fc):
    """Surrogate bank vs paper-mode banks from reference profiles, all against
    the exact bank of the same configuration.  A paper-mode build costs more
    than the surrogate's forward pass at any number of profiles (bench.py,
    surrogate workload, measures both), so at equal or lower build time the
    paper's strategy has one delay curve for the line -- its own line setting
    (Sec. 3.4) -- and the test asserts the surrogate is closer than that; the
    banks with 16 and 64 profiles (one per 128 and 32 rows) are reported
    beside it."""
    import paper_2507_15464_amd as td
    K, Z = S5.K, S5.nz
    zs = S5.z0 + np.arange(Z) * S5.dz
    P = torch.from_numpy(np.stack([zs, np.full(Z, fnum), np.full(Z, np.radians(angle_deg)), np.full(Z, fc)], 1))
    P = P.to(dev)
    exact, s = sg.kernels_at(S5, S5.fs, S5.t0, S5.cycles, S5.n_samples, S5.dz, P, K)
    net = trained.forward(sg.features(P, LO, HI), scale=s)
    setup = S5.replace(fnumber=fnum, fc=fc, angles=(float(np.radians(angle_deg)),))
    # the surrogate's data generator and the library's exact mode agree (FP64 builds, float32 out)
    assert sg.rel_l2(td.build_kernels(setup, K=K, mode="exact"), exact) <= 1e-6
    err = {}
    for per in (Z, 128, 32):
        refs = np.minimum((np.arange(Z) // per) * per + per // 2, Z - 1)
        err[per] = sg.rel_l2(td.build_kernels(setup, K=K, mode="paper", ref_row=refs), exact)
    err_net = sg.rel_l2(net, exact)
    print(f"F#{fnum} {angle_deg} deg {fc / 1e6} MHz: surrogate {err_net:.3e}, paper mode "
          f"1 profile {err[Z]:.3e}, 16 profiles {err[128]:.3e}, 64 profiles {err[32]:.3e}")
    assert err_net < err[Z]


def test_error_judge_falls_back_to_exact_kernels(dev, trained):
    K, Z = S5.K, 256
    zs = S5.z0 + (np.arange(Z) * 8) * S5.dz
    P = torch.from_numpy(np.stack([zs, np.full(Z, 2.0), np.full(Z, 0.1), np.full(Z, 5e6)], 1)).to(dev)
    exact, _ = sg.kernels_at(S5, S5.fs, S5.t0, S5.cycles, S5.n_samples, S5.dz, P, K)
    bank, info = trained.kernel_bank(S5, P, LO, HI, judge_rows=16, tol=1e-9)
    assert info["fallback"] and torch.equal(bank, exact)
    bank2, info2 = trained.kernel_bank(S5, P, LO, HI, judge_rows=16, tol=10.0)
    assert not info2["fallback"] and info2["judge_rel_l2"] > 0
    assert sg.rel_l2(bank2, exact) < 1.0
