"""GPU parity of ragged multi-frame, multi-angle batches (one persistent launch
per batch): every launch variant gives bit-identical results, equal to the
per-frame entry points and to the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2507_15464_amd as td  # noqa: E402
from paper_2507_15464_amd import _lib  # noqa: E402
from oracle import das as o_das, simulate as o_sim, tidas as o_t  # noqa: E402
from workloads import config, generators  # noqa: E402
from tests.helpers import axes, das_kw, sim_kw  # noqa: E402

pytestmark = pytest.mark.gpu
RTOL = 1e-5


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def g(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


SMALL_GRIDS = [(70, 33), (130, 64), (64, 4), (200, 37), (1, 5), (65, 8)]


def ragged_das_inputs(grids, seed0):
    base = config(3)
    frames = []
    for f, (nz, nx) in enumerate(grids):
        s = base.with_grid(nz, nx)
        x, z, a = generators.point_scatterers(20, s.field_w, s.field_d, seed=seed0 + f)
        rf = o_sim.to_fp32(o_sim.simulate_rf(x, z, a, **sim_kw(s)))
        frames.append((s, rf))
    return frames


def test_das_batch_all_variants_match_oracle_and_single_launch(dev):
    frames = ragged_das_inputs(SMALL_GRIDS, 50)
    setup = frames[0][0]
    rfs = [g(rf, dev) for _, rf in frames]
    grids = [s for s, _ in frames]
    results = []
    for v in range(_lib.DAS_BATCH_VARIANTS):
        outs = td.das_beamform_batch(setup, grids, rfs, variant=v)
        results.append([o.cpu().numpy() for o in outs])
    for v in range(1, len(results)):
        for f in range(len(frames)):
            assert np.array_equal(results[v][f], results[0][f]), (v, f)
    for f, (s, rf) in enumerate(frames):
        single = td.das_beamform(rfs[f], s).cpu().numpy()
        assert np.array_equal(single, results[0][f])
        xs, zs = axes(s)
        assert rel(results[0][f], o_das.das(rf, xs, zs, **das_kw(s))) <= RTOL


def test_apply_batch_all_variants_match_oracle_and_single_launch(dev):
    shapes = [(100, 64), (513, 257), (64, 255), (1, 3), (300, 256), (97, 512)]
    K = 65
    kbs = [generators.normal((Z, K), seed=10 + i).astype(np.float32) for i, (Z, X) in enumerate(shapes)]
    Rs = [generators.normal((Z, X), seed=20 + i).astype(np.float32) for i, (Z, X) in enumerate(shapes)]
    kd = [g(k, dev) for k in kbs]
    rd = [g(r, dev) for r in Rs]
    results = []
    for v in range(_lib.APPLY_BATCH_VARIANTS):
        results.append([o.cpu().numpy() for o in td.apply_batch(kd, rd, variant=v)])
    for v in range(1, len(results)):
        for f in range(len(shapes)):
            assert np.array_equal(results[v][f], results[0][f]), (v, f)
    for f in range(len(shapes)):
        single = td.apply(kd[f], rd[f]).cpu().numpy()
        assert np.array_equal(single, results[0][f])
        assert rel(results[0][f], o_t.apply(kbs[f], Rs[f])) <= RTOL


def test_full_size_ragged_batch_sampled_pixels(dev):
    """Frames at the batching workload's extreme sizes (512 x 2048 and the
    smallest 256 x 512), 11 compounded angles; the oracle computes a sampled
    sub-grid of each."""
    grids = [(2048, 512), (512, 256), (1500, 333)]
    frames = ragged_das_inputs(grids, 70)
    setup = frames[0][0]
    rfs = [g(rf, dev) for _, rf in frames]
    outs = td.das_beamform_batch(setup, [s for s, _ in frames], rfs, variant=3)
    rng = np.random.default_rng(3)
    for f, (s, rf) in enumerate(frames):
        img = outs[f].cpu().numpy()
        rows = np.sort(rng.choice(s.nz, 24, replace=False))
        cols = np.sort(rng.choice(s.nx, 12, replace=False))
        xs, zs = axes(s)
        ref = o_das.das(rf, xs[cols], zs[rows], **das_kw(s))
        assert rel(img[np.ix_(rows, cols)], ref) <= RTOL


def test_full_size_ragged_line_model_four_block_variant(dev):
    """The line model's four-block batch variant (band images of every frame
    prepared in the workspace, one workgroup per 128-row tile walking the
    frame's column tiles) on frames at the batching workload's extreme sizes
    and ragged ones: the same bits as the persistent two-block variant and as
    single launches; sampled rows against the oracle.  Widths run past a
    multiple of 256 by 1, 32, 44, 77 and 88 columns, one of them into a third
    column tile."""
    shapes = [(2048, 512), (512, 256), (1500, 333), (129, 300), (640, 257), (150, 288), (200, 600)]
    K = 65
    kbs = [generators.normal((Z, K), seed=30 + i).astype(np.float32) for i, (Z, X) in enumerate(shapes)]
    Rs = [generators.normal((Z, X), seed=40 + i).astype(np.float32) for i, (Z, X) in enumerate(shapes)]
    kd = [g(k, dev) for k in kbs]
    rd = [g(r, dev) for r in Rs]
    four = td.apply_batch(kd, rd, variant=_lib.APPLY_BATCH_FOUR_BLOCK)
    two = td.apply_batch(kd, rd, variant=0)
    # prepared once, applied twice (the maps change between the calls)
    pb = td.PreparedBatch(kd, rd)
    first = [o.clone() for o in pb.apply()]
    for r in rd:
        r.mul_(-2.0)
    second = pb.apply()
    rng = np.random.default_rng(5)
    for f, (Z, X) in enumerate(shapes):
        assert torch.equal(first[f], four[f]), f
        assert torch.equal(second[f], td.apply(kd[f], rd[f])), f
        rd[f].mul_(-0.5)
        assert torch.equal(four[f], two[f]), f
        assert torch.equal(four[f], td.apply(kd[f], rd[f])), f
        rows = np.sort(rng.choice(Z, 16, replace=False))
        full = o_t.apply(kbs[f], Rs[f])
        assert rel(four[f].cpu().numpy()[rows], full[rows]) <= RTOL


def test_autotuner_picks_and_caches_a_variant(dev, tmp_path, monkeypatch):
    monkeypatch.setenv("TIDAS_TUNE_CACHE", str(tmp_path / "tune.json"))
    shapes = [(256, 256), (512, 300)]
    kd = [g(generators.normal((Z, 65), seed=i), dev) for i, (Z, X) in enumerate(shapes)]
    rd = [g(generators.normal((Z, X), seed=9 + i), dev) for i, (Z, X) in enumerate(shapes)]
    outs = [torch.empty_like(r) for r in rd]
    best, times = td.autotune.tune("apply_batch", lambda v: td.apply_batch(kd, rd, outs, variant=v), key="test")
    assert 0 <= best < _lib.APPLY_BATCH_VARIANTS and len(times) == _lib.APPLY_BATCH_VARIANTS
    assert td.autotune.lookup("apply_batch", "test") == best
    again, t2 = td.autotune.tune("apply_batch", lambda v: td.apply_batch(kd, rd, outs, variant=v), key="test")
    assert again == best and t2 is None

