"""GPU parity of the kernel surrogate: per-row exact kernels and scales, input
features, MLP forward, gradients (vs the oracle's BF16-emulating backward),
Adam (vs FP64), training progress and bit-exact checkpoint / resume."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2507_15464_amd as td  # noqa: E402
from paper_2507_15464_amd import surrogate as sg  # noqa: E402
from oracle import kernels as o_k, mlp as o_mlp  # noqa: E402
from workloads import config, generators  # noqa: E402
from workloads.configs import SURROGATE  # noqa: E402
from tests.helpers import oracle_kw  # noqa: E402

pytestmark = pytest.mark.gpu
S5 = config(5)
LO = (S5.z0, SURROGATE["fnumber"][0], np.radians(SURROGATE["angle_deg"][0]), SURROGATE["fc"][0])
HI = (S5.z0 + (S5.nz - 1) * S5.dz, SURROGATE["fnumber"][1], np.radians(SURROGATE["angle_deg"][1]), SURROGATE["fc"][1])


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


def draws(n, seed):
    return generators.kernel_params(n, LO[0], HI[0], SURROGATE["fnumber"], SURROGATE["angle_deg"], SURROGATE["fc"],
                                    seed)


def oracle_row_kernel(p, K):
    z, F, a, fc = p
    s = S5.replace(fc=fc, fnumber=F, angles=(a,))
    return o_k.exact_kernels([z], S5.dz, K, **oracle_kw(s))[0]


def test_kernels_at_match_oracle(dev):
    P = draws(24, seed=5)
    P[0, 0] = 0.2e-3  # aperture empty: kernel 0, scale floored at 1
    k, s = sg.kernels_at(S5, S5.fs, S5.t0, S5.cycles, S5.n_samples, S5.dz, torch.from_numpy(P).to(dev), 129)
    k, s = k.cpu().numpy(), s.cpu().numpy()
    ref = np.stack([oracle_row_kernel(p, 129) for p in P])
    assert rel(k, ref) <= 1e-5
    sref = np.array([o_mlp.kernel_scale(p[0], p[1], S5.n_elem, S5.pitch) for p in P])
    assert np.max(np.abs(s - sref) / sref) <= 1e-6
    assert s[0] == 1.0 and np.all(k[0] == 0)
    kn, _ = sg.kernels_at(S5, S5.fs, S5.t0, S5.cycles, S5.n_samples, S5.dz, torch.from_numpy(P).to(dev), 129,
                          normalise=True)
    assert rel(kn.cpu().numpy(), ref / sref[:, None]) <= 1e-5


def test_features_match_oracle(dev):
    P = draws(1000, seed=6)
    x = sg.features(torch.from_numpy(P).to(dev), LO, HI).cpu().numpy()
    ref = o_mlp.features(P, LO, HI)
    assert np.max(np.abs(x - ref)) <= 1e-6
    assert np.all(np.abs(ref) <= 1.0 + 1e-12)


def net(seed, widths=(4, 256, 256, 256, 129)):
    p = generators.mlp_init(widths, seed)
    return [(W, 0.05 * generators.normal(W.shape[0], seed=seed + 10 + l)) for l, (W, _) in enumerate(p)]


def test_forward_matches_bf16_oracle(dev):
    layers = net(0)
    m = sg.Surrogate()
    m.load_layers(layers)
    x = generators.uniform((300, 4), -1, 1, seed=2).astype(np.float32)
    scale = generators.uniform(300, 1, 40, seed=3).astype(np.float32)
    y = m.forward(torch.from_numpy(x).to(dev)).cpu().numpy()
    ref, _ = o_mlp.forward(layers, x, bf16_mode=True)
    assert rel(y, ref) <= 2e-3
    ys = m.forward(torch.from_numpy(x).to(dev), torch.from_numpy(scale).to(dev)).cpu().numpy()
    assert rel(ys, ref * scale[:, None]) <= 2e-3
    # bf16 copy of the weights is exactly the oracle's rounding of the float32 masters
    w16 = m.params16.float().cpu().numpy()
    w32 = m.params.cpu().numpy()
    assert np.array_equal(w16, o_mlp.bf16(w32).astype(np.float32))


def test_train_step_gradients_match_bf16_oracle(dev):
    layers = net(1)
    m = sg.Surrogate()
    m.load_layers(layers)
    R, N = 700, 256
    x = generators.uniform((R, 4), -1, 1, seed=4).astype(np.float32)
    t = (0.3 * generators.normal((R, 129), seed=5)).astype(np.float32)
    idx = np.random.default_rng(6).choice(R, N, replace=False).astype(np.int32)
    loss = m.train_step(torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev),
                        idx=torch.from_numpy(idx).to(dev))
    y, cache = o_mlp.forward(layers, x[idx], bf16_mode=True)
    grads = o_mlp.backward(cache, y, t[idx], bf16_mode=True)
    assert abs(float(loss) - o_mlp.loss(y, t[idx])) <= 1e-4 * o_mlp.loss(y, t[idx])
    g = m.grad.cpu().numpy()
    off = 0
    for (dW, db) in grads:
        nW = dW.size
        assert rel(g[off:off + nW].reshape(dW.shape), dW) <= 5e-3
        off += nW
        assert rel(g[off:off + db.size], db) <= 5e-3
        off += db.size
    assert off == m.P


def test_adam_matches_fp64(dev):
    layers = net(2, (4, 16, 16, 16, 9))
    m = sg.Surrogate(widths=(4, 16, 16, 16, 9))
    m.load_layers(layers)
    rng = np.random.default_rng(7)
    g = rng.standard_normal(m.P).astype(np.float32)
    m.grad.copy_(torch.from_numpy(g))
    m.m.copy_(torch.from_numpy((0.1 * rng.standard_normal(m.P)).astype(np.float32)))
    m.v.copy_(torch.from_numpy((0.01 * rng.random(m.P)).astype(np.float32)))
    m.step = 4
    m0, v0, p0 = (t.cpu().numpy().astype(np.float64) for t in (m.m, m.v, m.params))
    m.adam(1e-3)
    c1, c2 = 1 - 0.9 ** 5, 1 - 0.999 ** 5
    mm = 0.9 * m0 + 0.1 * g
    vv = 0.999 * v0 + 0.001 * g.astype(np.float64) ** 2
    ref = p0 - 1e-3 * (mm / c1) / (np.sqrt(vv / c2) + 1e-8)
    assert np.max(np.abs(m.params.cpu().numpy() - ref)) <= 1e-6
    # and the same step through the oracle's per-layer Adam
    state = []
    off = 0
    for W, b in m.layers():
        nW = W.size
        state.append((m0[off:off + nW].reshape(W.shape), v0[off:off + nW].reshape(W.shape),
                      m0[off + nW:off + nW + b.size], v0[off + nW:off + nW + b.size]))
        off += nW + b.size
    grads = []
    off = 0
    for (W, b) in layers:
        grads.append((g[off:off + W.size].reshape(W.shape).astype(np.float64),
                      g[off + W.size:off + W.size + b.size].astype(np.float64)))
        off += W.size + b.size
    p_layers = []
    off = 0
    for (W, b) in layers:
        p_layers.append((p0[off:off + W.size].reshape(W.shape), p0[off + W.size:off + W.size + b.size]))
        off += W.size + b.size
    new, _ = o_mlp.adam_step(p_layers, grads, state, 1e-3, 5)
    flat = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in new])
    assert np.max(np.abs(m.params.cpu().numpy() - flat)) <= 1e-6


def small_dataset(dev, n, seed):
    P = torch.from_numpy(draws(n, seed)).to(dev)
    x = sg.features(P, LO, HI)
    t, _ = sg.kernels_at(S5, S5.fs, S5.t0, S5.cycles, S5.n_samples, S5.dz, P, 129, normalise=True)
    return x, t


def test_training_reduces_loss_and_resumes_bit_exactly(dev, tmp_path):
    x, t = small_dataset(dev, 4096, 11)
    idx = [torch.from_numpy(b.astype(np.int32)).to(dev) for b in generators.batch_indices(4096, 256, 120, seed=3)]
    layers = [(W, b) for W, b in generators.mlp_init((4, 256, 256, 256, 129), 0)]
    a = sg.Surrogate()
    a.load_layers(layers)
    first = float(a.train_step(x, t, idx=idx[0]))
    a.fit(x, t, idx, total_steps=120)
    last = float(a.train_step(x, t, idx=idx[0]))
    assert last < 0.5 * first
    b = sg.Surrogate()
    b.load_layers(layers)
    b.fit(x, t, idx[:60], total_steps=120)
    b.save(tmp_path / "ck.pt")
    c = sg.Surrogate()
    c.load(tmp_path / "ck.pt")
    c.fit(x, t, idx[60:], total_steps=120)
    assert c.step == a.step == 120
    assert torch.equal(c.params, a.params) and torch.equal(c.m, a.m) and torch.equal(c.v, a.v)
