"""GPU tests of the warm-start MLP (BF16 MFMA GEMMs, FP32 accumulate) against
the FP64 NumPy oracle, through the C ABI.

The GPU multiplies BF16 copies of the weights and of every layer's input
activations.  The oracle therefore runs on BF16-rounded weights and inputs;
the remaining differences come from rounding the hidden activations (and the
back-propagated gradients) to BF16, about 2^-9 relative per element, so the
bar is 2e-2 relative in norm per layer.
"""
import numpy as np
import pytest

import synthmesh as sm
from oracle import mlp_oracle as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL = 2e-2


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_06347_amd import cgks
    return cgks


def bf16(a):
    """Round to bfloat16 (nearest even) and return as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflat(v, sizes=M.SIZES):
    out, o = [], 0
    for i in range(len(sizes) - 1):
        n_in, n_out = sizes[i], sizes[i + 1]
        W = v[o:o + n_in * n_out].reshape(n_out, n_in).astype(np.float64)
        o += n_in * n_out
        b = v[o:o + n_out].astype(np.float64)
        o += n_out
        out.append([W, b])
    return out


def params(seed):
    p = M.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for layer in p:
        layer[1] = rng.normal(scale=0.1, size=layer[1].shape)
    # keep the master weights representable in float32, as the library holds them
    return [[W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)] for W, b in p]


def data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 5)).astype(np.float32)
    A = rng.normal(size=(5, 4)) / np.sqrt(5)
    Y = np.tanh(X.astype(np.float64) @ A).astype(np.float32)
    return X, Y


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


@pytest.mark.parametrize("n", [37, 1000, 4133])
def test_forward_matches_oracle(cg, n):
    p = params(7)
    net = cg.MLP(seed=1)
    net.set_weights(flat(p))
    X, _ = data(n, 11 + n)
    Yd = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    net.forward(dev(X), Yd)
    got = Yd.cpu().numpy().astype(np.float64)
    ref, _ = M.forward([[bf16(W), b] for W, b in p], bf16(X))
    assert np.all(np.isfinite(got))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel < REL, rel


def test_weights_roundtrip(cg):
    p = params(3)
    net = cg.MLP(seed=2)
    net.set_weights(flat(p))
    assert np.array_equal(net.get_weights(), flat(p).astype(np.float32))
    assert net.get_weights().size == sum(W.size + b.size for W, b in p)


@pytest.mark.parametrize("n", [200, 5000])
def test_gradients_match_oracle(cg, n):
    """n = 5000 exercises the split-K weight-gradient path with a ragged last chunk."""
    p = params(5)
    net = cg.MLP(seed=1)
    net.set_weights(flat(p))
    X, Y = data(n, 21 + n)
    loss, g = net.grads(dev(X), dev(Y))
    pb = [[bf16(W), b] for W, b in p]
    ref_loss = M.loss(pb, bf16(X), Y.astype(np.float64))
    ref = M.grads(pb, bf16(X), Y.astype(np.float64))
    assert abs(loss - ref_loss) <= REL * ref_loss
    got = unflat(g)
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(got, ref)):
        for name, a, r in (("W", gW, rW), ("b", gb, rb)):
            rel = np.linalg.norm(a - r) / np.linalg.norm(r)
            assert rel < REL, (li, name, rel)


def test_adam_step_matches_oracle(cg):
    """One Adam step from the GPU's own gradient equals the oracle's step."""
    p = params(9)
    net = cg.MLP(seed=1)
    net.set_weights(flat(p))
    X, Y = data(777, 31)
    w0 = net.get_weights().astype(np.float64)
    _, g = net.grads(dev(X), dev(Y))
    lr = 1e-3
    net.train_step(dev(X), dev(Y), lr)
    w1 = net.get_weights().astype(np.float64)
    ref = M.adam_step(unflat(w0), unflat(g.astype(np.float64)), {"t": 0}, lr=lr)
    np.testing.assert_allclose(w1, flat(ref), rtol=1e-6, atol=1e-9)


def test_training_is_reproducible_and_reduces_loss(cg):
    X, Y = data(4096, 41)
    Xd, Yd = dev(X), dev(Y)
    nets = [cg.MLP(seed=4), cg.MLP(seed=4)]
    losses = [[], []]
    for _ in range(150):
        for k in range(2):
            losses[k].append(nets[k].train_step(Xd, Yd, 1e-3))
    assert losses[0] == losses[1]
    assert np.array_equal(nets[0].get_weights(), nets[1].get_weights())
    assert losses[0][-1] < 0.2 * losses[0][0], (losses[0][0], losses[0][-1])


def _solver(cg):
    mesh = sm.annulus(12, 4, jitter=0.1, seed=3, nref=1, wall_tag=sm.SLIP)
    return cg.Solver(mesh, n_levels=2, mach=0.38)


def test_warm_start_from_zero_network_is_free_stream(cg):
    net = cg.MLP(seed=0)
    net.set_weights(np.zeros(net.num_params(), dtype=np.float32))
    s = _solver(cg)
    s.init_freestream()
    Wf, _, _ = s.get_state()
    s.set_state(np.zeros_like(Wf))
    nfb = net.init_solver(s, np.zeros(5), np.ones(5), [0.0, 1.0, 0.0, 0.0], np.ones(4))
    W, G, A = s.get_state()
    assert nfb == 0
    np.testing.assert_allclose(W, Wf, rtol=1e-15, atol=1e-15)
    assert np.all(G == 0.0) and np.all(A == 1.0)


def test_warm_start_falls_back_on_garbage_weights(cg):
    net = cg.MLP(seed=0)
    net.set_weights(np.full(net.num_params(), 1e30, dtype=np.float32))
    s = _solver(cg)
    s.init_freestream()
    Wf, _, _ = s.get_state()
    s.set_state(np.zeros_like(Wf))
    nfb = net.init_solver(s, np.zeros(5), np.ones(5), np.zeros(4), np.ones(4))
    W, _, _ = s.get_state()
    assert nfb == W.shape[0]
    np.testing.assert_allclose(W, Wf, rtol=1e-15, atol=1e-15)


def test_warm_start_state_is_physical_and_usable(cg):
    net = cg.MLP(seed=6)
    s = _solver(cg)
    nfb = net.init_solver(s, np.zeros(5), np.full(5, 4.0), np.zeros(4), np.full(4, 0.05))
    W, _, _ = s.get_state()
    assert 0 <= nfb < W.shape[0]
    assert np.all(W[:, 0] > 0) and np.all(np.isfinite(W))
    p = 0.4 * (W[:, 3] - 0.5 * (W[:, 1] ** 2 + W[:, 2] ** 2) / W[:, 0])
    assert np.all(p > 0)
    n = s.vcycle()
    assert np.isfinite(n)


def test_device_features_follow_their_definition(cg):
    """cgks_mlp_features (the one feature kernel behind training data and the
    warm start): Mach, log10 Re, centroid, distance to the nearest wall-face
    centre, against the definition evaluated here in FP64."""
    mesh = sm.annulus(12, 4, jitter=0.1, seed=3, nref=1, wall_tag=sm.ISOTHERMAL)
    s = cg.Solver(mesh, n_levels=2, mach=0.25, reynolds=35.0)
    X = s.mlp_features()
    _, C = s.cell_geometry(0)
    wall = mesh.btags == sm.ISOTHERMAL
    wc = mesh.coords[mesh.bfaces[wall]].mean(axis=1)
    d = np.sqrt(((C[:, None, :] - wc[None, :, :]) ** 2).sum(axis=2).min(axis=1))
    ref = np.column_stack([np.full(len(C), 0.25), np.full(len(C), np.log10(35.0)), C[:, 0], C[:, 1], d])
    np.testing.assert_allclose(X, ref, rtol=2e-7, atol=1e-7)


def test_warm_start_outside_training_range_falls_back(cg):
    """A problem whose Mach number lies outside the network's training range
    starts from the free stream in every cell; inside it, the network is used."""
    net = cg.MLP(seed=6)
    s = _solver(cg)
    s.init_freestream()
    Wf, _, _ = s.get_state()
    X = s.mlp_features()
    lo, hi = X.min(axis=0), X.max(axis=0)
    lo[0], hi[0] = 0.5, 0.8                    # Mach 0.38 is outside
    net.set_range(lo, hi)
    s.set_state(np.zeros_like(Wf))
    nfb = net.init_solver(s, np.zeros(5), np.full(5, 4.0), np.zeros(4), np.full(4, 0.05))
    W, _, _ = s.get_state()
    assert nfb == W.shape[0]
    np.testing.assert_allclose(W, Wf, rtol=1e-15, atol=1e-15)
    lo[0], hi[0] = 0.3, 0.5                    # inside
    net.set_range(lo, hi)
    nfb = net.init_solver(s, np.zeros(5), np.full(5, 4.0), np.zeros(4), np.full(4, 0.05))
    assert nfb < W.shape[0]
    net.set_range(None, None)
