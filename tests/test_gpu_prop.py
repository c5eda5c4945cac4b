"""GPU checks of the proposal network against the FP64 reference (oracle.mlp):
forward outputs, gradients, descriptors, features, ranking and training."""
import sys

import numpy as np
import pytest

import synth
from oracle import mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_05075_amd as p
    p.load_library()
    return p


def _inputs(n, seed):
    g = np.random.default_rng(seed)
    q = synth.random_quaternions(n, seed)
    da = mlp.descriptor(synth.mixture_balls(300, seed))
    db = mlp.descriptor(synth.mixture_balls(200, seed + 1))
    X = mlp.features(q, da, db)
    y = g.standard_normal(n) * 0.1
    return X, y


def test_forward_matches_reference(pkg):
    _say("case: forward, 256 rows (matrix-core layout check)")
    p = pkg.Proposer(batch=128, seed=3)
    X, _ = _inputs(256, 11)
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    out = p.predict(Xt).double().cpu().numpy()
    ref, _ = mlp.forward(pkg.unpack_params(p.get_params().astype(np.float64)), X.astype(np.float32), quant=True)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    _say("  forward max error / max |y| = %.3g" % err)
    assert err <= 1e-2
    p.close()


def test_gradient_matches_reference(pkg):
    _say("case: gradient of one batch of 100 (64-row padding exercised)")
    p = pkg.Proposer(batch=128, seed=5)
    X, y = _inputs(100, 21)
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    g = p.gradient(Xt, yt).astype(np.float64)
    params = pkg.unpack_params(p.get_params().astype(np.float64))
    out, cache = mlp.forward(params, X.astype(np.float32), quant=True)
    ref = mlp.backward(cache, out, y.astype(np.float32))
    got = pkg.unpack_params(g)
    for l in range(4):
        for k, name in ((0, "W"), (1, "b")):
            a, r = got[l][k].reshape(-1), ref[l][k].reshape(-1)
            err = np.abs(a - r).max() / max(np.abs(r).max(), 1e-30)
            _say("  layer %d %s: max error / max |grad| = %.3g" % (l + 1, name, err))
            assert err <= 1e-2
    p.close()


def test_descriptor_and_features_match_reference(pkg):
    p = pkg.Proposer(batch=64, seed=1)
    A = synth.mixture_balls(5000, 77)
    B = synth.mixture_balls(1500, 78)
    da, db = p.descriptor(A), p.descriptor(B)
    np.testing.assert_allclose(da.cpu().numpy(), mlp.descriptor(A), atol=1e-6)
    q = synth.random_quaternions(50, 9)
    X = p.features(q, da, db).cpu().numpy()
    ref = mlp.features(q, da.cpu().numpy().astype(np.float64), db.cpu().numpy().astype(np.float64))
    # one FP64 -> FP32 rounding per input
    np.testing.assert_allclose(X, ref, rtol=1.2e-7, atol=1e-7)
    p.close()


def test_rank_is_sorted_predictions(pkg):
    p = pkg.Proposer(batch=256, seed=7)
    X, _ = _inputs(4096, 31)
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    pred = p.predict(Xt).cpu().numpy()
    idx = p.rank(Xt, 64).cpu().numpy()
    order = np.lexsort((np.arange(len(pred)), -pred))[:64]
    np.testing.assert_array_equal(idx, order)
    p.close()


def test_training_fits_a_smooth_target(pkg):
    # a smooth function of the rotation (of R(q), so equal for q and -q):
    # training must cut the loss well down
    _say("case: training on 8192 samples, 30 epochs")
    p = pkg.Proposer(batch=256, seed=13)
    q = synth.random_quaternions(8192, 41, canonical=True)
    da = mlp.descriptor(synth.mixture_balls(300, 1))
    db = mlp.descriptor(synth.mixture_balls(300, 2))
    X = mlp.features(q, da, db)
    R = np.array([mlp.rotation_matrix(v) for v in q])
    y = np.cos(3 * R[:, 0, 1]) * np.sin(2 * R[:, 1, 2]) + 0.5 * R[:, 2, 0] ** 2
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    losses = p.train(Xt, yt, 30, 1e-3)
    _say("  loss first/last epoch: %.4g / %.4g (target variance %.4g)" % (losses[0], losses[-1], y.var()))
    assert losses[-1] < 0.05 * y.var()
    # checkpoint round trip
    params = p.get_params()
    p2 = pkg.Proposer(batch=256, seed=99)
    p2.set_params(params)
    np.testing.assert_array_equal(p.predict(Xt[:500]).cpu().numpy(), p2.predict(Xt[:500]).cpu().numpy())
    p.close()
    p2.close()


def test_trained_network_beats_search_without_it(pkg):
    # The method without the network picks rotations blindly: the best of k random
    # candidates holds the exhaustive peak with probability k / candidates.  The
    # trained network's top-k must hold it far more often (small workload: 12
    # pairs on 32^3 grids, 600 evenly spread training rotations each, top 32 of
    # 1024 fresh candidates).
    n_pairs, n_train, n_cand, top = 12, 600, 1024, 32
    _say("case: proposal gain, %d pairs, n=32, top %d of %d" % (n_pairs, top, n_cand))
    pairs = synth.proposal_pairs(n_pairs, 8100, lo=300, hi=1500, n=32)
    prop = pkg.Proposer(batch=256, seed=5)
    X, y, evals = [], [], []
    for p, (A, B, g) in enumerate(pairs):
        c = pkg.Correlator(A, B, g.n, g.box, g.origin, batch=64)
        qt = synth.super_fibonacci_quaternions(n_train, 8200 + p)
        qc = synth.random_quaternions(n_cand, 8300 + p, canonical=True)
        yt = c.eval(qt, scores=False)[1].double().cpu().numpy()
        peaks = c.eval(qc, scores=False)[1].double().cpu().numpy()
        c.close()
        da, db = prop.descriptor(A), prop.descriptor(B)
        X.append(prop.features(qt, da, db))
        y.append(torch.tensor((yt - yt.mean()) / yt.std(), dtype=torch.float32, device="cuda"))
        evals.append((prop.features(qc, da, db), peaks))
    X, y = torch.cat(X), torch.cat(y)
    for ep, lr in ((100, 1e-3), (40, 3e-4), (20, 1e-4)):
        losses = prop.train(X, y, ep, lr)
    rng = np.random.default_rng(8400)
    hit_net = hit_rand = 0
    for Xc, peaks in evals:
        best = peaks.max()
        idx = prop.rank(Xc, top).cpu().numpy()
        hit_net += peaks[idx].max() >= (1 - 1e-4) * best
        hit_rand += peaks[rng.choice(n_cand, top, replace=False)].max() >= (1 - 1e-4) * best
    prop.close()
    _say("  final loss %.3g; exhaustive peak in the network's top %d: %d of %d pairs; in %d random: %d"
         % (losses[-1], top, hit_net, n_pairs, top, hit_rand))
    assert hit_net >= n_pairs // 2
    assert hit_net >= hit_rand + n_pairs // 3


@pytest.mark.parametrize("w", [0.0, -1.0])
def test_descriptor_rejects_weights_without_volume(pkg, w):
    # the descriptor is a histogram of volumes w r^3 normalised by their total:
    # a weight <= 0 is refused rather than giving an infinite scale
    p = pkg.Proposer(batch=64, seed=1)
    A = synth.mixture_balls(50, 79).copy()
    A[7, 4] = w
    with pytest.raises(pkg.CorrError) as e:
        p.descriptor(A)
    assert e.value.code == pkg.CORR_EINVAL
    assert "weight" in str(e.value)
    p.close()
