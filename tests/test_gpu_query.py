"""GPU parity of the single-configuration query (Sec. 4.1, eq. eq_single).

corr_query sums F_A conj(F_RB) exp(i k.t) / L^3 over the modes |m|^2 <= r2 at
arbitrary translations.  Reference: the same truncated sum of the FP64 oracle
spectra.  Gate: max |s_gpu - s_ref| / max |full-band score| <= 1e-4.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_05075_amd as pkg
    pkg.load_library()


def _corr(A, B, g, **kw):
    from paper_1711_05075_amd import Correlator
    return Correlator(A, B, g.n, g.box, g.origin, **kw)


def _pair(n=64):
    A = synth.mixture_balls(600, 1600)
    B = synth.mixture_balls(450, 2600)
    return A, B, synth.grid_for(A, B, n)


def test_query_matches_the_truncated_oracle_sum():
    A, B, g = _pair()
    q = synth.random_quaternions(1, 3600)[0]
    FA = oracle.o2_spectrum(A, np.eye(3), g.n, g.box)
    FB = oracle.o2_spectrum(B, oracle.quat_to_rot(q), g.n, g.box)
    t = np.random.default_rng(5).uniform(-0.4, 0.4, (40, 3))
    full = 3 * (g.n // 2 - 1) ** 2
    scale = np.abs(oracle.o2_query(FA, FB, g.box, t, full)).max()
    c = _corr(A, B, g)
    for r2 in (0, 4, 64, 400, full):
        s, nm = c.query(q, t, r2)
        torch.cuda.synchronize()
        ref = oracle.o2_query(FA, FB, g.box, t, r2)
        e = np.abs(s.double().cpu().numpy() - ref).max() / scale
        _say("  r2=%d modes=%d: max error / max |s| = %.3g" % (r2, nm, e))
        assert nm == oracle.query_mode_count(g.n, r2)
        assert e <= TOL
    c.close()


def test_full_band_query_equals_eval_on_grid_points():
    A, B, g = _pair(32)
    q = synth.random_quaternions(1, 3601)
    c = _corr(A, B, g)
    s, _, _ = c.eval(q, peaks=False)
    idx = np.random.default_rng(9).integers(0, g.n, (50, 3))
    t = np.asarray(g.origin)[None, :] + g.h * idx[:, ::-1]
    sq, _ = c.query(q[0], t, 10 ** 6)
    torch.cuda.synchronize()
    grid = s[0].double().cpu().numpy()[tuple(idx.T)]
    e = np.abs(sq.double().cpu().numpy() - grid).max() / s.abs().max().item()
    _say("  query vs eval at grid points: %.3g" % e)
    assert e <= TOL
    c.close()


def test_query_of_the_complementarity_score():
    A, B, g0 = _pair(32)
    r0, lam = 0.01, 2.0
    g = synth.grid_for(A, B, 32, pad=2 * r0)
    q = synth.random_quaternions(1, 3602)[0]
    FA = oracle.o2_sc_spectrum(A, np.eye(3), g.n, g.box, r0, lam)
    FB = oracle.o2_sc_spectrum(B, oracle.quat_to_rot(q), g.n, g.box, r0, lam)
    t = np.random.default_rng(6).uniform(-0.3, 0.3, (20, 3))
    c = _corr(A, B, g, sc=(r0, lam))
    s, _ = c.query(q, t, 200)
    torch.cuda.synchronize()
    ref = oracle.o2_query(FA, FB, g.box, t, 200)
    scale = np.abs(oracle.o2_query(FA, FB, g.box, t, 10 ** 6)).max()
    e = np.abs(s.double().cpu().numpy() - ref).max() / scale
    _say("  SC query: %.3g" % e)
    assert e <= TOL
    c.close()


def test_query_with_an_empty_shape_and_no_translations():
    A = synth.mixture_balls(50, 1)
    g = synth.Grid(n=16, box=2.0, origin=(-1, -1, -1))
    c = _corr(A, np.zeros((0, 5)), g)
    s, nm = c.query([1.0, 0, 0, 0], np.zeros((3, 3)), 20)
    torch.cuda.synchronize()
    assert float(s.abs().max()) == 0.0 and nm == oracle.query_mode_count(16, 20)
    s, nm = c.query([1.0, 0, 0, 0], np.zeros((0, 3)), 20)
    assert s.shape[0] == 0
    c.close()
