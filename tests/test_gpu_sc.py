"""GPU parity of the shape-complementarity score (Sec. 4.2, eq. eq_score).

With CORR_SC_SCORE the pipeline scores <a_A, a_(R,t)B>, a_S = f_{S (+) B0} -
lambda f_S, by expanding the per-ball kernel Bhat(k; r + r0) - lambda Bhat(k; r)
on the radius basis.  The reference is the FP64 band-limited SC oracle
(affinity spectra by direct NDFT).  Gate: max |G_gpu - G_o2| / max |G_o2| <= 1e-4
per rotation.
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


def _o2_sc(A, B, quats, g, r0, lam):
    FA = oracle.o2_sc_spectrum(A, np.eye(3), g.n, g.box, r0, lam)
    out = []
    for q in quats:
        FB = oracle.o2_sc_spectrum(B, oracle.quat_to_rot(q), g.n, g.box, r0, lam)
        out.append(oracle.o2_scores_from_spectra(FA, FB, g.box, g.origin))
    return np.array(out)


def _check(name, s_gpu, ref):
    for r in range(len(ref)):
        e = np.abs(s_gpu[r] - ref[r]).max() / np.abs(ref[r]).max()
        _say("  %s rot %d: e_rel vs FP64 = %.3g (min %.3g, max %.3g)" % (name, r, e, ref[r].min(), ref[r].max()))
        assert e <= TOL, "%s rotation %d: %.3g > %g" % (name, r, e, TOL)


def test_sc_spectrum_stage_matches_ndft():
    A = synth.mixture_balls(400, 1500)
    B = synth.mixture_balls(300, 2500)
    g = synth.grid_for(A, B, 64)
    r0, lam = 0.01, 2.0
    q = synth.random_quaternions(1, 3500)[0]
    _say("case: SC spectrum, n=64, r0=%g lambda=%g" % (r0, lam))
    c = _corr(A, B, g, sc=(r0, lam))
    _say("  q_a=%d q_b=%d" % (c.info["q_a"], c.info["q_b"]))
    for which, balls, R in ((0, A, np.eye(3)), (1, B, oracle.quat_to_rot(q))):
        F = c.spectrum(which, q)
        torch.cuda.synchronize()
        F = F.double().cpu().numpy()
        F = F[..., 0] + 1j * F[..., 1]
        ref = oracle.o2_sc_spectrum(balls, R, g.n, g.box, r0, lam)[:, :, : g.n // 2]
        e = np.abs(F - ref).max() / np.abs(ref).max()
        _say("  which=%d: max error / max |F| = %.3g" % (which, e))
        assert e <= 2e-5
    c.close()


@pytest.mark.parametrize("r0,lam", [(0.01, 2.0), (0.02, 0.5)])
def test_sc_mixture_pair_rotations(r0, lam):
    A = synth.mixture_balls(600, 1501)
    B = synth.mixture_balls(450, 2501)
    g = synth.grid_for(A, B, 64, pad=2 * r0)
    q = synth.random_quaternions(3, 3501)
    _say("case: SC scores 600+450 balls, n=64, r0=%g lambda=%g" % (r0, lam))
    c = _corr(A, B, g, sc=(r0, lam), batch=2)
    s, pv, pi = c.eval(q)
    torch.cuda.synchronize()
    s = s.double().cpu().numpy()
    _check("sc", s, _o2_sc(A, B, q, g, r0, lam))
    flat = s.reshape(len(q), -1)
    assert np.array_equal(pv.cpu().numpy(), flat.max(axis=1).astype(np.float32))
    assert np.array_equal(pi.cpu().numpy(), flat.argmax(axis=1))
    c.close()


def test_sc_equal_radii():
    g0 = np.random.default_rng(15)
    A = np.column_stack([g0.uniform(-0.3, 0.3, (80, 3)), np.full(80, 0.05), np.ones(80)])
    B = np.column_stack([g0.uniform(-0.3, 0.3, (60, 3)), np.full(60, 0.03), np.ones(60)])
    g = synth.grid_for(A, B, 32, pad=0.04)
    q = synth.random_quaternions(2, 19)
    _say("case: SC with equal radii (one radius node per shape)")
    c = _corr(A, B, g, sc=(0.02, 3.0))
    s, _, _ = c.eval(q, peaks=False)
    torch.cuda.synchronize()
    _check("sc equal radii", s.double().cpu().numpy(), _o2_sc(A, B, q, g, 0.02, 3.0))
    c.close()


def test_sc_with_zero_offset_and_penalty_is_the_overlap_score():
    # r0 = lambda = 0 expands the ball transform itself: the same tables, so the
    # same scores bit for bit
    A = synth.mixture_balls(300, 1502)
    B = synth.mixture_balls(250, 2502)
    g = synth.grid_for(A, B, 32)
    q = synth.random_quaternions(2, 3502)
    c1, c2 = _corr(A, B, g), _corr(A, B, g, sc=(0.0, 0.0))
    s1, _, _ = c1.eval(q, peaks=False)
    s2, _, _ = c2.eval(q, peaks=False)
    torch.cuda.synchronize()
    assert torch.equal(s1, s2)
    c1.close()
    c2.close()


def test_sc_single_rotation_full_size():
    # the single-rotation workload (4096 + 4096 balls, 128^3) scored for complementarity
    A, B, q, g0 = synth.single_rotation_case()
    r0, lam = 0.01, 2.0
    g = synth.grid_for(A, B, g0.n, pad=2 * r0)
    _say("case: SC single rotation 4096+4096, n=128 (oracle takes a while)")
    c = _corr(A, B, g, sc=(r0, lam))
    s, _, _ = c.eval(q)
    torch.cuda.synchronize()
    _say("  q_a=%d q_b=%d" % (c.info["q_a"], c.info["q_b"]))
    _check("sc c2", s.double().cpu().numpy(), _o2_sc(A, B, q, g, r0, lam))
    c.close()
