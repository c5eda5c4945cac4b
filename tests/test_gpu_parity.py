"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Gate: for every rotation, max_n |s_gpu - s_o2| / max_n |s_o2| <= 1e-4 (the
stated relative tolerance of the FP32 path), where s_o2 is the band-limited FP64
oracle on the same grid.  The plain lens-sum oracle's gap is printed, not gated
(the band limit, not the GPU, sets it).
"""
import math
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


def _o2(A, B, quats, g):
    FA = oracle.o2_spectrum(A, np.eye(3), g.n, g.box)
    out = []
    for q in quats:
        FB = oracle.o2_spectrum(B, oracle.quat_to_rot(q), g.n, g.box)
        out.append(oracle.o2_scores_from_spectra(FA, FB, g.box, g.origin))
    return np.array(out)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _check_scores(name, s_gpu, s_ref):
    for r in range(len(s_ref)):
        e = _rel(s_gpu[r], s_ref[r])
        _say("  %s rot %d: e_rel vs FP64 = %.3g" % (name, r, e))
        assert e <= TOL, "%s rotation %d: %.3g > %g" % (name, r, e, TOL)


def test_tiny_plain_case():
    A, B, q, g, plain = synth.tiny_case()
    _say("case: tiny 64+64 balls, n=32, L=4")
    c = _corr(A, B, g)
    s, pv, pi = c.eval(q)
    torch.cuda.synchronize()
    s = s.double().cpu().numpy()
    ref = _o2(A, B, q, g)
    _check_scores("tiny", s, ref)
    lo, hi = plain["crop"]
    s1 = oracle.o1_grid(A, B, np.eye(3), plain["origin"], plain["h"], plain["n"])
    crop = s[0, lo:hi, lo:hi, lo:hi]
    _say("  tiny: gap to the plain lens sum (band limit, reported) = %.3g" % _rel(crop, s1))
    c.close()


@pytest.mark.parametrize("n", [32, 64])
def test_spectrum_stage_matches_ndft(n):
    # stages a0..a3 alone: the shape spectrum against the direct FP64 NDFT
    A = synth.mixture_balls(400, 1000 + n)
    B = synth.mixture_balls(300, 2000 + n)
    g = synth.grid_for(A, B, n)
    q = synth.random_quaternions(1, 77)[0]
    _say("case: spectrum n=%d" % n)
    c = _corr(A, B, g)
    for which, balls, R in ((0, A, np.eye(3)), (1, B, oracle.quat_to_rot(q))):
        F = c.spectrum(which, q)
        torch.cuda.synchronize()
        F = F.double().cpu().numpy()
        F = F[..., 0] + 1j * F[..., 1]
        ref = oracle.o2_spectrum(balls, R, n, g.box)[:, :, : n // 2]
        e = np.abs(F - ref).max() / np.abs(ref).max()
        _say("  spectrum which=%d: max error / max |F| = %.3g" % (which, e))
        assert e <= 2e-5
    c.close()


def test_mixture_pair_several_rotations_ragged_batches():
    A = synth.mixture_balls(600, 1001)
    B = synth.mixture_balls(450, 2001)
    g = synth.grid_for(A, B, 64)
    q = synth.random_quaternions(7, 3001)
    _say("case: 600+450 balls, n=64, 7 rotations in batches of 3")
    c = _corr(A, B, g, batch=3)
    s, pv, pi = c.eval(q)
    torch.cuda.synchronize()
    s = s.double().cpu().numpy()
    ref = _o2(A, B, q, g)
    _check_scores("mixture", s, ref)
    # peaks: exactly the max of the returned scores, lowest index on ties
    pv, pi = pv.cpu().numpy(), pi.cpu().numpy()
    flat = s.reshape(len(q), -1)
    for r in range(len(q)):
        assert pv[r] == np.float32(flat[r].max())
        assert pi[r] == int(np.argmax(flat[r]))
        # the oracle's peak value is reached at the GPU's peak index within tolerance
        rmax = ref[r].max()
        assert ref[r].reshape(-1)[pi[r]] >= rmax - TOL * np.abs(ref[r]).max()
    c.close()


@pytest.mark.parametrize("w", [6, 10, 12])
def test_other_window_widths(w):
    # every accepted Kaiser-Bessel width (8 is the default, covered above): the
    # window's own error is ~1e-5 at w = 6 and far below it from 8 on, so the
    # 1e-4 gate holds at each; w changes the staged-knot capacity, the 2w key
    # ranges and the LDS layout of the spreading pass
    A, B, q, g, _ = synth.tiny_case()
    _say("case: tiny 64+64 balls, n=32, KB width %d" % w)
    c = _corr(A, B, g, kb_width=w)
    assert c.info["kb_width"] == w
    s, _, _ = c.eval(q, peaks=False)
    torch.cuda.synchronize()
    _check_scores("tiny w=%d" % w, s.double().cpu().numpy(), _o2(A, B, q, g))
    c.close()
    # heavy tiles: more candidate knots than one staging round holds
    A = synth.mixture_balls(20000, 1200 + w)
    B = synth.mixture_balls(2000, 2200 + w)
    g = synth.grid_for(A, B, 64)
    q = synth.random_quaternions(2, 3200 + w)
    _say("case: 20000+2000 mixture balls, n=64, KB width %d, 2 rotations" % w)
    c = _corr(A, B, g, kb_width=w)
    s, pv, pi = c.eval(q)
    torch.cuda.synchronize()
    s = s.double().cpu().numpy()
    _check_scores("mixture w=%d" % w, s, _o2(A, B, q, g))
    assert np.array_equal(pv.cpu().numpy(), s.reshape(len(q), -1).max(axis=1).astype(np.float32))
    c.close()


@pytest.mark.parametrize("w", [6, 8, 12])
def test_window_widths_on_whole_plane_tiles(w):
    # at n = 16 a spreading tile spans every row of its plane, so windows wrap
    # inside the tile and the knot loop keeps each knot's cell instead of a
    # staged window origin
    A = synth.mixture_balls(300, 1300 + w)
    B = synth.mixture_balls(200, 2300 + w)
    g = synth.grid_for(A, B, 16)
    q = synth.random_quaternions(3, 3300 + w)
    _say("case: 300+200 mixture balls, n=16, KB width %d, 3 rotations" % w)
    c = _corr(A, B, g, kb_width=w)
    s, _, _ = c.eval(q, peaks=False)
    torch.cuda.synchronize()
    _check_scores("n=16 w=%d" % w, s.double().cpu().numpy(), _o2(A, B, q, g))
    c.close()


def test_window_width_4_is_rejected():
    from paper_1711_05075_amd import CorrError, CORR_EUNSUPPORTED
    A, B, q, g, _ = synth.tiny_case()
    with pytest.raises(CorrError) as e:
        _corr(A, B, g, kb_width=4)
    assert e.value.code == CORR_EUNSUPPORTED


@pytest.mark.parametrize("n", [16, 128, 256])
def test_every_grid_size(n):
    A = synth.mixture_balls(24, 1100 + n)
    B = synth.mixture_balls(20, 2100 + n)
    g = synth.grid_for(A, B, n)
    q = synth.random_quaternions(1, 3100 + n)
    _say("case: grid n=%d, 24+20 balls" % n)
    c = _corr(A, B, g)
    s, _, _ = c.eval(q, peaks=False)
    torch.cuda.synchronize()
    _check_scores("n=%d" % n, s.double().cpu().numpy(), _o2(A, B, q, g))
    c.close()


def test_equal_radii_single_component():
    g0 = np.random.default_rng(5)
    A = np.column_stack([g0.uniform(-0.3, 0.3, (80, 3)), np.full(80, 0.05), g0.uniform(0.5, 2, 80)])
    B = np.column_stack([g0.uniform(-0.3, 0.3, (60, 3)), np.full(60, 0.03), np.ones(60)])
    g = synth.grid_for(A, B, 32)
    q = synth.random_quaternions(2, 9)
    _say("case: equal radii (one expansion component each)")
    c = _corr(A, B, g)
    assert c.info["q_a"] == 1 and c.info["q_b"] == 1
    s, _, _ = c.eval(q, peaks=False)
    torch.cuda.synchronize()
    _check_scores("equal radii", s.double().cpu().numpy(), _o2(A, B, q, g))
    c.close()


def test_empty_shape_gives_zero_scores():
    A = synth.mixture_balls(50, 1)
    g = synth.Grid(n=16, box=2.0, origin=(-1, -1, -1))
    _say("case: empty B")
    c = _corr(A, np.zeros((0, 5)), g)
    s, pv, pi = c.eval(synth.random_quaternions(2, 1))
    torch.cuda.synchronize()
    assert float(s.abs().max()) == 0.0
    assert list(pi.cpu().numpy()) == [0, 0]
    c.close()


def test_zero_rotations_is_a_no_op():
    A = synth.mixture_balls(20, 1)
    g = synth.Grid(n=16, box=2.0, origin=(-1, -1, -1))
    c = _corr(A, A, g)
    s, pv, pi = c.eval(np.zeros((0, 4)))
    torch.cuda.synchronize()
    assert s.shape[0] == 0
    c.close()


def test_dc_and_swap_invariants_on_gpu_output():
    A = synth.mixture_balls(300, 1200)
    B = synth.mixture_balls(250, 2200)
    g = synth.grid_for(A, B, 64)
    I = [1.0, 0, 0, 0]
    _say("case: DC and swap invariants")
    c1, c2 = _corr(A, B, g), _corr(B, A, g)
    s1, _, _ = c1.eval([I], peaks=False)
    s2, _, _ = c2.eval([I], peaks=False)
    torch.cuda.synchronize()
    s1, s2 = s1.double().cpu().numpy()[0], s2.double().cpu().numpy()[0]
    va = np.sum(A[:, 4] * 4 * np.pi * A[:, 3] ** 3 / 3)
    vb = np.sum(B[:, 4] * 4 * np.pi * B[:, 3] ** 3 / 3)
    assert s1.sum() * g.h ** 3 == pytest.approx(va * vb, rel=1e-4)
    neg = (-np.arange(g.n)) % g.n
    assert _rel(s1, s2[np.ix_(neg, neg, neg)]) <= TOL
    c1.close()
    c2.close()


def test_single_rotation_full_size():
    # 4096 + 4096 balls, 128^3 translations: the single-rotation workload
    A, B, q, g = synth.single_rotation_case()
    _say("case: single rotation 4096+4096, n=128 (oracle takes a while)")
    c = _corr(A, B, g)
    s, pv, pi = c.eval(q)
    torch.cuda.synchronize()
    _say("  Q_A=%d Q_B=%d" % (c.info["q_a"], c.info["q_b"]))
    _check_scores("c2", s.double().cpu().numpy(), _o2(A, B, q, g))
    c.close()


def test_batched_rotations_full_size_sampled():
    # 20000 + 2000 balls, 64^3, 512 rotations in the launch configuration of the
    # batched workload; 3 sampled rotations against the oracle, every peak
    # against the returned scores.
    A, B, q, g = synth.batched_rotations_case()
    _say("case: 512 rotations of 20000+2000, n=64")
    c = _corr(A, B, g)
    s, pv, pi = c.eval(q)
    torch.cuda.synchronize()
    flat = s.reshape(len(q), -1)
    mx = flat.max(dim=1)
    assert torch.equal(mx.values, pv)
    pick = [0, 257, 511]
    ref = _o2(A, B, q[pick], g)
    _check_scores("c3", s[pick].double().cpu().numpy(), ref)
    c.close()


def test_repeated_evaluation_is_bitwise_identical():
    # spreading sums are exact fixed-point integers: no dependence on scheduling
    A = synth.mixture_balls(3000, 1300)
    B = synth.mixture_balls(2500, 2300)
    g = synth.grid_for(A, B, 64)
    q = synth.random_quaternions(3, 3300)
    _say("case: bitwise repeatability, 3000+2500 balls, n=64")
    c = _corr(A, B, g, batch=2)
    s1, p1, i1 = c.eval(q)
    c.prepare_a()
    s2, p2, i2 = c.eval(q)
    torch.cuda.synchronize()
    assert torch.equal(s1, s2) and torch.equal(p1, p2) and torch.equal(i1, i2)
    c.close()


def test_ball_order_does_not_change_scores():
    # the library keeps balls in an order of its own (by position) and the
    # spreading sums are exact integers: any input order gives the same bits.
    # Balls sharing a centre (equal position keys) keep their input order
    # among themselves, so the reversed input also reorders knots on the device.
    A = synth.mixture_balls(2000, 1400)
    B = synth.mixture_balls(1500, 2400)
    twins = B[:400].copy()
    twins[:, 3] *= 0.5
    B = np.concatenate([B, twins])
    g = synth.grid_for(A, B, 64)
    q = synth.random_quaternions(3, 3400)
    rng = np.random.default_rng(3401)
    _say("case: ball order, 2000 + 1900 balls (400 sharing a centre), n=64")
    outs = []
    for pa, pb in ((np.arange(len(A)), np.arange(len(B))), (rng.permutation(len(A)), rng.permutation(len(B))),
                   (np.arange(len(A))[::-1], np.arange(len(B))[::-1])):
        c = _corr(A[pa], B[pb], g, batch=2)
        s, p, i = c.eval(q)
        torch.cuda.synchronize()
        outs.append((s.clone(), p.clone(), i.clone()))
        c.close()
    for s, p, i in outs[1:]:
        assert torch.equal(s, outs[0][0]) and torch.equal(p, outs[0][1]) and torch.equal(i, outs[0][2])
    _check_scores("ball order", outs[0][0].cpu().numpy().astype(np.float64), _o2(A, B, q[:1], g))


def _reached_tiles(balls, R, m, box, w, ty):
    """Tiles (z row, y tile) that some knot's window reaches, counted on the host
    from the rotated centres: a knot in cell c covers cells c - w/2 + 1 .. c + w/2."""
    u = (np.asarray(balls)[:, :3] @ np.asarray(R).T) * (m / box)
    c = np.mod(np.floor(u).astype(np.int64), m)
    lo = w // 2 - 1
    hit = np.zeros((m, m // ty), dtype=bool)
    for cy, cz in zip(c[:, 1], c[:, 2]):
        zs = (cz - lo + np.arange(w)) % m
        ts = np.unique(((cy - lo + np.arange(w)) % m) // ty)
        hit[np.ix_(zs, ts)] = True
    return hit


def test_pass_info_counts_the_tiles_knots_reach():
    # the spreading pass skips tiles no window reaches; its occupancy report
    # must agree with the tiles reached, counted independently on the host
    A = synth.mixture_balls(2000, 1400)
    B = synth.mixture_balls(1500, 2400)
    g = synth.grid_for(A, B, 64)
    q = synth.random_quaternions(1, 3400)
    _say("case: pass occupancy, 2000+1500 balls, n=64")
    c = _corr(A, B, g, batch=1)
    c.eval(q, peaks=False)
    info = c.pass_info()
    m, ty = info["m"], info["tile_rows"]
    hit = _reached_tiles(B, oracle.quat_to_rot(q[0]), m, g.box, c.info["kb_width"], ty)
    _say("  live tiles %d of %d (host count %d), live rows %d" % (info["live_tiles"], info["tiles"], hit.sum(),
                                                                  info["live_rows"]))
    assert info["tiles"] == hit.size and info["knots"] == len(B) and info["rotations"] == 1
    assert info["live_tiles"] == int(hit.sum())
    assert info["live_rows"] == int(hit.any(axis=1).sum())
    c.prepare_a()
    info = c.pass_info()
    hit = _reached_tiles(A, np.eye(3), m, g.box, c.info["kb_width"], ty)
    assert info["live_tiles"] == int(hit.sum()) and info["knots"] == len(A)
    c.close()
