"""Pins of the 4D lifted-correlation oracle (oracle.lift_*, o1_lift_grid,
o2_lift_*) against things other than itself.

The lift (Sec. 2.2 eq. eq_rhoA, eq_L2cone, eq_coneconv; Sec. 3.1 Lemma 2,
eq. eq_ORA, eq_convgA): knot (x, r) of the fixed shape carries the downward
half-cone {(y, s) : |y - x| <= r - s}, knot (y0, rho) of the moved shape the
r-mirrored, upward cone {(y, s) : |y - y0| <= rho + s}; the moved shape is
translated by (t, h) in 4D.  The slice at height h of the lifted correlation is
the sum over pairs of the 4D volume of the two cones' intersection.
"""
import math

import numpy as np
import pytest

import oracle
import synth

mp = pytest.importorskip("mpmath")
quad = pytest.importorskip("scipy.integrate").quad


def _cones_mc(x, r, c, rho, h, n, seed):
    """Monte Carlo 4D volume of {|y - x| <= r - s} & {|y - c| <= rho + s - h}
    (explicit cone memberships, no reduction), with its standard error."""
    g = np.random.default_rng(seed)
    lo = np.minimum(x, c) - (r + rho)
    hi = np.maximum(x, c) + (r + rho)
    s_lo, s_hi = h - rho, r  # heights where both cross-sections exist
    y = lo + (hi - lo) * g.random((n, 3))
    s = s_lo + (s_hi - s_lo) * g.random(n)
    inside = (np.linalg.norm(y - x, axis=1) <= r - s) & (np.linalg.norm(y - c, axis=1) <= rho + s - h)
    box = np.prod(hi - lo) * (s_hi - s_lo)
    p = inside.mean()
    return box * p, box * math.sqrt(p * (1 - p) / n)


@pytest.mark.parametrize("d,r,rho,h", [(0.03, 0.05, 0.04, 0.0), (0.07, 0.05, 0.04, 0.0), (0.0, 0.06, 0.02, 0.0),
                                       (0.02, 0.05, 0.04, 0.03), (0.08, 0.05, 0.04, -0.02)])
def test_cone_intersection_volume_by_monte_carlo(d, r, rho, h):
    x = np.array([0.1, -0.2, 0.3])
    e = np.array([2.0, -1.0, 2.0]) / 3.0
    c = x + d * e
    v, se = _cones_mc(x, r, c, rho, h, 2_000_000, 5)
    w = oracle.lift_w(d, r + rho - h)
    assert abs(w - v) <= 4 * se + 1e-15, (w, v, se)


def test_cone_volume_is_the_height_integral_of_lens_volumes():
    # at height s the two cross-sections are balls of radii a and P - a
    for d, P in [(0.0, 0.1), (0.03, 0.1), (0.07, 0.1), (0.099, 0.1)]:
        q, _ = quad(lambda a: oracle.lens_volume(d, a, P - a), 0.0, P, epsabs=1e-16, epsrel=1e-12, limit=200,
                    points=[(P - d) / 2, (P + d) / 2])
        assert oracle.lift_w(d, P) == pytest.approx(q, rel=1e-9)
    assert oracle.lift_w(0.1, 0.1) == 0.0 and oracle.lift_w(0.2, 0.1) == 0.0
    assert oracle.lift_w(0.0, -0.01) == 0.0 and oracle.lift_w(0.0, 0.0) == 0.0


def test_cone_transform_by_quadrature_and_40_digits():
    P = 0.09
    for k in (0.0, 3.0, 21.0, 22.3, 23.0, 80.0, 150.0):
        # radial transform of W: (4 pi / k) int t W(t) sin(kt) dt
        if k == 0:
            ref = quad(lambda t: 4 * math.pi * t * t * oracle.lift_w(t, P), 0, P, epsabs=0, epsrel=1e-13)[0]
        else:
            ref = quad(lambda t: 4 * math.pi / k * t * oracle.lift_w(t, P) * math.sin(k * t), 0, P, epsabs=0,
                       epsrel=1e-13, limit=400)[0]
        assert oracle.lift_what(k, P) == pytest.approx(ref, rel=1e-9, abs=1e-12 * abs(oracle.lift_what(0, P)))
        # the convolution in radius of two ball transforms
        conv = quad(lambda u: oracle.ball_ft(k, u) * oracle.ball_ft(k, P - u), 0, P, epsabs=0, epsrel=1e-13,
                    limit=400)[0]
        assert oracle.lift_what(k, P) == pytest.approx(conv, rel=1e-9, abs=1e-12 * abs(oracle.lift_what(0, P)))
    # the k -> 0 limit (the integral of W) and the series / closed form hand-off
    assert oracle.lift_what(0.0, P) == pytest.approx(4 * math.pi ** 2 * P ** 7 / 315, rel=1e-15)
    mp.mp.dps = 40
    for x in (0.3, 1.9999, 2.0, 2.0001, 5.0):
        k = x / P
        xm = mp.mpf(x)
        exact = 4 * mp.pi ** 2 * (xm ** 3 * mp.cos(xm) - 6 * xm ** 2 * mp.sin(xm) - 15 * xm * mp.cos(xm)
                                  + 15 * mp.sin(xm)) / (3 * mp.mpf(k) ** 7)
        assert oracle.lift_what(k, P) == pytest.approx(float(exact), rel=1e-12)
    assert oracle.lift_what(10.0, -0.01) == 0.0


def test_zero_slice_positive_set_is_the_obstacle_of_the_balls():
    # Lemma 2: the r = 0 slice of the lifted correlation is positive exactly
    # where the 3D plain score is (some pair of balls overlaps)
    A, B, q, g, plain = synth.tiny_case()
    R = oracle.quat_to_rot(synth.random_quaternions(1, 91)[0])
    o, h, n = plain["origin"], plain["h"], plain["n"]
    s1 = oracle.o1_grid(A, B, R, o, h, n)
    l0 = oracle.o1_lift_grid(A, B, R, o, h, n, 0.0)
    assert (s1 > 0).sum() > 100
    assert np.array_equal(s1 > 0, l0 > 0)
    # the scores themselves differ (cone volumes, not lens volumes)
    assert not np.allclose(s1 / s1.max(), l0 / l0.max(), atol=1e-2)


@pytest.mark.parametrize("height", [0.02, -0.03])
def test_slices_at_other_heights_are_offset_obstacles(height):
    # a slice at height h is the obstacle of the primitives offset by a total
    # of -h (Sec. 3.1): the positive set of the plain score with every radius
    # of A changed by -h
    A, B, q, g, plain = synth.tiny_case()
    R = oracle.quat_to_rot(synth.random_quaternions(1, 92)[0])
    o, h, n = plain["origin"], plain["h"], plain["n"]
    lh = oracle.o1_lift_grid(A, B, R, o, h, n, height)
    s1 = oracle.o1_grid(oracle.offset_balls(A, -height), B, R, o, h, n)
    assert np.array_equal(s1 > 0, lh > 0)
    # and the split of the offset between the shapes does not matter
    s1b = oracle.o1_grid(oracle.offset_balls(A, -height / 2), oracle.offset_balls(B, -height / 2), R, o, h, n)
    assert np.array_equal(s1b > 0, lh > 0)


def test_slice_is_the_height_integral_of_offset_overlap_scores():
    # slicing the 4D correlation at height h integrates, over the common
    # heights s, the 3D overlap score of A's balls shrunk by s and B's grown
    # by s - h (balls of radius <= 0 absent): checked at translations near the
    # support, with the 3D plain score evaluated pair by pair
    A = synth.uniform_balls(6, 93)
    B = synth.uniform_balls(5, 94)
    R = oracle.quat_to_rot(synth.random_quaternions(1, 95)[0])
    height = 0.01
    g = np.random.default_rng(96)
    ia, ib = g.integers(0, 6, 4), g.integers(0, 5, 4)
    t = A[ia, :3] - B[ib, :3] @ R.T + g.normal(0, 0.02, (4, 3))

    def score_at(s, tt):
        a = A.copy()
        b = B.copy()
        a[:, 3] = A[:, 3] - s
        b[:, 3] = B[:, 3] + s - height
        a, b = a[a[:, 3] > 0], b[b[:, 3] > 0]
        if len(a) == 0 or len(b) == 0:
            return 0.0
        return float(oracle.o1_points(a, b, R, tt[None, :])[0])

    s_lo = height - B[:, 3].max()
    s_hi = A[:, 3].max()
    for tt in t:
        direct = oracle.o1_lift_grid(A, B, R, tt, 1.0, 1, height)[0, 0, 0]
        kinks = sorted(set(list(A[:, 3]) + list(height - B[:, 3])))
        integ = quad(lambda s: score_at(s, tt), s_lo, s_hi, epsabs=1e-14, epsrel=1e-9, limit=400,
                     points=[k for k in kinks if s_lo < k < s_hi])[0]
        assert direct == pytest.approx(integ, rel=1e-6, abs=1e-12)


def test_lifted_o2_dc_term_and_realness():
    A = synth.mixture_balls(40, 97)
    B = synth.mixture_balls(30, 98)
    gr = synth.grid_for(A, B, 16)
    q = synth.random_quaternions(1, 99)[0]
    for height in (0.0, -0.01):
        G = oracle.o2_lift_spectrum(A, B, oracle.quat_to_rot(q), gr.n, gr.box, height)
        P = A[:, 3][:, None] + B[:, 3][None, :] - height
        dc = np.sum(A[:, 4][:, None] * B[:, 4][None, :] * 4 * math.pi ** 2 * P ** 7 / 315)
        assert G[0, 0, 0].real == pytest.approx(dc, rel=1e-12) and abs(G[0, 0, 0].imag) < 1e-14 * dc
        s = oracle.o2_lift_scores(A, B, q, gr.n, gr.box, gr.origin, height)
        assert s.sum() * gr.h ** 3 == pytest.approx(dc, rel=1e-12)
        # Hermitian: the inverse transform is real
        m = oracle.mode_numbers(gr.n)
        neg = (-m) % gr.n
        np.testing.assert_allclose(G[np.ix_(neg, neg, neg)], np.conj(G), atol=1e-12 * abs(dc))


def test_lifted_o2_is_band_limited_projection_of_lifted_o1():
    # as for the overlap score: sample the plain slice ever finer on the
    # periodic box, keep the |m_d| < N/2 modes; the gap must fall
    A, B, q, g, _ = synth.tiny_case()
    qr = synth.random_quaternions(1, 100)[0]
    R = oracle.quat_to_rot(qr)
    height = -0.01
    s2 = oracle.o2_lift_scores(A, B, qr, g.n, g.box, g.origin, height)
    errs = []
    for qf in (2, 4, 8):
        M = qf * g.n
        sf = oracle.o1_lift_grid(A, B, R, g.origin, g.box / M, M, height)
        C = np.fft.fftn(sf) / M ** 3
        m = oracle.mode_numbers(M)
        mi = np.where(np.abs(m) < g.n // 2)[0]
        Ck = np.zeros((g.n,) * 3, complex)
        mn = m[mi] % g.n
        Ck[np.ix_(mn, mn, mn)] = C[np.ix_(mi, mi, mi)]
        sp = np.real(np.fft.ifftn(Ck)) * g.n ** 3
        errs.append(np.abs(sp - s2).max() / np.abs(s2).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4


def test_single_pair_lifted_spectrum():
    # one ball each: G(k) = c d What(|k|; r + rho - h) exp(-i k . (x - R y))
    A = np.array([[0.1, 0.05, -0.2, 0.05, 2.0]])
    B = np.array([[-0.1, 0.2, 0.05, 0.03, 0.5]])
    qr = synth.random_quaternions(1, 101)[0]
    R = oracle.quat_to_rot(qr)
    n, L, height = 8, 1.5, 0.01
    G = oracle.o2_lift_spectrum(A, B, R, n, L, height)
    m = oracle.mode_numbers(n)
    p = A[0, :3] - R @ B[0, :3]
    for iz, iy, ix in [(0, 0, 0), (1, 2, 3), (7, 5, 1), (3, 7, 6)]:
        k = 2 * math.pi * np.array([m[ix], m[iy], m[iz]]) / L
        ref = 2.0 * 0.5 * oracle.lift_what(np.linalg.norm(k), 0.05 + 0.03 - height) * np.exp(-1j * k @ p)
        assert G[iz, iy, ix] == pytest.approx(ref, rel=1e-12, abs=1e-20)
