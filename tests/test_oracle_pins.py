"""Pins for the FP64 oracle: checks against facts the paper and the mathematics fix.

None of these re-types the oracle's own formulas.  Each is a different route to
the same number -- Monte Carlo volumes, quadrature, limits, symmetries of the
correlation (Sec. 3.1 eq. eq_relg, App. B group law, App. C transform rules),
brute force on tiny inputs -- chosen so that a dropped term, a wrong sign, a
transposed rotation or a wrong index in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth

RNG = np.random.default_rng(12345)


# --------------------------------------------------------------------------
# Lens volume (pair term of the plain method)
# --------------------------------------------------------------------------

def _mc_overlap(c1, a, c2, b, n=2_000_000, seed=0):
    """Monte Carlo volume of B(c1, a) & B(c2, b), sampled in the bounding box of B(c1, a)."""
    g = np.random.default_rng(seed)
    p = c1 + a * (2.0 * g.random((n, 3)) - 1.0)
    inside = (np.sum((p - c1) ** 2, 1) <= a * a) & (np.sum((p - c2) ** 2, 1) <= b * b)
    frac = inside.mean()
    box = (2 * a) ** 3
    return box * frac, box * math.sqrt(frac * (1 - frac) / n)


@pytest.mark.parametrize("a,b,d", [(0.05, 0.03, 0.06), (0.04, 0.04, 0.01), (0.08, 0.03, 0.07),
                                   (0.03, 0.07, 0.05), (0.05, 0.05, 0.095)])
def test_lens_volume_matches_monte_carlo(a, b, d):
    v = oracle.lens_volume(d, a, b)
    mc, sd = _mc_overlap(np.zeros(3), a, np.array([d, 0.0, 0.0]), b)
    assert abs(v - mc) < 4 * sd + 1e-12


def test_lens_volume_limits_and_symmetry():
    for a, b in [(0.05, 0.03), (0.02, 0.07), (0.04, 0.04)]:
        assert oracle.lens_volume(a + b, a, b) == 0.0
        assert oracle.lens_volume(a + b + 1e-3, a, b) == 0.0
        m = min(a, b)
        full = 4 * math.pi * m ** 3 / 3
        # continuous where the small ball touches the inside of the large one
        d0 = abs(a - b)
        if d0 > 0:
            assert abs(oracle.lens_volume(d0 + 1e-9, a, b) - full) < 1e-8 * full
            assert oracle.lens_volume(d0 * 0.5, a, b) == pytest.approx(full, rel=1e-15)
        # C1 at first contact: V ~ (a+b-d)^2 so V / (a+b-d) -> 0
        eps = 1e-6
        assert oracle.lens_volume(a + b - eps, a, b) / eps < 1e-3
        for d in np.linspace(0.0, a + b, 17):
            assert oracle.lens_volume(d, a, b) == pytest.approx(oracle.lens_volume(d, b, a), rel=1e-14)
    r = 0.05
    assert oracle.lens_volume(0.0, r, r) == pytest.approx(4 * math.pi * r ** 3 / 3, rel=1e-15)
    # equal radii: dV/dd = -pi r^2 at d = 0+
    e = 1e-7
    slope = (oracle.lens_volume(e, r, r) - oracle.lens_volume(0.0, r, r)) / e
    assert slope == pytest.approx(-math.pi * r * r, rel=1e-4)


def test_lens_volume_integrates_to_product_of_volumes():
    # int V(|t|; a, b) d^3t = vol(B_a) vol(B_b): the zero-frequency form of the
    # convolution theorem (App. C) for two indicators.
    for a, b in [(0.05, 0.03), (0.02, 0.02), (0.07, 0.01)]:
        val, _ = integrate.quad(lambda rho: 4 * math.pi * rho * rho * oracle.lens_volume(rho, a, b),
                                0.0, a + b, points=[abs(a - b)], epsabs=0, epsrel=1e-12, limit=200)
        assert val == pytest.approx((4 * math.pi / 3) ** 2 * a ** 3 * b ** 3, rel=1e-10)


# --------------------------------------------------------------------------
# Ball transform
# --------------------------------------------------------------------------

def test_ball_ft_zero_frequency_is_volume():
    for r in [0.004, 0.02, 0.1, 1.0]:
        assert oracle.ball_ft(0.0, r) == pytest.approx(4 * math.pi * r ** 3 / 3, rel=1e-15)


@pytest.mark.parametrize("k", [0.0, 1.0, 7.5, 40.0, 150.0, 600.0])
@pytest.mark.parametrize("r", [0.006, 0.03, 0.09])
def test_ball_ft_matches_radial_quadrature(k, r):
    # F{1_B}(k) = int_B exp(-i k.x) dx = 4 pi int_0^r rho^2 sin(k rho)/(k rho) d rho
    f = (lambda rho: 4 * math.pi * rho * rho * (math.sin(k * rho) / (k * rho) if k * rho > 0 else 1.0))
    val, _ = integrate.quad(f, 0.0, r, epsabs=0, epsrel=1e-13, limit=200)
    ref_scale = 4 * math.pi * r ** 3 / 3
    assert abs(oracle.ball_ft(k, r) - val) < 1e-12 * ref_scale


def test_ball_ft_series_switch_is_continuous():
    # Both sides of the switch between the small-kr series and the closed form
    # agree with a 40-digit evaluation of 4 pi (sin x - x cos x) / k^3.
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    r = 0.05
    for x in [1e-6, 1e-3, 0.2, 0.5 * (1 - 1e-12), 0.5, 0.5 * (1 + 1e-12), 0.8, 3.0]:
        k = x / r
        xm = mp.mpf(x)
        ref = 4 * mp.pi * (mp.sin(xm) - xm * mp.cos(xm)) / mp.mpf(k) ** 3
        assert abs(float((oracle.ball_ft(k, r) - ref) / ref)) < 2e-15


@pytest.mark.parametrize("a,b", [(0.05, 0.03), (0.04, 0.04), (0.07, 0.012)])
@pytest.mark.parametrize("k", [0.5, 13.0, 61.0, 140.0])
def test_ball_ft_product_is_transform_of_lens(a, b, k):
    # The lens volume is the correlation of two ball indicators, so its radial
    # transform equals Bhat(k; a) * Bhat(k; b) (convolution theorem, App. C).
    # This ties the spectral oracle's kernel to the plain oracle's closed form.
    def f(rho):
        return 4 * math.pi * rho * rho * math.sin(k * rho) / (k * rho) * oracle.lens_volume(rho, a, b)
    val, _ = integrate.quad(f, 1e-300, a + b, points=[abs(a - b)], epsabs=0, epsrel=1e-13, limit=400)
    prod = oracle.ball_ft(k, a) * oracle.ball_ft(k, b)
    scale = (4 * math.pi / 3) ** 2 * a ** 3 * b ** 3
    assert abs(val - prod) < 1e-10 * scale


# --------------------------------------------------------------------------
# Rotations (App. B)
# --------------------------------------------------------------------------

def _rodrigues(axis, angle):
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) * math.cos(angle) + math.sin(angle) * K + (1 - math.cos(angle)) * np.outer(a, a)


def _hamilton(p, q):
    w1, v1 = p[0], np.asarray(p[1:])
    w2, v2 = q[0], np.asarray(q[1:])
    return np.concatenate([[w1 * w2 - v1 @ v2], w1 * v2 + w2 * v1 + np.cross(v1, v2)])


def test_quaternion_rotation_matches_rodrigues_and_group_law():
    for _ in range(20):
        axis = RNG.standard_normal(3)
        ang = RNG.uniform(-math.pi, math.pi)
        q = np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * axis / np.linalg.norm(axis)])
        R = oracle.quat_to_rot(q)
        np.testing.assert_allclose(R, _rodrigues(axis, ang), atol=1e-14)
        np.testing.assert_allclose(oracle.quat_to_rot(-q), R, atol=1e-15)
        np.testing.assert_allclose(oracle.quat_to_rot(3.0 * q), R, atol=1e-15)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-14)
    # composition: (R1, 0)(R2, 0) = (R1 R2, 0)
    q1, q2 = synth.random_quaternions(2, 7)
    np.testing.assert_allclose(oracle.quat_to_rot(_hamilton(q1, q2)),
                               oracle.quat_to_rot(q1) @ oracle.quat_to_rot(q2), atol=1e-14)
    # a quarter turn about z takes e_x to e_y
    R = oracle.quat_to_rot([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)])
    np.testing.assert_allclose(R @ [1, 0, 0], [0, 1, 0], atol=1e-15)


# --------------------------------------------------------------------------
# Plain oracle O1
# --------------------------------------------------------------------------

def test_o1_single_pair_direction_by_monte_carlo():
    # One ball in each shape; B's centre off its frame origin so that R matters.
    # The moved ball sits at R y + t (App. B action); its overlap with A's ball
    # is estimated by sampling, with R from the axis-angle formula.
    A = np.array([[0.10, -0.05, 0.02, 0.05, 1.0]])
    B = np.array([[0.12, 0.03, -0.04, 0.035, 1.0]])
    axis, ang = np.array([0.3, -0.5, 0.8]), 1.1
    q = np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * axis / np.linalg.norm(axis)])
    R = _rodrigues(axis, ang)
    yb = R @ B[0, :3]
    for delta in [np.array([0.02, -0.01, 0.03]), np.array([-0.045, 0.02, 0.0])]:
        t = A[0, :3] - yb + delta
        s = oracle.o1_points(A, B, oracle.quat_to_rot(q), t)[0]
        mc, sd = _mc_overlap(A[0, :3], A[0, 3], yb + t, B[0, 3], seed=3)
        assert mc > 0.2 * 4 * math.pi * 0.035 ** 3 / 3  # a real overlap, not a trivial zero
        assert abs(s - mc) < 4 * sd
        # the reflected translation does not overlap at all here
        assert oracle.o1_points(A, B, oracle.quat_to_rot(q), -t)[0] == 0.0


def test_o1_union_brute_force_monte_carlo():
    # <f_A, f_(R,t)B> with f a sum of indicators (union as sum, overlaps counted
    # with multiplicity), sampled directly on tiny shapes with weights != 1.
    A = np.array([[0.0, 0.0, 0.0, 0.06, 1.0], [0.05, 0.0, 0.0, 0.04, 2.0], [0.0, 0.07, 0.0, 0.03, 0.5]])
    B = np.array([[0.01, 0.0, 0.02, 0.05, 1.5], [-0.04, 0.02, 0.0, 0.03, 1.0]])
    q = synth.random_quaternions(1, 11)[0]
    R = oracle.quat_to_rot(q)
    t = np.array([0.03, 0.02, -0.01])
    g = np.random.default_rng(5)
    n = 4_000_000
    lo, hi = np.array([-0.07] * 3), np.array([0.1] * 3)
    p = lo + (hi - lo) * g.random((n, 3))
    fA = sum(w * (np.sum((p - c) ** 2, 1) <= r * r) for *c, r, w in A)
    fB = sum(w * (np.sum((p - (R @ np.array(c) + t)) ** 2, 1) <= r * r) for *c, r, w in B)
    vals = fA * fB
    vol = np.prod(hi - lo)
    mc, sd = vol * vals.mean(), vol * vals.std() / math.sqrt(n)
    s = oracle.o1_points(A, B, R, t)[0]
    assert mc > 0
    assert abs(s - mc) < 4 * sd


def test_o1_grid_matches_point_evaluation():
    A, B, q, g, plain = synth.tiny_case()
    R = oracle.quat_to_rot(synth.random_quaternions(1, 21)[0])
    n, h, o = plain["n"], plain["h"], plain["origin"]
    grid = oracle.o1_grid(A, B, R, o, h, n)
    idx = np.argwhere(grid > 0)
    sel = idx[np.random.default_rng(0).choice(len(idx), 200, replace=False)]
    sel = np.concatenate([sel, np.random.default_rng(1).integers(0, n, (50, 3))])
    t = np.asarray(o)[None, :] + h * sel[:, ::-1]
    np.testing.assert_allclose(oracle.o1_points(A, B, R, t), grid[tuple(sel.T)], rtol=1e-12, atol=1e-18)


def test_o1_support_is_union_of_obstacle_balls():
    # Equal radii: the translational obstacle is a union of balls of radius
    # r_A + r_B at the pairwise centres x_i - R y_j (Sec. 3.1 eq. eq_ORP), and
    # the score is zero exactly outside it (collision predicate, eq. eq_pred).
    g = np.random.default_rng(9)
    A = np.column_stack([g.random((6, 3)) * 0.4, np.full(6, 0.04), np.ones(6)])
    B = np.column_stack([g.random((5, 3)) * 0.4, np.full(5, 0.03), np.ones(5)])
    R = oracle.quat_to_rot(synth.random_quaternions(1, 4)[0])
    c = A[:, None, :3] - (B[:, :3] @ R.T)[None, :, :]
    near = c.reshape(-1, 3)[g.integers(0, 30, 2000)] + g.uniform(-0.09, 0.09, (2000, 3))
    t = np.concatenate([g.uniform(-0.8, 0.8, (1000, 3)), near])
    s = oracle.o1_points(A, B, R, t)
    dist = np.linalg.norm(t[:, None, None, :] - c[None], axis=-1).min(axis=(1, 2))
    inside = dist < 0.07
    assert np.all(s[~inside] == 0.0)
    assert np.all(s[inside] > 0.0)
    assert inside.sum() > 300 and (~inside).sum() > 300


def test_o1_rotation_and_swap_identities():
    # g_AB(R, t) = g_BA(R^T, -R^T t): the relative configuration of A seen from B
    # is the inverse motion (App. B inversion).
    A = synth.uniform_balls(20, 31) * [0.3, 0.3, 0.3, 1, 1]
    B = synth.uniform_balls(15, 32) * [0.3, 0.3, 0.3, 1, 1]
    R = oracle.quat_to_rot(synth.random_quaternions(1, 33)[0])
    t = np.random.default_rng(2).uniform(-0.3, 0.3, (40, 3))
    lhs = oracle.o1_points(A, B, R, t)
    rhs = oracle.o1_points(B, A, R.T, -(t @ R))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-18)
    assert lhs.max() > 0


# --------------------------------------------------------------------------
# Band-limited oracle O2
# --------------------------------------------------------------------------

def test_o2_dc_term_is_product_of_volumes():
    A, B, q, g, _ = synth.tiny_case()
    s2 = oracle.o2_scores(A, B, synth.random_quaternions(1, 8)[0], g.n, g.box, g.origin)
    va = np.sum(A[:, 4] * 4 * np.pi * A[:, 3] ** 3 / 3)
    vb = np.sum(B[:, 4] * 4 * np.pi * B[:, 3] ** 3 / 3)
    assert s2.sum() * g.h ** 3 == pytest.approx(va * vb, rel=1e-12)


def test_o2_is_band_limited_projection_of_o1():
    # s2 = the |m_d| < N/2 Fourier projection of the L-periodic plain score.
    # Sample s1 on finer grids M = qN, transform, keep the central modes, go
    # back to the N-grid: the gap must fall as the sampling aliasing does.
    A, B, q, g, _ = synth.tiny_case()
    qr = synth.random_quaternions(1, 12)[0]
    R = oracle.quat_to_rot(qr)
    s2 = oracle.o2_scores(A, B, qr, g.n, g.box, g.origin)
    errs = []
    for qf in (2, 4, 8):
        M = qf * g.n
        sf = oracle.o1_grid(A, B, R, g.origin, g.box / M, M)
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


def test_o2_spectrum_hermitian_and_nyquist_zero():
    A = synth.mixture_balls(50, 77)
    F = oracle.o2_spectrum(A, oracle.quat_to_rot(synth.random_quaternions(1, 3)[0]), 16, 2.5)
    m = oracle.mode_numbers(16)
    neg = (-m) % 16
    np.testing.assert_allclose(F[np.ix_(neg, neg, neg)], np.conj(F), atol=1e-13 * np.abs(F).max())
    assert np.all(F[8] == 0) and np.all(F[:, 8] == 0) and np.all(F[:, :, 8] == 0)


def test_o2_matches_direct_sum_at_grid_points():
    # The FFT step of the oracle equals the plain sum over kept modes.
    A = synth.uniform_balls(10, 41) * [0.5, 0.5, 0.5, 1, 1]
    B = synth.uniform_balls(9, 42) * [0.5, 0.5, 0.5, 1, 1]
    q = synth.random_quaternions(1, 43)[0]
    n, L, o = 8, 2.0, (-1.0, -0.75, -1.25)
    FA = oracle.o2_spectrum(A, np.eye(3), n, L)
    FB = oracle.o2_spectrum(B, oracle.quat_to_rot(q), n, L)
    s = oracle.o2_scores_from_spectra(FA, FB, L, o)
    idx = np.array([[0, 0, 0], [3, 1, 7], [5, 6, 2], [7, 7, 7]])
    t = np.asarray(o)[None, :] + (L / n) * idx
    np.testing.assert_allclose(s[idx[:, 2], idx[:, 1], idx[:, 0]], oracle.o2_eval_at(FA, FB, L, t),
                               rtol=1e-10, atol=1e-14 * np.abs(s).max())


def test_o2_spectrum_single_knot_is_shifted_ball_transform():
    # One knot at x: F(k) = c Bhat(|k|; r) exp(-i k.x) (shift rule, App. C).
    x = np.array([0.13, -0.27, 0.31])
    ball = np.array([[*x, 0.05, 2.0]])
    n, L = 8, 1.7
    F = oracle.o2_spectrum(ball, np.eye(3), n, L)
    m = oracle.mode_numbers(n)
    for iz, iy, ix in [(1, 2, 3), (7, 0, 5), (0, 0, 0), (3, 3, 3)]:
        k = 2 * np.pi / L * np.array([m[ix], m[iy], m[iz]])
        want = 2.0 * oracle.ball_ft(np.linalg.norm(k), 0.05) * np.exp(-1j * (k @ x))
        assert F[iz, iy, ix] == pytest.approx(want, rel=1e-12, abs=1e-18)


def test_o2_swap_identity_on_grid():
    A = synth.mixture_balls(40, 51)
    B = synth.mixture_balls(30, 52)
    g = synth.grid_for(A, B, 16)
    I = [1.0, 0, 0, 0]
    sab = oracle.o2_scores(A, B, I, g.n, g.box, g.origin)
    sba = oracle.o2_scores(B, A, I, g.n, g.box, g.origin)
    # t_n = -L/2 + h n, so -t_n sits at index (N - n) mod N
    neg = (-np.arange(g.n)) % g.n
    np.testing.assert_allclose(sab, sba[np.ix_(neg, neg, neg)], atol=1e-12 * np.abs(sab).max())


def test_o2_rotation_identity_off_grid():
    # g_AB(R, t) = g_BA(R^T, -R^T t) (App. B inversion).  For the band-limited
    # score it holds exactly when R maps the cube of kept modes onto itself,
    # i.e. for the 24 rotations of the cube; a general rotation is covered by
    # the plain-score version of this test.
    A = synth.mixture_balls(30, 61)
    B = synth.mixture_balls(25, 62)
    L, n = 2.5, 16
    t = np.random.default_rng(4).uniform(-0.4, 0.4, (6, 3))
    s = math.sqrt(0.5)
    for q in ([1.0, 0, 0, 0], [s, 0, 0, s], [0.5, 0.5, 0.5, 0.5], [0, s, s, 0]):
        R = oracle.quat_to_rot(q)
        FA, FB = oracle.o2_spectrum(A, np.eye(3), n, L), oracle.o2_spectrum(B, R, n, L)
        GA, GB = oracle.o2_spectrum(B, np.eye(3), n, L), oracle.o2_spectrum(A, R.T, n, L)
        lhs = oracle.o2_eval_at(FA, FB, L, t)
        rhs = oracle.o2_eval_at(GA, GB, L, -(t @ R))
        np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-12 * np.abs(lhs).max())
        assert np.abs(lhs).max() > 0


def test_o2_grid_shift_of_a_is_cyclic_shift_of_scores():
    # Moving A by one grid step h along x moves the score by one index along x:
    # g(t) = <f_A, f_B(. - t)> so shifting A by +h e_x gives g(t - h e_x).
    A = synth.mixture_balls(30, 71)
    B = synth.mixture_balls(20, 72)
    g = synth.grid_for(A, B, 16)
    q = synth.random_quaternions(1, 73)[0]
    s = oracle.o2_scores(A, B, q, g.n, g.box, g.origin)
    A2 = A.copy()
    A2[:, 0] += g.h
    s2 = oracle.o2_scores(A2, B, q, g.n, g.box, g.origin)
    np.testing.assert_allclose(s2, np.roll(s, 1, axis=2), atol=1e-12 * np.abs(s).max())


def test_o2_approaches_o1_as_band_grows():
    # Balls much wider than the grid step: the band-limit gap must shrink as N grows.
    A = np.array([[0.0, 0.0, 0.0, 0.3, 1.0], [0.25, 0.1, 0.0, 0.25, 1.0]])
    B = np.array([[0.05, -0.1, 0.1, 0.28, 1.0]])
    L = 3.0
    q = [1.0, 0, 0, 0]
    errs = []
    for n in (16, 32, 64):
        o = (-L / 2,) * 3
        s2 = oracle.o2_scores(A, B, q, n, L, o)
        s1 = oracle.o1_grid(A, B, np.eye(3), o, L / n, n)
        errs.append(np.sqrt(np.sum((s2 - s1) ** 2) / np.sum(s1 ** 2)))
    # relative L2 gap; the max-norm gap is not monotone near the kinks of V
    assert errs[0] > 3 * errs[1] > 9 * errs[2]
    assert errs[2] < 1e-3


def test_peak_ties_take_lowest_index():
    s = np.zeros((2, 2, 2, 2))
    s[0, 1, 0, 1] = 3.0
    s[0, 1, 1, 0] = 3.0
    s[1, 0, 0, 0] = -1.0
    s[1, 1, 1, 1] = -0.5
    v, i = oracle.peak(s)
    assert list(v) == [3.0, 0.0] and list(i) == [5, 1]


# --------------------------------------------------------------------------
# Shape-complementarity score (Sec. 4.2, eq. eq_score)
# --------------------------------------------------------------------------

def test_sc_single_pair_by_monte_carlo():
    # G(t) = integral of a_A(x) a_B(x - t) with a = 1[ball grown by r0] - lam 1[ball]:
    # sampled directly from the two signed indicators, not from lens volumes
    A = np.array([[0.0, 0.0, 0.0, 0.05, 1.0]])
    B = np.array([[0.0, 0.0, 0.0, 0.035, 1.0]])
    r0, lam = 0.015, 3.0
    g = np.random.default_rng(17)
    n = 4_000_000
    for t in (np.array([0.02, 0.01, -0.01]), np.array([0.075, 0.0, 0.02])):
        lo, hi = np.full(3, -0.07), np.full(3, 0.07)
        p = lo + (hi - lo) * g.random((n, 3))
        dA = np.sum(p ** 2, 1)
        dB = np.sum((p - t) ** 2, 1)
        aA = (dA <= (0.05 + r0) ** 2) - lam * (dA <= 0.05 ** 2)
        aB = (dB <= (0.035 + r0) ** 2) - lam * (dB <= 0.035 ** 2)
        vals = aA * aB
        vol = np.prod(hi - lo)
        mc, sd = vol * vals.mean(), vol * vals.std() / math.sqrt(n)
        origin = t - np.array([0.0, 0.0, 0.0])
        G = oracle.o1_sc_grid(A, B, np.eye(3), origin, 1.0, 1, r0, lam)[0, 0, 0]
        assert abs(G - mc) < 4 * sd
        assert abs(G) > 10 * sd


def test_sc_four_terms_equal_the_signed_union():
    # the four-term expansion against the plain score of the signed unions
    A = synth.uniform_balls(12, 51) * [0.3, 0.3, 0.3, 0.5, 1]
    B = synth.uniform_balls(9, 52) * [0.3, 0.3, 0.3, 0.5, 1]
    R = oracle.quat_to_rot(synth.random_quaternions(1, 53)[0])
    r0, lam = 0.012, 2.5
    G = oracle.o1_sc_grid(A, B, R, (-0.4, -0.4, -0.4), 0.05, 16, r0, lam)
    Gs = oracle.o1_grid(oracle.sc_affinity_balls(A, r0, lam), oracle.sc_affinity_balls(B, r0, lam), R,
                        (-0.4, -0.4, -0.4), 0.05, 16)
    np.testing.assert_allclose(G, Gs, rtol=1e-10, atol=1e-15)
    assert G.min() < 0 < G.max()


def test_sc_cross_terms_are_two_functions():
    # Sec. 4.2 writes the expanded score with one cross term taken twice
    # (-2 lam). With S (+) B0 read as every ball grown by r0, the cross terms
    # are g(A+, B) and g(A, B+): equal for one ball each of equal radius, but
    # not in general. Concentric balls, closed form: the overlap is the smaller ball.
    a, b, r0, lam = 0.1, 0.2, 0.02, 2.0
    A = np.array([[0.0, 0.0, 0.0, a, 1.0]])
    B = np.array([[0.0, 0.0, 0.0, b, 1.0]])
    t0 = np.zeros((1, 3))
    gA = oracle.o1_points(oracle.sc_grown(A, r0), B, np.eye(3), t0)[0]
    gB = oracle.o1_points(A, oracle.sc_grown(B, r0), np.eye(3), t0)[0]
    vol = lambda r: 4.0 * np.pi / 3.0 * r ** 3
    assert gA == pytest.approx(vol(a + r0), rel=1e-12)
    assert gB == pytest.approx(vol(a), rel=1e-12)
    G = oracle.o1_sc_grid(A, B, np.eye(3), (0.0, 0.0, 0.0), 1.0, 1, r0, lam)[0, 0, 0]
    # the four-term score at t = 0 by hand: V(a+r0, b+r0) = vol(a+r0), ...
    assert G == pytest.approx(vol(a + r0) - lam * vol(a + r0) - lam * vol(a) + lam * lam * vol(a), rel=1e-12)
    merged = vol(a + r0) - 2 * lam * gA + lam * lam * vol(a)
    assert abs(merged - G) > 0.5 * abs(G)
    # one ball each of equal radius: the two cross terms agree by symmetry
    t = np.array([[0.05, 0.0, 0.0], [0.13, 0.04, -0.02]])
    Ae = np.array([[0.0, 0.0, 0.0, 0.1, 1.0]])
    e1 = oracle.o1_points(oracle.sc_grown(Ae, r0), Ae, np.eye(3), t)
    e2 = oracle.o1_points(Ae, oracle.sc_grown(Ae, r0), np.eye(3), t)
    np.testing.assert_allclose(e1, e2, rtol=1e-12)
    # a mixture pair at n = 16: the cross terms differ by 0.41 of their peak
    Am, Bm = synth.mixture_balls(60, 4200), synth.mixture_balls(45, 4300)
    g = synth.grid_for(Am, Bm, 16, pad=0.04)
    R = oracle.quat_to_rot(synth.random_quaternions(1, 4400)[0])
    cA = oracle.o1_grid(oracle.sc_grown(Am, r0), Bm, R, g.origin, g.h, g.n)
    cB = oracle.o1_grid(Am, oracle.sc_grown(Bm, r0), R, g.origin, g.h, g.n)
    assert np.abs(cA - cB).max() > 0.05 * cA.max()


def test_sc_zero_offset_is_scaled_plain_score():
    # r0 -> 0: a_S = (1 - lam) f_S, so G = (1 - lam)^2 g (O1 and O2)
    A, B, q, g, plain = synth.tiny_case()
    lam = 1.7
    R = oracle.quat_to_rot(q[0])
    lo = plain["origin"]
    G1 = oracle.o1_sc_grid(A, B, R, lo, plain["h"], 8, 0.0, lam)
    s1 = oracle.o1_grid(A, B, R, lo, plain["h"], 8)
    np.testing.assert_allclose(G1, (1 - lam) ** 2 * s1, rtol=1e-12, atol=1e-18)
    G2 = oracle.o2_sc_scores(A, B, q[0], g.n, g.box, g.origin, 0.0, lam)
    s2 = oracle.o2_scores(A, B, q[0], g.n, g.box, g.origin)
    np.testing.assert_allclose(G2, (1 - lam) ** 2 * s2, rtol=1e-9, atol=1e-12 * np.abs(s2).max())


def test_sc_dc_term_is_product_of_affinity_integrals():
    # sum_n G h^3 = (integral a_A)(integral a_B), integral a_S = sum c 4 pi/3 ((r + r0)^3 - lam r^3)
    A, B, q, g, _ = synth.tiny_case()
    r0, lam = 0.02, 2.0
    G2 = oracle.o2_sc_scores(A, B, synth.random_quaternions(1, 8)[0], g.n, g.box, g.origin, r0, lam)
    ia = np.sum(A[:, 4] * 4 * np.pi / 3 * ((A[:, 3] + r0) ** 3 - lam * A[:, 3] ** 3))
    ib = np.sum(B[:, 4] * 4 * np.pi / 3 * ((B[:, 3] + r0) ** 3 - lam * B[:, 3] ** 3))
    assert G2.sum() * g.h ** 3 == pytest.approx(ia * ib, rel=1e-11)


def test_sc_o2_is_band_limited_projection_of_o1():
    # as for the plain score: the band-limited SC score is the |m_d| < N/2
    # projection of the periodic plain SC score, approached by finer sampling
    # (the gap falls at the plain score's rate; with lam = 1 the cancellation
    # between the terms is mild enough that 8x sampling reaches 1e-4)
    A, B, q, g, _ = synth.tiny_case()
    qr = synth.random_quaternions(1, 14)[0]
    R = oracle.quat_to_rot(qr)
    r0, lam = 0.015, 1.0
    s2 = oracle.o2_sc_scores(A, B, qr, g.n, g.box, g.origin, r0, lam)
    errs = []
    for qf in (2, 4, 8):
        M = qf * g.n
        sf = oracle.o1_sc_grid(A, B, R, g.origin, g.box / M, M, r0, lam)
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


# --------------------------------------------------------------------------
# Single-configuration query (Sec. 4.1, eq. eq_single)
# --------------------------------------------------------------------------

def test_query_with_every_mode_is_the_band_limited_score_on_the_grid():
    A, B, q, g, _ = synth.tiny_case()
    qr = synth.random_quaternions(1, 61)[0]
    FA = oracle.o2_spectrum(A, np.eye(3), g.n, g.box)
    FB = oracle.o2_spectrum(B, oracle.quat_to_rot(qr), g.n, g.box)
    s2 = oracle.o2_scores_from_spectra(FA, FB, g.box, g.origin)
    idx = np.random.default_rng(7).integers(0, g.n, (20, 3))
    t = np.asarray(g.origin)[None, :] + g.h * idx[:, ::-1]
    full = 3 * (g.n // 2) ** 2
    np.testing.assert_allclose(oracle.o2_query(FA, FB, g.box, t, full), s2[tuple(idx.T)], rtol=1e-9,
                               atol=1e-12 * np.abs(s2).max())


def test_query_with_only_the_dc_mode_is_the_mean_score():
    # |m|^2 <= 0 keeps the DC mode: V_A V_B / L^3 at every translation
    A, B, q, g, _ = synth.tiny_case()
    FA = oracle.o2_spectrum(A, np.eye(3), g.n, g.box)
    FB = oracle.o2_spectrum(B, np.eye(3), g.n, g.box)
    va = np.sum(A[:, 4] * 4 * np.pi * A[:, 3] ** 3 / 3)
    vb = np.sum(B[:, 4] * 4 * np.pi * B[:, 3] ** 3 / 3)
    t = np.random.default_rng(3).uniform(-1, 1, (5, 3))
    np.testing.assert_allclose(oracle.o2_query(FA, FB, g.box, t, 0), va * vb / g.box ** 3, rtol=1e-12)
    assert oracle.query_mode_count(g.n, 0) == 1
    assert oracle.query_mode_count(g.n, 1) == 7
    assert oracle.query_mode_count(g.n, 3 * (g.n // 2) ** 2) == (g.n - 1) ** 3


def test_query_approaches_the_plain_score_as_modes_are_added():
    # away from the grid, the truncated Parseval sum tends to the band-limited
    # score, whose gap to the plain lens sum (O1) is the band limit's
    A, B, q, g, _ = synth.tiny_case()
    qr = synth.random_quaternions(1, 62)[0]
    R = oracle.quat_to_rot(qr)
    FA = oracle.o2_spectrum(A, np.eye(3), g.n, g.box)
    FB = oracle.o2_spectrum(B, R, g.n, g.box)
    t = np.random.default_rng(11).uniform(-0.3, 0.3, (40, 3))
    s1 = oracle.o1_points(A, B, R, t)
    # (the tiny case's balls are smaller than a grid step, so the full band
    # still differs from O1 by ~27 %; the decrease is not monotone shell by shell)
    errs = [np.abs(oracle.o2_query(FA, FB, g.box, t, r2) - s1).max() / np.abs(s1).max()
            for r2 in (1, 9, 100, 3 * (g.n // 2) ** 2)]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 0.3


# --------------------------------------------------------------------------
# Configuration obstacle and offset obstacles (Sec. 3.1 eq. eq_obs, offset slices)
# --------------------------------------------------------------------------

def _gap(A, B, R, t):
    """min over pairs of |x_i - R y_j - t| - r_i - rho_j, written out directly."""
    c = A[:, None, :3] - (B[:, :3] @ R.T)[None, :, :]                       # [i][j][3]
    rs = A[:, None, 3] + B[None, :, 3]
    d = np.linalg.norm(t[:, None, None, :] - c[None], axis=-1) - rs[None]
    return d.reshape(len(t), -1).min(axis=1)


def _obstacle_probe_points(A, B, R, g, n_uniform=800, n_near=1600, spread=0.1):
    c = (A[:, None, :3] - (B[:, :3] @ R.T)[None, :, :]).reshape(-1, 3)
    near = c[g.integers(0, len(c), n_near)] + g.uniform(-spread, spread, (n_near, 3))
    return np.concatenate([g.uniform(-0.8, 0.8, (n_uniform, 3)), near])


def test_obstacle_of_the_plain_score_is_the_pairwise_minkowski_union():
    # unequal radii: the plain score is > 0 exactly on the union of the balls of
    # radius r_i + rho_j about x_i - R y_j (eq. eq_obs, eq. eq_ORA pair by pair)
    g = np.random.default_rng(71)
    A = np.column_stack([g.random((7, 3)) * 0.4, g.uniform(0.02, 0.07, 7), np.ones(7)])
    B = np.column_stack([g.random((6, 3)) * 0.4, g.uniform(0.01, 0.05, 6), np.ones(6)])
    R = oracle.quat_to_rot(synth.random_quaternions(1, 72)[0])
    t = _obstacle_probe_points(A, B, R, g)
    inside = _gap(A, B, R, t) < 0
    assert inside.sum() > 300 and (~inside).sum() > 300
    assert np.array_equal(oracle.o1_obstacle_points(A, B, R, t), inside)
    assert np.array_equal(oracle.obstacle(oracle.o1_points(A, B, R, t)), inside)


@pytest.mark.parametrize("delta", [0.015, -0.008])
def test_offset_obstacle_depends_only_on_the_total_offset(delta):
    # the slice at offset delta is the obstacle of the primitives offset by a
    # total of delta, however the offset is split between the two shapes
    g = np.random.default_rng(73)
    A = np.column_stack([g.random((6, 3)) * 0.4, g.uniform(0.02, 0.06, 6), np.ones(6)])
    B = np.column_stack([g.random((5, 3)) * 0.4, g.uniform(0.015, 0.04, 5), np.ones(5)])
    R = oracle.quat_to_rot(synth.random_quaternions(1, 74)[0])
    t = _obstacle_probe_points(A, B, R, g)
    want = _gap(A, B, R, t) < delta
    assert want.sum() > 300 and (~want).sum() > 300
    on_a = oracle.obstacle(oracle.o1_points(oracle.offset_balls(A, delta), B, R, t))
    split = oracle.obstacle(oracle.o1_points(oracle.offset_balls(A, delta / 2),
                                             oracle.offset_balls(B, delta / 2), R, t))
    assert np.array_equal(on_a, want)
    assert np.array_equal(split, want)
    # the score values of the two splits differ: only the obstacle is shared
    assert not np.allclose(oracle.o1_points(oracle.offset_balls(A, delta), B, R, t),
                           oracle.o1_points(oracle.offset_balls(A, delta / 2),
                                            oracle.offset_balls(B, delta / 2), R, t))


def test_offset_slice_dc_term_is_the_offset_volumes():
    # sum_n s h^3 = (sum_i 4 pi (r_i + delta)^3 / 3) (sum_j 4 pi rho_j^3 / 3):
    # the offset is on A's balls only
    A, B, q, g, _ = synth.tiny_case()
    h = g.box / g.n
    for delta in (0.01, -0.01):
        s = oracle.o2_offset_scores(A, B, q, g.n, g.box, g.origin, delta)
        va = np.sum(A[:, 4] * 4 * np.pi * (A[:, 3] + delta) ** 3 / 3)
        vb = np.sum(B[:, 4] * 4 * np.pi * B[:, 3] ** 3 / 3)
        assert abs(s.sum() * h ** 3 - va * vb) <= 1e-12 * va * vb


def test_offset_balls_keeps_radii_positive():
    A = np.array([[0, 0, 0, 0.25, 1.0], [0.1, 0, 0, 0.5, 2.0]])
    assert np.array_equal(oracle.offset_balls(A, 0.125)[:, 3], [0.375, 0.625])
    assert np.array_equal(oracle.offset_balls(A, 0.125)[:, [0, 1, 2, 4]], A[:, [0, 1, 2, 4]])
    with pytest.raises(ValueError):
        oracle.offset_balls(A, -0.25)
