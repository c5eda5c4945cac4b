"""Pins of the rasterization-baseline oracle (oracle.raster_*): the uniform-grid
method of Sec. 5.2 / Sec. 6.2 (sample both unions on the translation lattice,
count the samples where they meet), against things other than itself."""
import math

import numpy as np
import pytest

import oracle
import synth


def _np_bitmaps(A, B, R, origin, h, n):
    """The sample grids written again with numpy broadcasting."""
    idx = np.arange(n)
    sgn = np.where(idx < n // 2, idx, idx - n)
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    pa = np.stack([origin[0] + h * X, origin[1] + h * Y, origin[2] + h * Z], -1)
    Zs, Ys, Xs = np.meshgrid(sgn, sgn, sgn, indexing="ij")
    pb = np.stack([h * Xs, h * Ys, h * Zs], -1)
    a = np.zeros((n, n, n), bool)
    b = np.zeros((n, n, n), bool)
    for x, y, z, r, w in A:
        d = pa - np.array([x, y, z])
        a |= (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]) <= r * r
    for x, y, z, r, w in B:
        c = R @ np.array([x, y, z])
        d = pb - c
        b |= (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]) <= r * r
    return a.astype(np.uint8), b.astype(np.uint8)


def _big_balls(n, seed):
    g = np.random.default_rng(seed)
    c = g.uniform(-0.4, 0.4, (n, 3))
    return np.column_stack([c, g.uniform(0.12, 0.25, n), np.ones(n)])


def test_counts_by_brute_force_with_rolled_grids():
    A, B = _big_balls(5, 201), _big_balls(4, 202)
    q = synth.random_quaternions(1, 203)[0]
    R = oracle.quat_to_rot(q)
    n, L = 32, 2.4
    o = (-1.2, -1.2, -1.2)
    a, b = oracle.raster_bitmaps(A, B, R, o, L / n, n)
    na, nb = _np_bitmaps(A, B, R, o, L / n, n)
    assert np.array_equal(a, na) and np.array_equal(b, nb)
    assert a.sum() > 50 and b.sum() > 50
    counts = oracle.raster_counts_grid(A, B, q, n, L, o)
    for tz, ty, tx in [(0, 0, 0), (16, 16, 16), (13, 18, 17), (15, 21, 9)]:
        ref = int(np.sum(na * np.roll(nb, (tz, ty, tx), axis=(0, 1, 2))))
        assert counts[tz, ty, tx] == ref
    # every pair of samples is counted at exactly one translation
    assert counts.sum() == int(a.sum()) * int(b.sum())


def test_single_pair_count_approaches_the_lens_volume():
    # one ball each, centres d apart at the chosen translation: h^3 times the
    # count converges to the lens volume as the grid is refined
    a_r, b_r, d, L = 0.3, 0.25, 0.25, 2.0
    A = np.array([[0.0, 0.0, 0.0, a_r, 1.0]])
    B = np.array([[0.0, 0.0, 0.0, b_r, 1.0]])
    exact = oracle.lens_volume(d, a_r, b_r)
    errs = []
    for n in (32, 64, 128):
        h = L / n
        o = (-L / 2,) * 3
        a, b = oracle.raster_bitmaps(A, B, np.eye(3), o, h, n)
        # B moved by t = o + h idx has its centre at t; want (d, 0, 0)
        idx = [int(round((d - o[0]) / h)), int(round(-o[1] / h)), int(round(-o[2] / h))]
        c = oracle.raster_counts(a, b, [idx])[0]
        errs.append(abs(c * h ** 3 - exact) / exact)
    assert errs[2] < errs[0]
    assert errs[2] < 0.02


def test_separated_shapes_count_zero_and_union_not_sum():
    # overlapping balls inside one shape are counted once (the union), unlike
    # the overlap score's sum over pairs
    A = np.array([[0.0, 0.0, 0.0, 0.3, 1.0], [0.05, 0.0, 0.0, 0.3, 1.0]])
    B = np.array([[0.0, 0.0, 0.0, 0.2, 1.0]])
    n, L = 32, 2.0
    h = L / n
    o = (-1.0,) * 3
    a, b = oracle.raster_bitmaps(A, B, np.eye(3), o, h, n)
    a1, _ = oracle.raster_bitmaps(A[:1], B, np.eye(3), o, h, n)
    assert a.max() == 1 and a.sum() < 2 * a1.sum()
    # B far away (translation index 0 puts its centre at the box corner)
    assert oracle.raster_counts(a, b, [[0, 0, 0]])[0] == 0
    # B at the origin: every sample of B lies in A
    idx = [int(round(-o[0] / h))] * 3
    assert oracle.raster_counts(a, b, [idx])[0] == int(b.sum())


def test_rotation_turns_the_moved_shape_only():
    # a quarter turn about z maps B's sample grid onto itself rotated
    B = np.array([[0.3, 0.1, -0.2, 0.15, 1.0], [-0.1, 0.25, 0.05, 0.12, 1.0]])
    A = np.array([[0.0, 0.0, 0.0, 0.2, 1.0]])
    n, L = 32, 2.0
    h = L / n
    q = [math.cos(math.pi / 4), 0.0, 0.0, math.sin(math.pi / 4)]
    _, b0 = oracle.raster_bitmaps(A, B, np.eye(3), (-1.0,) * 3, h, n)
    _, b1 = oracle.raster_bitmaps(A, B, oracle.quat_to_rot(q), (-1.0,) * 3, h, n)
    # R_z(90): (x, y) -> (-y, x); sample v of b1 holds b0 at (v_y, -v_x)
    idx = np.arange(n)
    sgn = np.where(idx < n // 2, idx, idx - n)
    src_x = (sgn[None, :] * 0 + sgn[:, None]) % n   # v_y  (rows indexed by y)
    src_y = (-sgn[None, :]) % n                     # -v_x
    for z in range(n):
        np.testing.assert_array_equal(b1[z], b0[z][src_y, src_x])
