"""Seeded input generators: the rotation sets used for training the proposal
network and for candidates."""
import numpy as np

import synth


def _min_angle(q):
    # geodesic distance between rotations: 2 acos |q_i . q_j|
    d = np.abs(q @ q.T)
    np.fill_diagonal(d, 0.0)
    return 2.0 * np.arccos(np.clip(d.max(), -1.0, 1.0))


def test_super_fibonacci_set_is_unit_canonical_and_even():
    q = synth.super_fibonacci_quaternions(1000, 6000)
    assert q.shape == (1000, 4)
    np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-14)
    assert np.all(q[:, 0] >= 0)
    # evenly spread: its closest pair is far apart, unlike a random set's
    ev, rnd = _min_angle(q), _min_angle(synth.random_quaternions(1000, 6000, canonical=True))
    assert ev > 3 * rnd, (ev, rnd)
    # packing bound: rotations at mutual angle >= D are unit quaternions at
    # sphere distance >= D / 2, so caps of radius D / 4 on S^3 (volume
    # pi (D/2 - sin(D/2)) each) are disjoint within half the sphere (pi^2):
    # n pi (x - sin x) <= pi^2 with x = D / 2.  An even set reaches a good
    # fraction of the bound.
    x = 0.3
    for _ in range(60):  # Newton on x - sin x = pi / n
        x -= (x - np.sin(x) - np.pi / 1000) / (1 - np.cos(x))
    bound = 2 * x
    assert 0.5 * bound < ev <= bound, (ev, bound)
    # the set is uniform: the mean of R(q) over the group is zero
    w, x, y, z = q.T
    r00 = 1 - 2 * (y * y + z * z)
    r12 = 2 * (y * z - w * x)
    assert abs(r00.mean()) < 0.01 and abs(r12.mean()) < 0.01
    # different seeds turn the whole set
    q2 = synth.super_fibonacci_quaternions(1000, 6001)
    assert not np.allclose(q2, q)
    np.testing.assert_allclose(_min_angle(q2), ev, rtol=1e-6)
