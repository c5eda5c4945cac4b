"""Pins for the FP64 reference of the proposal network: central finite
differences for the gradients, a hand-solvable case for Adam, bfloat16 rounding
against exactly representable values, and descriptor invariants."""
import numpy as np
import pytest

from oracle import mlp


def test_bf16_rounding_exact_cases():
    # values with at most 8 significant bits are kept; ties go to even
    exact = np.array([1.0, -2.5, 0.15625, 3.0 * 2 ** -20, 255.0])
    np.testing.assert_array_equal(mlp.bf16(exact), exact)
    one = 1.0
    ulp = 2 ** -7
    assert mlp.bf16(one + ulp / 2) == one            # tie -> even mantissa (1.0)
    assert mlp.bf16(one + 3 * ulp / 2) == one + 2 * ulp  # tie -> even (1 + 2 ulp)
    assert mlp.bf16(one + 0.6 * ulp) == one + ulp
    x = np.random.default_rng(0).standard_normal(1000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8)


def test_gradients_match_central_differences():
    g = np.random.default_rng(1)
    params = mlp.init_params(7)
    X = g.standard_normal((12, 160)) * 0.5
    y = g.standard_normal(12)
    out, cache = mlp.forward(params, X, quant=False)
    grads = mlp.backward(cache, out, y)
    eps = 1e-6
    for l, (W, b) in enumerate(params):
        for (i, j) in [(0, 0), (5, 3 % W.shape[1]), (W.shape[0] - 1, W.shape[1] - 1)]:
            Wp = [(w.copy(), bb.copy()) for w, bb in params]
            Wm = [(w.copy(), bb.copy()) for w, bb in params]
            Wp[l][0][i, j] += eps
            Wm[l][0][i, j] -= eps
            fp = mlp.mse(mlp.forward(Wp, X, quant=False)[0], y)
            fm = mlp.mse(mlp.forward(Wm, X, quant=False)[0], y)
            num = (fp - fm) / (2 * eps)
            assert abs(num - grads[l][0][i, j]) <= 1e-6 * max(1.0, abs(num))
        k = b.shape[0] - 1
        Bp = [(w.copy(), bb.copy()) for w, bb in params]
        Bm = [(w.copy(), bb.copy()) for w, bb in params]
        Bp[l][1][k] += eps
        Bm[l][1][k] -= eps
        num = (mlp.mse(mlp.forward(Bp, X, quant=False)[0], y) - mlp.mse(mlp.forward(Bm, X, quant=False)[0], y)) / (2 * eps)
        assert abs(num - grads[l][1][k]) <= 1e-6 * max(1.0, abs(num))


def test_adam_first_step_moves_by_lr():
    # after one step with a nonzero gradient, each parameter moves by lr * sign(g)
    params = [(np.ones((2, 2)), np.zeros(2))]
    grads = [(np.array([[0.3, -2.0], [1e-3, 5.0]]), np.array([0.0, -1.0]))]
    st = mlp.adam_state(params)
    new = mlp.adam_step(params, grads, st, lr=0.01)
    np.testing.assert_allclose(new[0][0], 1.0 - 0.01 * np.sign(grads[0][0]), rtol=1e-6)
    np.testing.assert_allclose(new[0][1], [0.0, 0.01], atol=1e-9)


def test_descriptor_invariants():
    g = np.random.default_rng(3)
    balls = np.column_stack([g.normal(0.3, 0.1, (500, 3)), g.uniform(0.01, 0.05, 500), np.ones(500)])
    d = mlp.descriptor(balls)
    assert d.shape == (64,) and abs(d.sum() - 1) < 1e-12 and np.all(d >= 0)
    # invariant under rigid motions of the shape
    R, _ = np.linalg.qr(g.standard_normal((3, 3)))
    moved = balls.copy()
    moved[:, :3] = balls[:, :3] @ R.T + np.array([1.0, -2.0, 0.5])
    np.testing.assert_allclose(mlp.descriptor(moved), d, atol=1e-12)
    # a single ball: all mass in the first bin
    one = mlp.descriptor(np.array([[0.2, 0.1, 0.0, 0.03, 1.0]]))
    assert one[0] == 1.0


def _hamilton(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_rotation_matrix_is_the_quaternion_rotation():
    rng = np.random.default_rng(3)
    for _ in range(20):
        q1, q2 = rng.standard_normal(4), rng.standard_normal(4)
        R = mlp.rotation_matrix(q1)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14
        np.testing.assert_allclose(mlp.rotation_matrix(-q1), R, atol=1e-15)
        # a homomorphism: the product of quaternions is the product of rotations
        np.testing.assert_allclose(mlp.rotation_matrix(_hamilton(q1, q2)), R @ mlp.rotation_matrix(q2), atol=1e-13)
        # R v equals the quaternion sandwich q (0, v) q*
        qn = q1 / np.linalg.norm(q1)
        v = rng.standard_normal(3)
        conj = qn * np.array([1, -1, -1, -1])
        np.testing.assert_allclose(_hamilton(_hamilton(qn, np.r_[0.0, v]), conj)[1:], R @ v, atol=1e-13)
    # a quarter turn about z takes x to y
    h = np.sqrt(0.5)
    np.testing.assert_allclose(mlp.rotation_matrix([h, 0, 0, h]) @ [1, 0, 0], [0, 1, 0], atol=1e-15)


def test_features_layout():
    q = np.array([[-0.5, 0.5, -0.5, 0.5], [0.6, 0.8, 0, 0], [2.0, 0, 0, 0]])
    da = np.arange(64) / np.arange(64).sum()
    X = mlp.features(q, da, np.zeros(64))
    assert X.shape == (3, 160)
    # q and -q: the same inputs
    np.testing.assert_allclose(mlp.features(-q, da, np.zeros(64)), X, atol=1e-15)
    # the identity (any positive scale): R = I, sin(pi R) = 0, cos(pi R) = -1 on the diagonal, 1 off it
    np.testing.assert_allclose(X[2, 0:9], np.eye(3).reshape(-1), atol=1e-15)
    np.testing.assert_allclose(X[2, 9:18], 0, atol=1e-15)
    np.testing.assert_allclose(X[2, 18:27], np.where(np.eye(3).reshape(-1) > 0, -1.0, 1.0), atol=1e-15)
    np.testing.assert_allclose(X[:, 9:18] ** 2 + X[:, 18:27] ** 2, 1.0, atol=1e-14)
    np.testing.assert_allclose(X[0, 27:91], 64 * da, atol=1e-15)
    assert np.all(X[:, 91:155] == 0) and np.all(X[:, mlp.IN_USED:] == 0)