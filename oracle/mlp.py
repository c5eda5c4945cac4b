"""FP64 CPU reference of the rotation-proposal network (test infrastructure only).

The network maps a rotation quaternion and two 64-bin radial shape descriptors
to a predicted peak score: four linear layers 160 -> 256 -> 256 -> 256 -> 1 with
ReLU between them.  Input: the quaternion's rotation matrix R (9), sin(pi R) and
cos(pi R) entrywise (9 + 9), 64 x descriptor of A (64), 64 x descriptor of B
(64), zero-padded to 160.  On the GPU the weights and the inputs of every layer are
rounded to bfloat16 and the products accumulate in FP32; with ``quant=True`` this
reference applies the same roundings and then computes in FP64, so the two can
be compared at the size of FP32 accumulation error.

The loss is the mean squared error; training uses Adam.  Everything here is the
textbook definition, written out in numpy.
"""
from __future__ import annotations

import numpy as np

DIMS = (160, 256, 256, 256, 1)
IN_USED = 155
BINS = 64


def bf16(x) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    return out.reshape(np.shape(x))


def init_params(seed: int):
    """He-uniform weights, zero biases (W[l] has shape (in, out))."""
    g = np.random.Generator(np.random.PCG64(seed))
    params = []
    for l in range(4):
        fan_in, fan_out = DIMS[l], DIMS[l + 1]
        bound = np.sqrt(6.0 / fan_in)
        params.append((g.uniform(-bound, bound, (fan_in, fan_out)), np.zeros(fan_out)))
    return params


def forward(params, X, quant=True):
    """Returns the outputs (n,) and the cache of layer inputs and pre-activations."""
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(params):
        a_in = bf16(a) if quant else a
        W_used = bf16(W) if quant else W
        z = a_in @ W_used + b
        cache.append((a_in, W_used, z))
        a = np.maximum(z, 0.0) if l < 3 else z
    return a[:, 0], cache


def mse(y_pred, y):
    d = y_pred - y
    return float(np.mean(d * d))


def backward(cache, y_pred, y):
    """Gradients of the mean squared error with respect to (W, b) of every layer.

    With rounding on, the gradient is taken through the rounded values (the
    rounding itself is treated as the identity), as the GPU kernels do.
    """
    n = len(y)
    dz = (2.0 / n) * (y_pred - y)[:, None]
    grads = [None] * 4
    for l in range(3, -1, -1):
        a_in, W_used, z = cache[l]
        grads[l] = (a_in.T @ dz, dz.sum(axis=0))
        if l > 0:
            da = dz @ W_used.T
            dz = da * (cache[l - 1][2] > 0)
    return grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; state = {'t': int, 'm': [...], 'v': [...]}."""
    state["t"] += 1
    t = state["t"]
    new = []
    for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        out = []
        for k, (p, gp) in enumerate(((W, gW), (b, gb))):
            m = state["m"][2 * l + k] = beta1 * state["m"][2 * l + k] + (1 - beta1) * gp
            v = state["v"][2 * l + k] = beta2 * state["v"][2 * l + k] + (1 - beta2) * gp * gp
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            out.append(p - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(out))
    return new


def adam_state(params):
    z = []
    for W, b in params:
        z += [np.zeros_like(W), np.zeros_like(b)]
    return {"t": 0, "m": [x.copy() for x in z], "v": [x.copy() for x in z]}


def descriptor(balls, bins: int = BINS) -> np.ndarray:
    """Histogram of ball volume (weight x r^3) over the distance of each centre
    from the shape's volume-weighted centroid, bins of width 1/bins on [0, 1]
    (farther centres go to the last bin), normalised to sum 1."""
    b = np.asarray(balls, dtype=np.float64)
    vol = b[:, 4] * b[:, 3] ** 3
    c = (vol[:, None] * b[:, :3]).sum(0) / vol.sum()
    d = np.linalg.norm(b[:, :3] - c, axis=1)
    idx = np.minimum((d * bins).astype(np.int64), bins - 1)
    h = np.zeros(bins)
    np.add.at(h, idx, vol)
    return h / h.sum()


def rotation_matrix(q) -> np.ndarray:
    """R(q) of a quaternion (w, x, y, z), Hamilton convention: the matrix of
    v -> q v q* for the normalised q, i.e. the rotation by angle 2 acos(w)
    about (x, y, z); q and -q give the same matrix."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q)
    w, v = q[0], q[1:]
    # Rodrigues form: R = (w^2 - |v|^2) I + 2 v v^T + 2 w [v]_x
    vx = np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])
    return (w * w - v @ v) * np.eye(3) + 2.0 * np.outer(v, v) + 2.0 * w * vx


def features(quats, desc_a, desc_b) -> np.ndarray:
    """Network inputs: the rotation matrix of each quaternion (row-major, the
    same for q and -q), sin and cos of pi times each entry, both descriptors
    times the bin count, zero padding to 160."""
    q = np.atleast_2d(np.asarray(quats, dtype=np.float64))
    X = np.zeros((len(q), DIMS[0]))
    for i in range(len(q)):
        R = rotation_matrix(q[i]).reshape(-1)
        X[i, 0:9] = R
        X[i, 9:18] = np.sin(np.pi * R)
        X[i, 18:27] = np.cos(np.pi * R)
    X[:, 27:27 + BINS] = BINS * np.asarray(desc_a, dtype=np.float64)
    X[:, 27 + BINS:27 + 2 * BINS] = BINS * np.asarray(desc_b, dtype=np.float64)
    return X
