"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module holds no arithmetic of the correlation method: it only draws ball
sets, rotations and translation grids from fixed seeds.  Both the FP64 oracle
and the GPU path receive the arrays it returns; neither computes them.

Ball sets are ``(n, 5)`` float64 arrays with columns ``x, y, z, r, w``: centre,
radius and weight of each ball.  The paper assigns the weights freely (its
equiradius construction, Sec. 2.2), so every generator uses unit weights.

The paper's own shapes are triangle meshes sampled by its Algorithm 1 (App. A);
they are not available, so these generators stand in for them.  The shapes live
in the unit-edge box, as the paper's Table 2 epsilon column implies.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "uniform_balls", "mixture_balls", "random_quaternions", "grid_for",
    "Grid", "tiny_case", "single_rotation_case", "batched_rotations_case",
    "uneven_batch_case", "loguniform_int",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_balls(n: int, seed: int, rlo: float = 0.03, rhi: float = 0.08) -> np.ndarray:
    """Centres uniform in the unit cube, radii uniform in [rlo, rhi], unit weights."""
    g = _rng(seed)
    out = np.empty((n, 5))
    out[:, :3] = g.random((n, 3))
    out[:, 3] = rlo + (rhi - rlo) * g.random(n)
    out[:, 4] = 1.0
    return out


def mixture_balls(n: int, seed: int, components: int = 8, centre: bool = True) -> np.ndarray:
    """Gaussian-mixture blob of ``components`` isotropic clusters.

    Cluster means are uniform in [0.25, 0.75]^3 and cluster standard deviations
    uniform in [0.05, 0.10]; each ball picks a cluster with equal probability and
    a centre is redrawn until it falls inside the unit cube.  Radii are
    lognormal with log-mean ln(0.02) and log-sd 0.3, clipped to [0.004, 0.1].
    With ``centre`` the set is translated so its volume-weighted centroid is the
    origin (rotations then turn the shape about its own centroid).
    """
    g = _rng(seed)
    means = 0.25 + 0.5 * g.random((components, 3))
    sds = 0.05 + 0.05 * g.random(components)
    pick = g.integers(0, components, size=n)
    pts = np.empty((n, 3))
    todo = np.arange(n)
    while todo.size:
        c = pick[todo]
        cand = means[c] + sds[c, None] * g.standard_normal((todo.size, 3))
        ok = np.all((cand >= 0.0) & (cand <= 1.0), axis=1)
        pts[todo[ok]] = cand[ok]
        todo = todo[~ok]
    r = np.clip(np.exp(math.log(0.02) + 0.3 * g.standard_normal(n)), 0.004, 0.1)
    out = np.empty((n, 5))
    out[:, :3] = pts
    out[:, 3] = r
    out[:, 4] = 1.0
    if centre:
        vol = r ** 3
        out[:, :3] -= (vol[:, None] * pts).sum(0) / vol.sum()
    return out


def random_quaternions(n: int, seed: int, canonical: bool = False) -> np.ndarray:
    """Uniform random unit quaternions (w, x, y, z): normalised 4D Gaussians."""
    g = _rng(seed)
    q = g.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    if canonical:
        q[q[:, 0] < 0] *= -1.0
    return q


def super_fibonacci_quaternions(n: int, seed: int) -> np.ndarray:
    """n unit quaternions (w, x, y, z), w >= 0, spread evenly over the rotations:
    the super-Fibonacci spiral of Alexa (CVPR 2022), point i of which has
    s = i + 1/2, radii sqrt(s/n) and sqrt(1 - s/n) in the two planes of R^4 and
    angles 2 pi s / sqrt(2) and 2 pi s / psi, psi the real root > 1 of
    psi^4 = psi + 4.  The whole set is turned by one rotation drawn from `seed`,
    so that different seeds give differently placed, equally even sets."""
    psi = 1.533751168755204288118041
    s = np.arange(n, dtype=np.float64) + 0.5
    t = s / n
    r, rr = np.sqrt(t), np.sqrt(1.0 - t)
    a, b = 2.0 * np.pi * s / math.sqrt(2.0), 2.0 * np.pi * s / psi
    p = np.stack([r * np.sin(a), r * np.cos(a), rr * np.sin(b), rr * np.cos(b)], axis=1)
    g = random_quaternions(1, seed)[0]
    w1, x1, y1, z1 = g
    w2, x2, y2, z2 = p.T
    q = np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                  w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=1)
    q[q[:, 0] < 0] *= -1.0
    return q


def loguniform_int(g: np.random.Generator, lo: int, hi: int, size: int) -> np.ndarray:
    return np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * g.random(size)).astype(np.int64)


@dataclass
class Grid:
    """Translation grid t_n = origin + (L/n) * idx, idx in [0, n)^3, period L."""
    n: int
    box: float
    origin: tuple
    sigma: float = 2.0
    kb_width: int = 8
    tol: float = 1e-6

    @property
    def h(self) -> float:
        return self.box / self.n


def grid_for(A: np.ndarray, B: np.ndarray, n: int, sigma: float = 2.0, kb_width: int = 8,
             tol: float = 1e-6, pad: float = 0.0) -> Grid:
    """Period L large enough that translated copies of the score never overlap.

    The score is non-zero only where some ball of A meets some ball of the moved
    B, i.e. for |t| < R_A + R_B + max r_A + max r_B with R_X the largest centre
    distance from the origin; pad widens that reach (balls grown by r0 on both
    sides need pad = 2 r0).  L is twice the reach, rounded up to a multiple of
    1/8, and the grid is centred on the origin.
    """
    ra = np.linalg.norm(A[:, :3], axis=1).max() + A[:, 3].max()
    rb = np.linalg.norm(B[:, :3], axis=1).max() + B[:, 3].max()
    L = math.ceil(2.0 * (ra + rb + pad) * 8.0) / 8.0
    return Grid(n=n, box=L, origin=(-L / 2,) * 3, sigma=sigma, kb_width=kb_width, tol=tol)


# ---------------------------------------------------------------------------
# Workloads.  Sizes follow the five benchmark configurations: a tiny plain case,
# one rotation of two 4096-ball shapes on a 128^3 grid, 512 rotations of a
# 20000/2000-ball pair on 64^3, an uneven batch of 64 pairs, and the proposal
# network's data.
# ---------------------------------------------------------------------------

def tiny_case():
    """64 + 64 uniform balls, radii in [0.03, 0.08], identity rotation.

    The plain lens sum is taken on the 16^3 grid over [-1, 1)^3 (spacing 1/8);
    the spectral route needs a period of at least 2.32, so it runs on the 32^3
    grid of period 4 whose index range [8, 24) is that same 16^3 grid.
    """
    A = uniform_balls(64, 1)
    B = uniform_balls(64, 2)
    q = np.array([[1.0, 0.0, 0.0, 0.0]])
    g = Grid(n=32, box=4.0, origin=(-2.0, -2.0, -2.0))
    plain = dict(n=16, h=0.125, origin=(-1.0, -1.0, -1.0), crop=(8, 24))
    return A, B, q, g, plain


def single_rotation_case(n_a: int = 4096, n_b: int = 4096, n: int = 128, pair: int = 0):
    A = mixture_balls(n_a, 1000 + pair)
    B = mixture_balls(n_b, 2000 + pair)
    q = random_quaternions(1, 3000 + pair)
    return A, B, q, grid_for(A, B, n)


def batched_rotations_case(n_a: int = 20000, n_b: int = 2000, n: int = 64, n_rot: int = 512,
                           pair: int = 0):
    A = mixture_balls(n_a, 1000 + pair)
    B = mixture_balls(n_b, 2000 + pair)
    q = random_quaternions(n_rot, 3000 + pair)
    return A, B, q, grid_for(A, B, n)


def uneven_batch_case(n_pairs: int = 64, n_rot: int = 32, seed: int = 4000,
                      lo: int = 500, hi: int = 50000, sizes=(32, 64, 128)):
    """Pairs with log-uniform ball counts and per-pair grid sizes."""
    g = _rng(seed)
    na = loguniform_int(g, lo, hi, n_pairs)
    nb = loguniform_int(g, lo, hi, n_pairs)
    ns = np.asarray(sizes)[g.integers(0, len(sizes), size=n_pairs)]
    pairs = []
    for p in range(n_pairs):
        A = mixture_balls(int(na[p]), 1000 + p)
        B = mixture_balls(int(nb[p]), 2000 + p)
        q = random_quaternions(n_rot, 3000 + p)
        pairs.append((A, B, q, grid_for(A, B, int(ns[p]))))
    return pairs


def proposal_pairs(n_pairs: int, seed: int, lo: int = 500, hi: int = 5000, n: int = 64):
    """Pairs for the rotation-proposal workflow: mixture shapes with log-uniform
    ball counts in [lo, hi] (the uneven batch's model with its upper count
    capped so that generating training data stays short) on an n^3 grid."""
    g = _rng(seed)
    na = loguniform_int(g, lo, hi, n_pairs)
    nb = loguniform_int(g, lo, hi, n_pairs)
    pairs = []
    for p in range(n_pairs):
        A = mixture_balls(int(na[p]), seed + 1000 + p)
        B = mixture_balls(int(nb[p]), seed + 2000 + p)
        pairs.append((A, B, grid_for(A, B, n)))
    return pairs
