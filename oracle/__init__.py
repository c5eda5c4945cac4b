"""FP64 CPU oracle for the ball-union correlation (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never does, and this package never
imports the product library: the two share no code.  Inputs come from the
seeded generators in ``synth``.

Two oracles, both written from Behandish & Ilies (CAD 2016):

* ``o1_*`` -- the plain method: the score g(R, t) = <f_A, f_{(R,t)B}>
  (Sec. 3.1 eq. eq_relg_0) of two unions of balls whose defining functions are
  weighted sums of ball indicators (Sec. 2.1 eq. eq_un, Sec. 2.2 eq. eq_Psum),
  summed pair by pair as closed-form lens volumes.
* ``o2_*`` -- the band-limited Fourier route: per-shape spectra from a direct
  NDFT of the knots (Sec. 2.5 eq. eq_rhoPhat) weighted by each ball's transform,
  their correlation spectrum F_A conj(F_RB) (Sec. 3.2 eq. eq_ccghat), and an FP64
  inverse FFT onto an L-periodic translation grid, keeping |m_d| < N/2.
* ``*_sc_*`` -- the shape-complementarity score (Sec. 4.2 eq. eq_score), built
  from the two above by its definition.
* ``lift_*`` -- the 4D lifted correlation of Sec. 2.2 (knots lifted to
  (x, r), each carrying a half-cone, eq. eq_rhoA, eq_L2cone, eq_coneconv) and
  Sec. 3.1 (one shape r-mirrored, Lemma 2, eq. eq_ORA, eq_convgA): its slice at
  height h is the sum over pairs of the 4D volume W of the intersection of a
  downward and an upward cone, in closed form; ``o2_lift_*`` is its
  band-limited Fourier route.
* ``raster_*`` -- the uniform-grid baseline of Sec. 5.2 / Sec. 6.2: both
  unions sampled on the translation lattice, and the number of samples where
  they meet, counted directly for each translation.
* ``obstacle``, ``o1_obstacle_points``, ``offset_balls`` -- the configuration
  obstacle as the positive set of the score (Sec. 3.1 eq. eq_obs), its
  pairwise Minkowski-sum form, and the offset slices (Sec. 3.1).

The heavy loops live in ``oracle.c`` (plain C, OpenMP), built on first use with
gcc into ``liboracle.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIBRARY names another build of oracle.c (an instrumented one, say);
# it is loaded as it is, never rebuilt
_LIB_OVERRIDE = os.environ.get("ORACLE_LIBRARY")
_LIB = _LIB_OVERRIDE or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (FP64, no fast-math)."""
    if _LIB_OVERRIDE:
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d, p, i64, i32 = ctypes.c_double, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.orc_lens_volume.restype = d
        lib.orc_lens_volume.argtypes = [d, d, d]
        lib.orc_ball_ft.restype = d
        lib.orc_ball_ft.argtypes = [d, d]
        lib.orc_quat_to_rot.argtypes = [p, p]
        lib.orc_o1_points.argtypes = [p, i64, p, i64, p, p, i64, p]
        lib.orc_o1_grid.argtypes = [p, i64, p, i64, p, p, d, i32, p]
        lib.orc_o2_spectrum.argtypes = [p, i64, p, i32, d, p, p]
        lib.orc_lift_w.restype = d
        lib.orc_lift_w.argtypes = [d, d]
        lib.orc_lift_what.restype = d
        lib.orc_lift_what.argtypes = [d, d]
        lib.orc_o1_lift_grid.argtypes = [p, i64, p, i64, p, p, d, i32, d, p]
        lib.orc_o2_lift_spectrum.argtypes = [p, i64, p, i64, p, i32, d, d, p, p]
        lib.orc_raster_bitmaps.argtypes = [p, i64, p, i64, p, p, d, i32, p, p]
        lib.orc_raster_counts.argtypes = [p, p, i32, p, i64, p]
        lib.orc_set_threads.argtypes = [i32]
        lib.orc_get_threads.restype = i32
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (for timing; results do not depend on it)."""
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def lens_volume(d, a, b):
    """Volume of the intersection of balls of radii a and b at centre distance d."""
    lib = _load()
    d, a, b = np.broadcast_arrays(np.asarray(d, float), np.asarray(a, float), np.asarray(b, float))
    out = np.array([lib.orc_lens_volume(x, y, z) for x, y, z in zip(d.ravel(), a.ravel(), b.ravel())])
    return out.reshape(d.shape) if d.shape else float(out[0])


def ball_ft(k, r):
    """Fourier transform of the indicator of a ball of radius r at |k| (rad / length)."""
    lib = _load()
    k, r = np.broadcast_arrays(np.asarray(k, float), np.asarray(r, float))
    out = np.array([lib.orc_ball_ft(x, y) for x, y in zip(k.ravel(), r.ravel())])
    return out.reshape(k.shape) if k.shape else float(out[0])


def quat_to_rot(q) -> np.ndarray:
    """Row-major rotation matrix of quaternion (w, x, y, z), Hamilton convention."""
    lib = _load()
    q = _f64(q)
    R = np.empty(9)
    lib.orc_quat_to_rot(_ptr(q), _ptr(R))
    return R.reshape(3, 3)


def o1_points(A, B, R, t) -> np.ndarray:
    """Plain score sum_ij c_i d_j V(|x_i - R y_j - t|) at each row of t (non-periodic)."""
    lib = _load()
    A, B, R, t = _f64(A), _f64(B), _f64(R), _f64(np.atleast_2d(t))
    out = np.empty(len(t))
    lib.orc_o1_points(_ptr(A), len(A), _ptr(B), len(B), _ptr(R), _ptr(t), len(t), _ptr(out))
    return out


def o1_grid(A, B, R, origin, h, n) -> np.ndarray:
    """Plain score on t = origin + h*(ix, iy, iz), returned as [iz][iy][ix] (non-periodic)."""
    lib = _load()
    A, B, R, o = _f64(A), _f64(B), _f64(R), _f64(origin)
    out = np.empty((n, n, n))
    lib.orc_o1_grid(_ptr(A), len(A), _ptr(B), len(B), _ptr(R), _ptr(o), float(h), int(n), _ptr(out))
    return out


def o2_spectrum(balls, R, n, L) -> np.ndarray:
    """F(k_m) = sum_i c_i Bhat(|k_m|; r_i) exp(-i k_m . R x_i), k_m = 2 pi m / L.

    Full cube in FFT order, [mz][my][mx]; modes with some m_d = -n/2 are zero.
    """
    lib = _load()
    balls, R = _f64(balls), _f64(R)
    re = np.empty((n, n, n))
    im = np.empty((n, n, n))
    lib.orc_o2_spectrum(_ptr(balls), len(balls), _ptr(R), int(n), float(L), _ptr(re), _ptr(im))
    return re + 1j * im


def mode_numbers(n) -> np.ndarray:
    """Signed mode number of each FFT-order index of an n-point axis."""
    i = np.arange(n)
    return np.where(i < n // 2, i, i - n)


def o2_correlation_spectrum(FA, FB, L, origin) -> np.ndarray:
    """S_m = F_A conj(F_RB) exp(i k_m . origin) / L^3, so that s(t_n) = sum_m S_m exp(2 pi i m.n / N)."""
    n = FA.shape[0]
    k = 2.0 * np.pi * mode_numbers(n) / L
    ph = (np.exp(1j * k * origin[2])[:, None, None] * np.exp(1j * k * origin[1])[None, :, None]
          * np.exp(1j * k * origin[0])[None, None, :])
    return FA * np.conj(FB) * ph / L ** 3


def o2_scores_from_spectra(FA, FB, L, origin) -> np.ndarray:
    n = FA.shape[0]
    S = o2_correlation_spectrum(FA, FB, L, origin)
    return np.real(np.fft.ifftn(S)) * n ** 3


def o2_scores(A, B, q, n, L, origin) -> np.ndarray:
    """Band-limited score on t_n = origin + (L/n) idx, [iz][iy][ix], for rotation quaternion q."""
    FA = o2_spectrum(A, np.eye(3), n, L)
    FB = o2_spectrum(B, quat_to_rot(q), n, L)
    return o2_scores_from_spectra(FA, FB, L, origin)


def o2_eval_at(FA, FB, L, t) -> np.ndarray:
    """The same band-limited score evaluated at arbitrary translations (direct mode sum)."""
    n = FA.shape[0]
    k = 2.0 * np.pi * mode_numbers(n) / L
    S = FA * np.conj(FB) / L ** 3
    out = []
    for p in np.atleast_2d(t):
        ph = (np.exp(1j * k * p[2])[:, None, None] * np.exp(1j * k * p[1])[None, :, None]
              * np.exp(1j * k * p[0])[None, None, :])
        out.append(np.real(np.sum(S * ph)))
    return np.array(out)


# ---- single-configuration query (Sec. 4.1, eq. eq_single) ---------------------

def o2_query(FA, FB, L, t, mode_radius2) -> np.ndarray:
    """The Parseval form of the score at arbitrary translations, summed only over
    the modes with |m|^2 <= mode_radius2 (and |m_d| < N/2):
    s(t) = (1/L^3) sum_m F_A(k_m) conj(F_RB(k_m)) exp(i k_m . t)."""
    n = FA.shape[0]
    m = mode_numbers(n)
    m2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    keep = (m2 <= mode_radius2) & (np.abs(m)[:, None, None] < n // 2) & (np.abs(m)[None, :, None] < n // 2) \
        & (np.abs(m)[None, None, :] < n // 2)
    k = 2.0 * np.pi * m / L
    S = np.where(keep, FA * np.conj(FB), 0.0) / L ** 3
    out = []
    for p in np.atleast_2d(t):
        ph = (np.exp(1j * k * p[2])[:, None, None] * np.exp(1j * k * p[1])[None, :, None]
              * np.exp(1j * k * p[0])[None, None, :])
        out.append(np.real(np.sum(S * ph)))
    return np.array(out)


def query_mode_count(n, mode_radius2) -> int:
    """Number of modes |m|^2 <= mode_radius2, |m_d| < n/2 (the full sphere)."""
    m = mode_numbers(n)
    ok = np.abs(m) < n // 2
    m2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    return int(np.sum((m2 <= mode_radius2) & ok[:, None, None] & ok[None, :, None] & ok[None, None, :]))


# ---- shape-complementarity score (Sec. 4.2, eq. eq_score) ---------------------
#
# The affinity of a shape is F_S = i (f_{S (+) B0} - lam f_S).  For a union of
# balls the offset by B0 = B(0, r0) is the union of the balls grown by r0, so
# with F_S = i a_S the score G = F_RS2 star F_S1 equals <a_S1, a_(R,t)S2>: the
# plain score of two signed unions.

def sc_grown(balls, r0) -> np.ndarray:
    """Every ball grown by r0 (the offset S (+) B(0, r0) of a union of balls)."""
    b = _f64(balls).copy()
    b[:, 3] += r0
    return b


def sc_affinity_balls(balls, r0, lam) -> np.ndarray:
    """a_S = f_{S (+) B0} - lam f_S as one signed union: the grown balls with
    their weights and the original balls with weights times -lam."""
    b = _f64(balls)
    neg = b.copy()
    neg[:, 4] *= -lam
    return np.vstack([sc_grown(b, r0), neg])


def o1_sc_grid(A, B, R, origin, h, n, r0, lam) -> np.ndarray:
    """Plain SC score, expanded into its four lens-sum terms:
    G = g(A+, B+) - lam g(A+, B) - lam g(A, B+) + lam^2 g(A, B), '+' = grown by r0."""
    Ag, Bg = sc_grown(A, r0), sc_grown(B, r0)
    return (o1_grid(Ag, Bg, R, origin, h, n) - lam * o1_grid(Ag, B, R, origin, h, n)
            - lam * o1_grid(A, Bg, R, origin, h, n) + lam * lam * o1_grid(A, B, R, origin, h, n))


def o2_sc_spectrum(balls, R, n, L, r0, lam) -> np.ndarray:
    """Spectrum of the affinity: F_{S (+) B0}(k) - lam F_S(k)."""
    return o2_spectrum(sc_grown(balls, r0), R, n, L) - lam * o2_spectrum(balls, R, n, L)


def o2_sc_scores(A, B, q, n, L, origin, r0, lam) -> np.ndarray:
    """Band-limited SC score on the translation grid, [iz][iy][ix]."""
    FA = o2_sc_spectrum(A, np.eye(3), n, L, r0, lam)
    FB = o2_sc_spectrum(B, quat_to_rot(q), n, L, r0, lam)
    return o2_scores_from_spectra(FA, FB, L, origin)


def peak(scores) -> tuple:
    """Largest score of each rotation and its linear index (lowest index on ties)."""
    s = np.asarray(scores).reshape(scores.shape[0], -1) if np.ndim(scores) == 4 else np.asarray(scores).reshape(1, -1)
    idx = np.argmax(s, axis=1)
    return s[np.arange(len(s)), idx], idx


# ---- configuration obstacle and offset obstacles ------------------------------
#
# For a fixed rotation the translational obstacle is the set of translations
# where the score is positive (Sec. 3.1 eq. eq_obs); for unions of balls it is
# the union, over every pair of primitives, of the ball of radius r_i + rho_j
# about x_i - R y_j (the Minkowski-sum form of Sec. 3.1, eqs. eq_ORP and
# eq_ORA, taken pair by pair).  Slices of the lifted obstacle away from r = 0
# are the obstacles of the primitives offset by a total of delta (Sec. 3.1,
# offset obstacles); here the whole offset is put on A's balls.

def obstacle(scores, threshold=0.0) -> np.ndarray:
    """The translations whose score exceeds threshold (threshold 0: eq. eq_obs)."""
    return np.asarray(scores) > threshold


def o1_obstacle_points(A, B, R, t) -> np.ndarray:
    """Obstacle membership from the Minkowski-sum form, by brute force over all
    pairs: t is inside iff |x_i - R y_j - t| < r_i + rho_j for some pair (for
    positive weights, where this is exactly where the plain score is > 0)."""
    A, B, R = _f64(A), _f64(B), _f64(R)
    t = _f64(np.atleast_2d(t))
    RB = B[:, :3] @ R.T
    inside = np.zeros(len(t), dtype=bool)
    for i in range(len(A)):
        d = A[i, None, None, :3] - RB[None, :, :] - t[:, None, :]     # [t][j][3]
        dist = np.sqrt(np.sum(d * d, axis=2))
        inside |= np.any(dist < A[i, 3] + B[None, :, 3], axis=1)
    return inside


def offset_balls(balls, delta) -> np.ndarray:
    """Every primitive ball's radius changed by delta (grown for delta > 0,
    shrunk for delta < 0; every radius must stay positive)."""
    b = _f64(balls).copy()
    b[:, 3] += delta
    if len(b) and not np.all(b[:, 3] > 0):
        raise ValueError("offset %g leaves a radius <= 0" % delta)
    return b


def o2_offset_scores(A, B, q, n, L, origin, delta) -> np.ndarray:
    """Band-limited score of the offset slice delta: A's balls offset by delta."""
    return o2_scores(offset_balls(A, delta), B, q, n, L, origin)


# ---- 4D lifted correlation (Sec. 2.2, Sec. 3.1) -------------------------------

def lift_w(d, P):
    """4D volume of the intersection of two opposite cones with axes d apart whose
    cross-sections' radii sum to P at every height: pi (P^2 - d^2)^2 / 24 for d < P."""
    lib = _load()
    d, P = np.broadcast_arrays(np.asarray(d, float), np.asarray(P, float))
    out = np.array([lib.orc_lift_w(x, y) for x, y in zip(d.ravel(), P.ravel())])
    return out.reshape(d.shape) if d.shape else float(out[0])


def lift_what(k, P):
    """3D Fourier transform of t -> lift_w(|t|, P) at |k|."""
    lib = _load()
    k, P = np.broadcast_arrays(np.asarray(k, float), np.asarray(P, float))
    out = np.array([lib.orc_lift_what(x, y) for x, y in zip(k.ravel(), P.ravel())])
    return out.reshape(k.shape) if k.shape else float(out[0])


def o1_lift_grid(A, B, R, origin, h, n, height) -> np.ndarray:
    """Plain slice at `height` of the lifted correlation on t = origin + h*idx,
    [iz][iy][ix], not periodic: sum_ij c_i d_j W(|x_i - R y_j - t|; r_i + rho_j - height)."""
    lib = _load()
    A, B, R, o = _f64(A), _f64(B), _f64(R), _f64(origin)
    out = np.empty((n, n, n))
    lib.orc_o1_lift_grid(_ptr(A), len(A), _ptr(B), len(B), _ptr(R), _ptr(o), float(h), int(n), float(height),
                         _ptr(out))
    return out


def o2_lift_spectrum(A, B, R, n, L, height) -> np.ndarray:
    """Band-limited spectrum of the lifted slice at `height` (FFT order, [mz][my][mx])."""
    lib = _load()
    A, B, R = _f64(A), _f64(B), _f64(R)
    re = np.empty((n, n, n))
    im = np.empty((n, n, n))
    lib.orc_o2_lift_spectrum(_ptr(A), len(A), _ptr(B), len(B), _ptr(R), int(n), float(L), float(height), _ptr(re),
                             _ptr(im))
    return re + 1j * im


def o2_lift_scores(A, B, q, n, L, origin, height) -> np.ndarray:
    """Band-limited lifted slice at `height` on t_n = origin + (L/n) idx, [iz][iy][ix]."""
    G = o2_lift_spectrum(A, B, quat_to_rot(q), n, L, height)
    k = 2.0 * np.pi * mode_numbers(n) / L
    ph = (np.exp(1j * k * origin[2])[:, None, None] * np.exp(1j * k * origin[1])[None, :, None]
          * np.exp(1j * k * origin[0])[None, None, :])
    return np.real(np.fft.ifftn(G * ph / L ** 3)) * n ** 3


# ---- rasterization baseline (Sec. 5.2, Sec. 6.2) ---------------------------------

def raster_bitmaps(A, B, R, origin, h, n):
    """Sample grids [z][y][x] (uint8): A at origin + h u, R B at h v (v signed, FFT order)."""
    lib = _load()
    A, B, R, o = _f64(A), _f64(B), _f64(R), _f64(origin)
    a = np.zeros((n, n, n), np.uint8)
    b = np.zeros((n, n, n), np.uint8)
    lib.orc_raster_bitmaps(_ptr(A), len(A), _ptr(B), len(B), _ptr(R), _ptr(o), float(h), int(n), _ptr(a), _ptr(b))
    return a, b


def raster_counts(a, b, idx) -> np.ndarray:
    """sum_u a(u) b(u - t) (periodic) at translation indices idx [k][3] = (tx, ty, tz)."""
    lib = _load()
    n = a.shape[0]
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1, 3))
    out = np.empty(len(idx), np.int64)
    lib.orc_raster_counts(_ptr(np.ascontiguousarray(a)), _ptr(np.ascontiguousarray(b)), int(n), _ptr(idx), len(idx),
                          _ptr(out))
    return out


def raster_counts_grid(A, B, q, n, L, origin) -> np.ndarray:
    """Counts at every translation index, [tz][ty][tx] (O(n^6): small n only)."""
    a, b = raster_bitmaps(A, B, quat_to_rot(q), origin, L / n, n)
    t = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)[:, ::-1]
    return raster_counts(a, b, t).reshape(n, n, n)
