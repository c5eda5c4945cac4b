"""Python binding of libcorr (include/corr.h): MI355X ball-union correlation.

The functions named like the C entry points (``corr_create``, ``corr_eval``, ...)
only marshal arguments: every step of the computation runs in the HIP kernels of
``libcorr.so``.  PyTorch supplies device memory and the stream.  If the library
has not been built, loading fails with an error; there is no fallback.

Typical use::

    from paper_1711_05075_amd import Correlator
    c = Correlator(A, B, n=64, box=2.5, origin=(-1.25,) * 3)   # A, B: (n, 5) float64 arrays
    scores, peak_val, peak_idx = c.eval(quats)                  # torch CUDA tensors
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# CORR_LIBRARY names another build of the same library (an instrumented one, say)
LIB_PATH = os.environ.get("CORR_LIBRARY") or os.path.join(_PKG, "libcorr.so")

CORR_OK = 0
CORR_EINVAL = -1
CORR_ENOMEM = -2
CORR_EHIP = -3
CORR_EUNSUPPORTED = -4
CORR_DETERMINISTIC = 1
CORR_SC_SCORE = 2
CORR_LIFTED_SCORE = 4
CORR_TUNE_WITH_A = 1
CORR_MAX_SLICES = 16

EXPORTS = ("corr_create", "corr_prepare_a", "corr_eval", "corr_spectrum", "corr_info", "corr_profile",
           "corr_profile_read", "corr_pass_info", "corr_query", "corr_query_noalloc", "corr_set_offsets",
           "corr_eval_slices", "corr_spread_work", "corr_raster_eval", "corr_get_tuning", "corr_set_tuning", "corr_tuning_choices", "corr_autotune",
           "corr_destroy", "corr_last_error",
           "corr_batch_create",
           "corr_batch_eval", "corr_batch_set_graph",
           "corr_batch_info", "corr_batch_profile", "corr_batch_profile_read", "corr_batch_spread_work",
           "corr_batch_autotune", "corr_batch_destroy", "corr_batch_last_error")
STAGES = ("rotate", "bin", "spread_fft_x", "fft_y", "fft_z_spectrum", "fft_z_product", "ifft_y", "ifft_x", "peak",
          "query", "graph", "raster")


class corr_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("box", ctypes.c_double), ("origin", ctypes.c_double * 3),
                ("sigma", ctypes.c_double), ("kb_width", ctypes.c_int32), ("tol", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("batch", ctypes.c_int32), ("sc_offset", ctypes.c_double),
                ("sc_lambda", ctypes.c_double), ("lift_range", ctypes.c_double)]


class corr_info_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("kb_width", ctypes.c_int32),
                ("q_a", ctypes.c_int32), ("q_b", ctypes.c_int32), ("n_a", ctypes.c_int64),
                ("n_b", ctypes.c_int64), ("batch", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64),
                ("beta", ctypes.c_double), ("radius_err_a", ctypes.c_double), ("radius_err_b", ctypes.c_double)]


class corr_pass_t(ctypes.Structure):
    _fields_ = [("rotations", ctypes.c_int32), ("q", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("m", ctypes.c_int32), ("knots", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("live_tiles", ctypes.c_int64), ("live_rows", ctypes.c_int64)]


class corr_slices_out(ctypes.Structure):
    _fields_ = [("scores", ctypes.c_void_p), ("peak_val", ctypes.c_void_p), ("peak_idx", ctypes.c_void_p),
                ("obstacle", ctypes.c_void_p), ("obstacle_count", ctypes.c_void_p), ("threshold", ctypes.c_float)]


class corr_tuning(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("spread_wgs", ctypes.c_int32), ("cols_y", ctypes.c_int32),
                ("cols_z", ctypes.c_int32), ("cols_iy", ctypes.c_int32), ("pairs_ix", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("bin_group", ctypes.c_int32), ("tile_rows", ctypes.c_int32)]


TUNING_FIELDS = tuple(k for k, _ in corr_tuning._fields_)


class CorrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libcorr error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcorr.so and declare its entry points (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libcorr.so is not built (%s); run `python -m paper_1711_05075_amd.build`" % path)
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.corr_create.argtypes = [vp, i64, vp, i64, ctypes.POINTER(corr_grid), vp, ctypes.POINTER(vp)]
    lib.corr_prepare_a.argtypes = [vp]
    lib.corr_eval.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.corr_spectrum.argtypes = [vp, i32, vp, vp]
    lib.corr_info.argtypes = [vp, ctypes.POINTER(corr_info_t)]
    lib.corr_profile.argtypes = [vp, i32]
    lib.corr_profile_read.argtypes = [vp, vp, vp, i32]
    lib.corr_pass_info.argtypes = [vp, ctypes.POINTER(corr_pass_t)]
    lib.corr_spread_work.argtypes = [vp, vp]
    lib.corr_raster_eval.argtypes = [vp, vp, i64, vp]
    lib.corr_query.argtypes = [vp, vp, vp, i64, i32, vp, ctypes.POINTER(ctypes.c_int64)]
    lib.corr_query_noalloc.argtypes = [vp, vp, vp, i64, i32, vp, ctypes.POINTER(ctypes.c_int64)]
    lib.corr_set_offsets.argtypes = [vp, vp, i32]
    lib.corr_eval_slices.argtypes = [vp, vp, i64, ctypes.POINTER(corr_slices_out)]
    lib.corr_get_tuning.argtypes = [vp, ctypes.POINTER(corr_tuning)]
    lib.corr_set_tuning.argtypes = [vp, ctypes.POINTER(corr_tuning)]
    lib.corr_tuning_choices.argtypes = [vp, i32, vp, ctypes.POINTER(i32)]
    lib.corr_autotune.argtypes = [vp, vp, i64, vp, vp, vp, i32, ctypes.c_uint32, ctypes.POINTER(corr_tuning)]
    lib.corr_destroy.argtypes = [vp]
    lib.corr_last_error.argtypes = [vp]
    lib.corr_last_error.restype = ctypes.c_char_p
    for name in ("corr_create", "corr_prepare_a", "corr_eval", "corr_spectrum", "corr_info", "corr_profile",
                 "corr_profile_read", "corr_pass_info", "corr_query", "corr_query_noalloc", "corr_set_offsets",
                 "corr_eval_slices", "corr_spread_work", "corr_raster_eval", "corr_get_tuning", "corr_set_tuning", "corr_tuning_choices", "corr_autotune", "corr_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc, ctx=None):
    if rc != CORR_OK:
        raise CorrError(rc, load_library().corr_last_error(ctx).decode())


def _balls(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 5))
    return a


# ---- thin wrappers with the C names -----------------------------------------

def corr_create(A, B, grid: corr_grid, stream: int = 0) -> ctypes.c_void_p:
    lib = load_library()
    A, B = _balls(A), _balls(B)
    out = ctypes.c_void_p()
    _check(lib.corr_create(A.ctypes.data if len(A) else None, len(A), B.ctypes.data if len(B) else None, len(B),
                           ctypes.byref(grid), ctypes.c_void_p(stream or None), ctypes.byref(out)))
    return out


def corr_prepare_a(ctx):
    _check(load_library().corr_prepare_a(ctx), ctx)


def corr_eval(ctx, quats, scores_ptr, peak_val_ptr, peak_idx_ptr):
    q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
    _check(load_library().corr_eval(ctx, q.ctypes.data if len(q) else None, len(q), scores_ptr or None,
                                    peak_val_ptr or None, peak_idx_ptr or None), ctx)


def corr_spectrum(ctx, which, quat, out_ptr):
    q = np.ascontiguousarray(np.asarray(quat if quat is not None else [1.0, 0, 0, 0], dtype=np.float64))
    _check(load_library().corr_spectrum(ctx, int(which), q.ctypes.data, out_ptr), ctx)


def corr_info(ctx) -> dict:
    info = corr_info_t()
    _check(load_library().corr_info(ctx, ctypes.byref(info)), ctx)
    return {k: getattr(info, k) for k, _ in corr_info_t._fields_}


def corr_profile(ctx, enable):
    _check(load_library().corr_profile(ctx, int(bool(enable))), ctx)


def corr_profile_read(ctx) -> dict:
    """{stage name: (total ms, launches)} since the last read."""
    ms = np.zeros(len(STAGES))
    cnt = np.zeros(len(STAGES), dtype=np.int64)
    _check(load_library().corr_profile_read(ctx, ms.ctypes.data, cnt.ctypes.data, len(STAGES)), ctx)
    return {STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(len(STAGES))}


def corr_pass_info(ctx) -> dict:
    """Occupancy of the last spreading pass (synchronises the stream)."""
    r = corr_pass_t()
    _check(load_library().corr_pass_info(ctx, ctypes.byref(r)), ctx)
    return {k: getattr(r, k) for k, _ in corr_pass_t._fields_}


def corr_raster_eval(ctx, quats, counts_ptr):
    """Voxel-overlap counts of the rasterization baseline into counts_ptr (int32 [n_rot][n][n][n])."""
    q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
    _check(load_library().corr_raster_eval(ctx, q.ctypes.data if len(q) else None, len(q), counts_ptr or None), ctx)


def corr_spread_work(ctx) -> dict:
    """Spreading work since the last read: bytes written, record bytes read, launches."""
    out = np.zeros(3, dtype=np.int64)
    _check(load_library().corr_spread_work(ctx, out.ctypes.data), ctx)
    return {"written_bytes": int(out[0]), "record_bytes": int(out[1]), "launches": int(out[2])}


def corr_query(ctx, quat, t, mode_radius2, out_ptr) -> int:
    """Score of single configurations (t: [n][3] host); returns the number of modes summed."""
    q = np.ascontiguousarray(np.asarray(quat, dtype=np.float64).reshape(4))
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(-1, 3))
    nm = ctypes.c_int64()
    _check(load_library().corr_query(ctx, q.ctypes.data, t.ctypes.data if len(t) else None, len(t), int(mode_radius2),
                                     out_ptr or None, ctypes.byref(nm)), ctx)
    return nm.value


def corr_query_noalloc(ctx, quat, t, mode_radius2, out_ptr) -> int:
    """corr_query without allocation (static per-device scratch); returns the number of modes summed."""
    q = np.ascontiguousarray(np.asarray(quat, dtype=np.float64).reshape(4))
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(-1, 3))
    nm = ctypes.c_int64()
    _check(load_library().corr_query_noalloc(ctx, q.ctypes.data, t.ctypes.data if len(t) else None, len(t),
                                             int(mode_radius2), out_ptr or None, ctypes.byref(nm)), ctx)
    return nm.value


def corr_set_offsets(ctx, offsets):
    d = np.ascontiguousarray(np.asarray(offsets, dtype=np.float64).reshape(-1))
    _check(load_library().corr_set_offsets(ctx, d.ctypes.data if len(d) else None, len(d)), ctx)


def corr_eval_slices(ctx, quats, scores_ptr=None, peak_val_ptr=None, peak_idx_ptr=None, obstacle_ptr=None,
                     count_ptr=None, threshold=0.0):
    q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
    o = corr_slices_out(scores_ptr or None, peak_val_ptr or None, peak_idx_ptr or None, obstacle_ptr or None,
                        count_ptr or None, float(threshold))
    _check(load_library().corr_eval_slices(ctx, q.ctypes.data if len(q) else None, len(q), ctypes.byref(o)), ctx)


def corr_get_tuning(ctx) -> dict:
    t = corr_tuning()
    _check(load_library().corr_get_tuning(ctx, ctypes.byref(t)), ctx)
    return {k: getattr(t, k) for k in TUNING_FIELDS}


def corr_set_tuning(ctx, **fields):
    """Change the named fields of the context's tuning (the others stay)."""
    t = corr_tuning()
    _check(load_library().corr_get_tuning(ctx, ctypes.byref(t)), ctx)
    for k, v in fields.items():
        if k not in TUNING_FIELDS:
            raise KeyError("unknown tuning field %r" % k)
        setattr(t, k, int(v))
    _check(load_library().corr_set_tuning(ctx, ctypes.byref(t)), ctx)


def corr_tuning_choices(ctx, pass_id) -> list:
    out = (ctypes.c_int32 * 3)()
    cnt = ctypes.c_int32()
    _check(load_library().corr_tuning_choices(ctx, int(pass_id), out, ctypes.byref(cnt)), ctx)
    return [out[i] for i in range(cnt.value)]


def corr_autotune(ctx, quats, scores_ptr, peak_val_ptr, peak_idx_ptr, reps=3, with_a=False) -> dict:
    """with_a: time corr_prepare_a + corr_eval as one unit (CORR_TUNE_WITH_A)."""
    q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
    t = corr_tuning()
    _check(load_library().corr_autotune(ctx, q.ctypes.data if len(q) else None, len(q), scores_ptr or None,
                                        peak_val_ptr or None, peak_idx_ptr or None, int(reps),
                                        CORR_TUNE_WITH_A if with_a else 0, ctypes.byref(t)), ctx)
    return {k: getattr(t, k) for k in TUNING_FIELDS}


def corr_destroy(ctx):
    load_library().corr_destroy(ctx)


def corr_last_error(ctx=None) -> str:
    return load_library().corr_last_error(ctx).decode()


def make_grid(n, box, origin, sigma=2.0, kb_width=8, tol=1e-6, flags=0, batch=0, sc=None, lift=None) -> corr_grid:
    """sc = (offset, lambda) scores shape complementarity (sets CORR_SC_SCORE);
    lift = range of slice heights scores the lifted correlation (sets CORR_LIFTED_SCORE)."""
    g = corr_grid()
    g.n, g.box, g.sigma, g.kb_width, g.tol, g.flags, g.batch = int(n), float(box), float(sigma), int(kb_width), \
        float(tol), int(flags), int(batch)
    if sc is not None:
        g.flags |= CORR_SC_SCORE
        g.sc_offset, g.sc_lambda = float(sc[0]), float(sc[1])
    if lift is not None:
        g.flags |= CORR_LIFTED_SCORE
        g.lift_range = float(lift)
    for d in range(3):
        g.origin[d] = float(origin[d])
    return g


# ---- convenience object over torch device memory ------------------------------

class Correlator:
    """One (A, B) pair on one translation grid; outputs are torch CUDA tensors."""

    def __init__(self, A, B, n, box, origin, sigma=2.0, kb_width=8, tol=1e-6, flags=0, batch=0, device=None,
                 sc=None, lift=None):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.grid = make_grid(n, box, origin, sigma, kb_width, tol, flags, batch, sc, lift)
            self.ctx = corr_create(A, B, self.grid, self.stream.cuda_stream)
        self.n = int(n)
        self.info = corr_info(self.ctx)

    def prepare_a(self):
        corr_prepare_a(self.ctx)

    def eval(self, quats, scores=True, peaks=True, out=None):
        torch = self.torch
        q = np.asarray(quats, dtype=np.float64).reshape(-1, 4)
        r = len(q)
        n = self.n
        s = None
        if scores:
            s = out if out is not None else torch.empty((r, n, n, n), dtype=torch.float32, device=self.device)
        pv = torch.empty(r, dtype=torch.float32, device=self.device) if peaks else None
        pi = torch.empty(r, dtype=torch.int64, device=self.device) if peaks else None
        with torch.cuda.device(self.device):
            corr_eval(self.ctx, q, s.data_ptr() if s is not None else None,
                      pv.data_ptr() if pv is not None else None, pi.data_ptr() if pi is not None else None)
        return s, pv, pi

    def set_offsets(self, offsets):
        """Radius offsets of A's balls for eval_slices (empty: no slices)."""
        with self.torch.cuda.device(self.device):
            corr_set_offsets(self.ctx, offsets)
        self.n_slices = max(1, len(np.atleast_1d(offsets)))

    def eval_slices(self, quats, scores=True, peaks=True, obstacle=False, count=False, threshold=0.0):
        """Outputs of corr_eval_slices as a dict of tensors shaped [slices][rotations]...;
        the obstacle masks are int32 [slices][rotations][n^3 / 32] (the uint32 bits)."""
        torch = self.torch
        q = np.asarray(quats, dtype=np.float64).reshape(-1, 4)
        S, r, n = getattr(self, "n_slices", 1), len(q), self.n
        dev = self.device
        out = {}
        if scores:
            out["scores"] = torch.empty((S, r, n, n, n), dtype=torch.float32, device=dev)
        if peaks:
            out["peak_val"] = torch.empty((S, r), dtype=torch.float32, device=dev)
            out["peak_idx"] = torch.empty((S, r), dtype=torch.int64, device=dev)
        if obstacle:
            out["obstacle"] = torch.empty((S, r, n ** 3 // 32), dtype=torch.int32, device=dev)
        if count:
            out["obstacle_count"] = torch.empty((S, r), dtype=torch.int64, device=dev)
        ptr = {k: v.data_ptr() for k, v in out.items()}
        with torch.cuda.device(dev):
            corr_eval_slices(self.ctx, q, ptr.get("scores"), ptr.get("peak_val"), ptr.get("peak_idx"),
                             ptr.get("obstacle"), ptr.get("obstacle_count"), threshold)
        return out

    def pass_info(self):
        return corr_pass_info(self.ctx)

    def tuning(self):
        return corr_get_tuning(self.ctx)

    def set_tuning(self, **fields):
        with self.torch.cuda.device(self.device):
            corr_set_tuning(self.ctx, **fields)

    def autotune(self, quats, scores=True, peaks=True, reps=3, with_a=False):
        """Run the autotuner on these rotations (with_a: timing A's spectrum with
        each evaluation); returns the tuning kept."""
        torch = self.torch
        q = np.asarray(quats, dtype=np.float64).reshape(-1, 4)
        r, n = len(q), self.n
        s = torch.empty((r, n, n, n), dtype=torch.float32, device=self.device) if scores else None
        pv = torch.empty(r, dtype=torch.float32, device=self.device) if peaks else None
        pi = torch.empty(r, dtype=torch.int64, device=self.device) if peaks else None
        with torch.cuda.device(self.device):
            return corr_autotune(self.ctx, q, s.data_ptr() if s is not None else None,
                                 pv.data_ptr() if pv is not None else None, pi.data_ptr() if pi is not None else None,
                                 reps, with_a)

    def query(self, quat, t, mode_radius2):
        """Score at translations t ([n][3]) over the modes |m|^2 <= mode_radius2;
        returns (scores tensor [n], modes summed)."""
        torch = self.torch
        t = np.asarray(t, dtype=np.float64).reshape(-1, 3)
        out = torch.empty(len(t), dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            nm = corr_query(self.ctx, quat, t, mode_radius2, out.data_ptr() if len(t) else None)
        return out, nm

    def raster(self, quats):
        """Counts of the rasterization baseline, int32 [rotations][n][n][n]."""
        torch = self.torch
        q = np.asarray(quats, dtype=np.float64).reshape(-1, 4)
        out = torch.empty((len(q), self.n, self.n, self.n), dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            corr_raster_eval(self.ctx, q, out.data_ptr())
        return out

    def spectrum(self, which, quat=None):
        torch = self.torch
        n = self.n
        out = torch.empty((n, n, n // 2, 2), dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            corr_spectrum(self.ctx, which, quat, out.data_ptr())
        return out

    def close(self):
        if getattr(self, "ctx", None):
            corr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- proposal network (include/prop.h) ----------------------------------------

PROP_EXPORTS = ("prop_create", "prop_descriptor", "prop_features", "prop_train", "prop_predict", "prop_rank",
                "prop_gradient", "prop_get_params", "prop_set_params", "prop_destroy", "prop_last_error")
PROP_IN, PROP_HIDDEN, PROP_BINS = 160, 256, 64
PROP_NPARAMS = 160 * 256 + 256 + 2 * (256 * 256 + 256) + 256 + 1


def _prop_lib():
    lib = load_library()
    if not getattr(lib, "_prop_declared", False):
        vp, i64, i32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
        lib.prop_create.argtypes = [i32, ctypes.c_uint64, vp, ctypes.POINTER(vp)]
        lib.prop_descriptor.argtypes = [vp, vp, i64, vp]
        lib.prop_features.argtypes = [vp, vp, i64, vp, vp, vp]
        lib.prop_train.argtypes = [vp, vp, vp, i64, i32, f32, vp]
        lib.prop_predict.argtypes = [vp, vp, i64, vp]
        lib.prop_rank.argtypes = [vp, vp, i64, i32, vp]
        lib.prop_gradient.argtypes = [vp, vp, vp, i64, vp]
        lib.prop_get_params.argtypes = [vp, vp]
        lib.prop_set_params.argtypes = [vp, vp]
        lib.prop_destroy.argtypes = [vp]
        lib.prop_last_error.argtypes = [vp]
        lib.prop_last_error.restype = ctypes.c_char_p
        for name in PROP_EXPORTS[:-1]:
            getattr(lib, name).restype = ctypes.c_int
        lib._prop_declared = True
    return lib


def _pcheck(rc, ctx=None):
    if rc != CORR_OK:
        raise CorrError(rc, _prop_lib().prop_last_error(ctx).decode())


def prop_create(batch, seed, stream=0):
    out = ctypes.c_void_p()
    _pcheck(_prop_lib().prop_create(int(batch), int(seed), ctypes.c_void_p(stream or None), ctypes.byref(out)))
    return out


def prop_descriptor(ctx, balls, desc_ptr):
    b = _balls(balls)
    _pcheck(_prop_lib().prop_descriptor(ctx, b.ctypes.data, len(b), desc_ptr), ctx)


def prop_features(ctx, quats, desc_a_ptr, desc_b_ptr, x_ptr):
    q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
    _pcheck(_prop_lib().prop_features(ctx, q.ctypes.data, len(q), desc_a_ptr, desc_b_ptr, x_ptr), ctx)


def prop_train(ctx, x_ptr, y_ptr, n, epochs, lr):
    losses = np.zeros(max(int(epochs), 1), dtype=np.float32)
    _pcheck(_prop_lib().prop_train(ctx, x_ptr, y_ptr, int(n), int(epochs), float(lr), losses.ctypes.data), ctx)
    return losses[:epochs]


def prop_predict(ctx, x_ptr, n, y_ptr):
    _pcheck(_prop_lib().prop_predict(ctx, x_ptr, int(n), y_ptr), ctx)


def prop_rank(ctx, x_ptr, n, k, idx_ptr):
    _pcheck(_prop_lib().prop_rank(ctx, x_ptr, int(n), int(k), idx_ptr), ctx)


def prop_gradient(ctx, x_ptr, y_ptr, n) -> np.ndarray:
    g = np.zeros(PROP_NPARAMS, dtype=np.float32)
    _pcheck(_prop_lib().prop_gradient(ctx, x_ptr, y_ptr, int(n), g.ctypes.data), ctx)
    return g


def prop_get_params(ctx) -> np.ndarray:
    p = np.zeros(PROP_NPARAMS, dtype=np.float32)
    _pcheck(_prop_lib().prop_get_params(ctx, p.ctypes.data), ctx)
    return p


def prop_set_params(ctx, params):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
    if p.size != PROP_NPARAMS:
        raise ValueError("need %d parameters" % PROP_NPARAMS)
    _pcheck(_prop_lib().prop_set_params(ctx, p.ctypes.data), ctx)


def prop_destroy(ctx):
    _prop_lib().prop_destroy(ctx)


def prop_last_error(ctx=None) -> str:
    return _prop_lib().prop_last_error(ctx).decode()


def unpack_params(flat):
    """Split a flat parameter vector into [(W (in, out), b)] for the four layers."""
    flat = np.asarray(flat)
    out, o = [], 0
    for fi, fo in ((160, 256), (256, 256), (256, 256), (256, 1)):
        W = flat[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        b = flat[o:o + fo]
        o += fo
        out.append((W, b))
    return out


class Proposer:
    """Proposal network on torch device memory."""

    def __init__(self, batch=1024, seed=0, device=None):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.ctx = prop_create(batch, seed, self.stream.cuda_stream)

    def descriptor(self, balls):
        d = self.torch.empty(PROP_BINS, dtype=self.torch.float32, device=self.device)
        prop_descriptor(self.ctx, balls, d.data_ptr())
        return d

    def features(self, quats, desc_a, desc_b):
        q = np.asarray(quats, dtype=np.float64).reshape(-1, 4)
        X = self.torch.empty((len(q), PROP_IN), dtype=self.torch.float32, device=self.device)
        prop_features(self.ctx, q, desc_a.data_ptr(), desc_b.data_ptr(), X.data_ptr())
        return X

    def train(self, X, y, epochs, lr):
        return prop_train(self.ctx, X.data_ptr(), y.data_ptr(), X.shape[0], epochs, lr)

    def predict(self, X):
        y = self.torch.empty(X.shape[0], dtype=self.torch.float32, device=self.device)
        prop_predict(self.ctx, X.data_ptr(), X.shape[0], y.data_ptr())
        return y

    def rank(self, X, k):
        idx = self.torch.empty(k, dtype=self.torch.int64, device=self.device)
        prop_rank(self.ctx, X.data_ptr(), X.shape[0], k, idx.data_ptr())
        return idx

    def gradient(self, X, y):
        return prop_gradient(self.ctx, X.data_ptr(), y.data_ptr(), X.shape[0])

    def get_params(self):
        return prop_get_params(self.ctx)

    def set_params(self, p):
        prop_set_params(self.ctx, p)

    def close(self):
        if getattr(self, "ctx", None):
            prop_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- uneven batches (corr_batch_*) ---------------------------------------------

BATCH_EXPORTS = ("corr_batch_create", "corr_batch_eval", "corr_batch_set_graph", "corr_batch_info",
                 "corr_batch_profile", "corr_batch_profile_read", "corr_batch_spread_work", "corr_batch_autotune",
                 "corr_batch_destroy", "corr_batch_last_error")


class corr_pair(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("nA", ctypes.c_int64), ("B", ctypes.c_void_p), ("nB", ctypes.c_int64),
                ("grid", corr_grid)]


def _batch_lib():
    lib = load_library()
    if not getattr(lib, "_batch_declared", False):
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.corr_batch_create.argtypes = [vp, i32, i32, vp, ctypes.POINTER(vp)]
        lib.corr_batch_eval.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        lib.corr_batch_set_graph.argtypes = [vp, i32]
        lib.corr_batch_info.argtypes = [vp, i32, ctypes.POINTER(corr_info_t)]
        lib.corr_batch_profile.argtypes = [vp, i32]
        lib.corr_batch_profile_read.argtypes = [vp, vp, vp, i32]
        lib.corr_batch_spread_work.argtypes = [vp, vp]
        lib.corr_batch_autotune.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, vp]
        lib.corr_batch_destroy.argtypes = [vp]
        lib.corr_batch_last_error.argtypes = [vp]
        lib.corr_batch_last_error.restype = ctypes.c_char_p
        for name in BATCH_EXPORTS[:-1]:
            getattr(lib, name).restype = ctypes.c_int
        lib._batch_declared = True
    return lib


def _bcheck(rc, b=None):
    if rc != CORR_OK:
        raise CorrError(rc, _batch_lib().corr_batch_last_error(b).decode())


def corr_batch_create(pairs, slots=0, stream=0):
    """pairs: list of (A, B, grid) with grid a corr_grid."""
    keep = []
    arr = (corr_pair * len(pairs))()
    for i, (A, B, g) in enumerate(pairs):
        A, B = _balls(A), _balls(B)
        keep += [A, B]
        arr[i].A = A.ctypes.data if len(A) else None
        arr[i].nA = len(A)
        arr[i].B = B.ctypes.data if len(B) else None
        arr[i].nB = len(B)
        arr[i].grid = g
    out = ctypes.c_void_p()
    _bcheck(_batch_lib().corr_batch_create(arr, len(pairs), int(slots), ctypes.c_void_p(stream or None),
                                           ctypes.byref(out)))
    return out


def corr_batch_eval(b, quats, rot_offsets, scores_ptr, score_offsets, peak_val_ptr, peak_idx_ptr):
    q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
    ro = np.ascontiguousarray(np.asarray(rot_offsets, dtype=np.int64))
    so = None if score_offsets is None else np.ascontiguousarray(np.asarray(score_offsets, dtype=np.int64))
    _bcheck(_batch_lib().corr_batch_eval(b, q.ctypes.data if len(q) else None, ro.ctypes.data, scores_ptr or None,
                                         so.ctypes.data if so is not None else None, peak_val_ptr or None,
                                         peak_idx_ptr or None), b)


def corr_batch_set_graph(b, enable):
    _bcheck(_batch_lib().corr_batch_set_graph(b, int(bool(enable))), b)


def corr_batch_info(b, pair) -> dict:
    info = corr_info_t()
    _bcheck(_batch_lib().corr_batch_info(b, int(pair), ctypes.byref(info)), b)
    return {k: getattr(info, k) for k, _ in corr_info_t._fields_}


def corr_batch_profile(b, enable):
    _bcheck(_batch_lib().corr_batch_profile(b, int(bool(enable))), b)


def corr_batch_profile_read(b) -> dict:
    """Per stage name: (summed ms, launches) since the last read, over every pair."""
    n = len(STAGES)
    ms = np.zeros(n)
    cnt = np.zeros(n, dtype=np.int64)
    _bcheck(_batch_lib().corr_batch_profile_read(b, ms.ctypes.data, cnt.ctypes.data, n), b)
    return {STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}


def corr_batch_spread_work(b) -> dict:
    out = np.zeros(3, dtype=np.int64)
    _bcheck(_batch_lib().corr_batch_spread_work(b, out.ctypes.data), b)
    return {"written_bytes": int(out[0]), "record_bytes": int(out[1]), "launches": int(out[2])}


def corr_batch_destroy(b):
    _batch_lib().corr_batch_destroy(b)


class Batch:
    """Uneven batch of pairs on torch device memory; peaks for every rotation and,
    optionally, the packed scores of every pair."""

    def __init__(self, pairs, slots=0, device=None, kb_width=8, tol=1e-6):
        """pairs: list of (A, B, n, box, origin); kb_width and tol (radius expansion):
        the same for every pair."""
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        self.ns = [int(p[2]) for p in pairs]
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.b = corr_batch_create([(A, B, make_grid(n, box, origin, kb_width=kb_width, tol=tol))
                                        for A, B, n, box, origin in pairs], slots, self.stream.cuda_stream)

    def set_graph(self, enable):
        corr_batch_set_graph(self.b, enable)

    def eval(self, quats_per_pair, scores=False, out=None):
        """out = (packed scores or None, peak_val, peak_idx) reuses caller tensors
        (a graph is replayed only while the output pointers stay the same)."""
        torch = self.torch
        counts = [len(q) for q in quats_per_pair]
        offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        q = np.concatenate([np.asarray(x, dtype=np.float64).reshape(-1, 4) for x in quats_per_pair])
        total = sum(c * n ** 3 for c, n in zip(counts, self.ns))
        if out is not None:
            s, pv, pi = out
            if pv.numel() != int(offs[-1]) or pi.numel() != int(offs[-1]) or (s is not None and s.numel() != total):
                raise ValueError("output tensors do not match the rotations")
            scores = s is not None
        else:
            pv = torch.empty(int(offs[-1]), dtype=torch.float32, device=self.device)
            pi = torch.empty(int(offs[-1]), dtype=torch.int64, device=self.device)
            s = torch.empty(total, dtype=torch.float32, device=self.device) if scores else None
        with torch.cuda.device(self.device):
            corr_batch_eval(self.b, q, offs, s.data_ptr() if s is not None else None, None, pv.data_ptr(),
                            pi.data_ptr())
        out = None
        if scores:
            out, o = [], 0
            for c, n in zip(counts, self.ns):
                out.append(s[o:o + c * n ** 3].view(c, n, n, n))
                o += c * n ** 3
        return out, pv, pi, offs

    def autotune(self, quats_per_pair, out, reps=2):
        """Run corr_batch_autotune on these rotations with the caller's output
        tensors out = (packed scores or None, peak_val, peak_idx); returns the
        kept choice {spread_wgs, rank of each column pass's width, rank of the
        bin group, rank of the tile height}, the ranks those of the largest
        grid (each grid size of the batch is tuned on its own)."""
        counts = [len(q) for q in quats_per_pair]
        offs = np.ascontiguousarray(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64))
        q = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64).reshape(-1, 4)
                                                 for x in quats_per_pair]))
        s, pv, pi = out
        res = np.zeros(7, dtype=np.int32)
        with self.torch.cuda.device(self.device):
            _bcheck(_batch_lib().corr_batch_autotune(self.b, q.ctypes.data, offs.ctypes.data,
                                                     s.data_ptr() if s is not None else None, None, pv.data_ptr(),
                                                     pi.data_ptr(), int(reps), res.ctypes.data), self.b)
        return {"spread_wgs": int(res[0]), "rank_cols_y": int(res[1]), "rank_cols_z": int(res[2]),
                "rank_cols_iy": int(res[3]), "rank_pairs_ix": int(res[4]), "rank_bin_group": int(res[5]),
                "rank_tile_rows": int(res[6])}

    def info(self, pair):
        return corr_batch_info(self.b, pair)

    def close(self):
        if getattr(self, "b", None):
            corr_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
