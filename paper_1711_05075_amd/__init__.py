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
LIB_PATH = os.path.join(_PKG, "libcorr.so")

CORR_OK = 0
CORR_EINVAL = -1
CORR_ENOMEM = -2
CORR_EHIP = -3
CORR_EUNSUPPORTED = -4
CORR_DETERMINISTIC = 1

EXPORTS = ("corr_create", "corr_prepare_a", "corr_eval", "corr_spectrum", "corr_info", "corr_profile",
           "corr_profile_read", "corr_destroy", "corr_last_error")
STAGES = ("rotate", "bin", "spread_fft_x", "fft_y", "fft_z_spectrum", "fft_z_product", "ifft_y", "ifft_x", "peak")


class corr_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("box", ctypes.c_double), ("origin", ctypes.c_double * 3),
                ("sigma", ctypes.c_double), ("kb_width", ctypes.c_int32), ("tol", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("batch", ctypes.c_int32)]


class corr_info_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("kb_width", ctypes.c_int32),
                ("q_a", ctypes.c_int32), ("q_b", ctypes.c_int32), ("n_a", ctypes.c_int64),
                ("n_b", ctypes.c_int64), ("batch", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64),
                ("beta", ctypes.c_double), ("radius_err_a", ctypes.c_double), ("radius_err_b", ctypes.c_double)]


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
    lib.corr_destroy.argtypes = [vp]
    lib.corr_last_error.argtypes = [vp]
    lib.corr_last_error.restype = ctypes.c_char_p
    for name in ("corr_create", "corr_prepare_a", "corr_eval", "corr_spectrum", "corr_info", "corr_profile",
                 "corr_profile_read", "corr_destroy"):
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


def corr_destroy(ctx):
    load_library().corr_destroy(ctx)


def corr_last_error(ctx=None) -> str:
    return load_library().corr_last_error(ctx).decode()


def make_grid(n, box, origin, sigma=2.0, kb_width=8, tol=1e-6, flags=0, batch=0) -> corr_grid:
    g = corr_grid()
    g.n, g.box, g.sigma, g.kb_width, g.tol, g.flags, g.batch = int(n), float(box), float(sigma), int(kb_width), \
        float(tol), int(flags), int(batch)
    for d in range(3):
        g.origin[d] = float(origin[d])
    return g


# ---- convenience object over torch device memory ------------------------------

class Correlator:
    """One (A, B) pair on one translation grid; outputs are torch CUDA tensors."""

    def __init__(self, A, B, n, box, origin, sigma=2.0, kb_width=8, tol=1e-6, flags=0, batch=0, device=None):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.grid = make_grid(n, box, origin, sigma, kb_width, tol, flags, batch)
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
