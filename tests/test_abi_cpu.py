"""C-ABI checks that need no GPU: every declared symbol is exported, and invalid
arguments are rejected with CORR_EINVAL / CORR_EUNSUPPORTED before any device work."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1711_05075_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*|void)\s+\**\s*(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pkg.LIB_PATH):
        pkg.build.build_library()
    return pkg.load_library()


def test_header_declares_the_entry_points():
    names = _declared("corr.h")
    for n in pkg.EXPORTS:
        assert n in names
    assert set(names) <= set(pkg.EXPORTS)
    pnames = _declared("prop.h")
    assert set(pnames) == set(pkg.PROP_EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", pkg.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(\w+)$", out, flags=re.M))
    for header in ("corr.h", "prop.h"):
        for name in _declared(header):
            assert name in exported, name
            assert hasattr(lib, name)


def _grid(**kw):
    d = dict(n=32, box=4.0, origin=(-2, -2, -2))
    d.update(kw)
    return pkg.make_grid(**d)


def _create(A, B, g):
    lib = pkg.load_library()
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    out = ctypes.c_void_p()
    rc = lib.corr_create(A.ctypes.data if A.size else None, len(A), B.ctypes.data if B.size else None, len(B),
                         ctypes.byref(g), None, ctypes.byref(out))
    return rc, out


GOOD = np.array([[0.0, 0.0, 0.0, 0.05, 1.0], [0.1, 0.0, 0.0, 0.04, 1.0]])


@pytest.mark.parametrize("bad,code", [
    (dict(n=48), pkg.CORR_EUNSUPPORTED),
    (dict(n=8), pkg.CORR_EUNSUPPORTED),
    (dict(box=0.0), pkg.CORR_EINVAL),
    (dict(box=float("nan")), pkg.CORR_EINVAL),
    (dict(origin=(0, float("inf"), 0)), pkg.CORR_EINVAL),
    (dict(sigma=1.5), pkg.CORR_EUNSUPPORTED),
    (dict(kb_width=7), pkg.CORR_EUNSUPPORTED),
    (dict(kb_width=4), pkg.CORR_EUNSUPPORTED),
    (dict(kb_width=14), pkg.CORR_EUNSUPPORTED),
    (dict(tol=-1.0), pkg.CORR_EINVAL),
    (dict(tol=2.0), pkg.CORR_EINVAL),
    (dict(flags=8), pkg.CORR_EINVAL),
    (dict(batch=-1), pkg.CORR_EINVAL),
    (dict(batch=1000), pkg.CORR_EINVAL),
    (dict(sc=(-0.01, 2.0)), pkg.CORR_EINVAL),
    (dict(sc=(0.01, -2.0)), pkg.CORR_EINVAL),
    (dict(sc=(float("nan"), 2.0)), pkg.CORR_EINVAL),
    (dict(sc=(0.01, float("inf"))), pkg.CORR_EINVAL),
    (dict(lift=-0.01), pkg.CORR_EINVAL),
    (dict(lift=float("nan")), pkg.CORR_EINVAL),
    (dict(lift=0.01, sc=(0.01, 1.0)), pkg.CORR_EINVAL),
])
def test_create_rejects_bad_grids(lib, bad, code):
    rc, out = _create(GOOD, GOOD, _grid(**bad))
    assert rc == code
    assert not out.value
    assert len(pkg.corr_last_error(None)) > 0


@pytest.mark.parametrize("col,val", [(3, 0.0), (3, -0.1), (3, float("nan")), (0, float("inf")), (4, float("nan"))])
def test_create_rejects_bad_balls(lib, col, val):
    B = GOOD.copy()
    B[1, col] = val
    rc, out = _create(GOOD, B, _grid())
    assert rc == pkg.CORR_EINVAL
    assert "B[1]" in pkg.corr_last_error(None)


def test_create_rejects_null_arguments(lib):
    out = ctypes.c_void_p()
    g = _grid()
    assert lib.corr_create(None, 3, None, 0, ctypes.byref(g), None, ctypes.byref(out)) == pkg.CORR_EINVAL
    A = np.ascontiguousarray(GOOD)
    assert lib.corr_create(A.ctypes.data, 2, A.ctypes.data, 2, None, None, ctypes.byref(out)) == pkg.CORR_EINVAL
    assert lib.corr_create(A.ctypes.data, 2, A.ctypes.data, 2, ctypes.byref(g), None, None) == pkg.CORR_EINVAL
    assert lib.corr_create(A.ctypes.data, -1, A.ctypes.data, 2, ctypes.byref(g), None, ctypes.byref(out)) == pkg.CORR_EINVAL


def test_null_context_calls_fail_cleanly(lib):
    assert lib.corr_eval(None, None, 0, None, None, None) == pkg.CORR_EINVAL
    assert lib.corr_query(None, None, None, 0, 0, None, None) == pkg.CORR_EINVAL
    assert lib.corr_set_offsets(None, None, 0) == pkg.CORR_EINVAL
    assert lib.corr_eval_slices(None, None, 0, None) == pkg.CORR_EINVAL
    assert lib.corr_prepare_a(None) == pkg.CORR_EINVAL
    assert lib.corr_spectrum(None, 0, None, None) == pkg.CORR_EINVAL
    assert lib.corr_info(None, None) == pkg.CORR_EINVAL
    assert lib.corr_destroy(None) == pkg.CORR_OK
    assert "NULL" in pkg.corr_last_error(None)
    t = pkg.corr_tuning()
    cnt = ctypes.c_int32()
    out3 = (ctypes.c_int32 * 3)()
    assert lib.corr_get_tuning(None, ctypes.byref(t)) == pkg.CORR_EINVAL
    assert lib.corr_set_tuning(None, ctypes.byref(t)) == pkg.CORR_EINVAL
    assert lib.corr_tuning_choices(None, 0, out3, ctypes.byref(cnt)) == pkg.CORR_EINVAL
    assert lib.corr_autotune(None, None, 1, None, None, None, 3, 0, None) == pkg.CORR_EINVAL
    assert pkg._batch_lib().corr_batch_set_graph(None, 1) == pkg.CORR_EINVAL


def test_prop_rejects_bad_arguments(lib):
    plib = pkg._prop_lib()
    out = ctypes.c_void_p()
    for batch in (0, 32, 100, 16384):
        assert plib.prop_create(batch, 1, None, ctypes.byref(out)) == pkg.CORR_EINVAL
        assert not out.value
    assert plib.prop_create(64, 1, None, None) == pkg.CORR_EINVAL
    assert plib.prop_train(None, None, None, 0, 1, 0.01, None) == pkg.CORR_EINVAL
    assert plib.prop_rank(None, None, 0, 1, None) == pkg.CORR_EINVAL
    assert plib.prop_destroy(None) == pkg.CORR_OK
    assert len(pkg.prop_last_error(None)) > 0


def test_unpack_params_layout():
    flat = np.arange(pkg.PROP_NPARAMS, dtype=np.float64)
    layers = pkg.unpack_params(flat)
    assert [W.shape for W, _ in layers] == [(160, 256), (256, 256), (256, 256), (256, 1)]
    assert layers[0][1][0] == 160 * 256 and layers[3][1][0] == pkg.PROP_NPARAMS - 1


def test_batch_rejects_bad_arguments(lib):
    blib = pkg._batch_lib()
    out = ctypes.c_void_p()
    assert blib.corr_batch_create(None, 0, 0, None, ctypes.byref(out)) == pkg.CORR_EINVAL
    A = np.ascontiguousarray(GOOD)
    bad = pkg.make_grid(48, 2.0, (-1, -1, -1))
    arr = (pkg.corr_pair * 2)()
    for i, g in enumerate((pkg.make_grid(32, 2.0, (-1, -1, -1)), bad)):
        arr[i].A = A.ctypes.data
        arr[i].nA = 2
        arr[i].B = A.ctypes.data
        arr[i].nB = 2
        arr[i].grid = g
    # pair 1 has an unsupported grid: rejected before any device work, and named
    arr[0].grid = bad
    assert blib.corr_batch_create(arr, 2, 0, None, ctypes.byref(out)) == pkg.CORR_EUNSUPPORTED
    assert "pair 0" in pkg._batch_lib().corr_batch_last_error(None).decode()
    assert blib.corr_batch_eval(None, None, None, None, None, None, None) == pkg.CORR_EINVAL
    assert blib.corr_batch_destroy(None) == pkg.CORR_OK


def test_lift_range_needs_its_flag(lib):
    g = _grid()
    g.lift_range = 0.01
    rc, out = _create(GOOD, GOOD, g)
    assert rc == pkg.CORR_EINVAL and not out.value


def test_complementarity_parameters_need_their_flag(lib):
    g = _grid()
    g.sc_offset = 0.01
    rc, out = _create(GOOD, GOOD, g)
    assert rc == pkg.CORR_EINVAL and not out.value
    g = _grid()
    g.sc_lambda = 1.0
    rc, out = _create(GOOD, GOOD, g)
    assert rc == pkg.CORR_EINVAL and not out.value


def test_slices_output_struct_matches_the_header():
    # the binding's mirror of corr_slices_out: five pointers, then the float threshold
    import ctypes as ct
    assert [f for f, _ in pkg.corr_slices_out._fields_] == ["scores", "peak_val", "peak_idx", "obstacle",
                                                             "obstacle_count", "threshold"]
    assert ct.sizeof(pkg.corr_slices_out) == 48
    assert pkg.corr_slices_out.threshold.offset == 40
    with open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "corr.h")) as f:
        h = f.read()
    body = h[h.index("typedef struct {\n    float* scores;"):h.index("} corr_slices_out;")]
    fields = re.findall(r"^\s*(?:float|int64_t|uint32_t)\*?\s+(\w+);", body, flags=re.M)
    assert fields == [f for f, _ in pkg.corr_slices_out._fields_]
    assert "#define CORR_MAX_SLICES 16" in h and pkg.CORR_MAX_SLICES == 16
