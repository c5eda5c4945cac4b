"""corr_query_noalloc, the variant of corr_query for callers that cannot
allocate: through the C ABI, against corr_query on the same inputs, on two
calls in a row (the second smaller, on another context), and the refusal of a
request beyond its static scratch.

Both entry points run the same kernels over the same mode list, launch plan
and summation order, so their results must agree bit for bit; the stated
1e-4 relative tolerance of the path is checked as well, and the oracle's
truncated sum pins the first call."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_05075_amd as p
    p.load_library()
    return p


def _both(pkg, c, q, t, r2):
    """corr_query and corr_query_noalloc on the same inputs, via the C ABI."""
    a = torch.empty(len(t), dtype=torch.float32, device="cuda")
    b = torch.full((len(t),), float("nan"), dtype=torch.float32, device="cuda")
    with torch.cuda.device(c.device):
        na = pkg.corr_query(c.ctx, q, t, r2, a.data_ptr())
        nb = pkg.corr_query_noalloc(c.ctx, q, t, r2, b.data_ptr())
    torch.cuda.synchronize()
    assert na == nb
    return a.double().cpu().numpy(), b.double().cpu().numpy(), nb


def test_noalloc_query_equals_query_on_two_calls(pkg):
    # first call: 600 + 450 balls at n = 64, 2048 translations, |m|^2 <= 400
    A = synth.mixture_balls(600, 1700)
    B = synth.mixture_balls(450, 2700)
    g = synth.grid_for(A, B, 64)
    q = synth.random_quaternions(1, 3700)[0]
    t = np.random.default_rng(7).uniform(-0.4, 0.4, (2048, 3))
    _say("case: no-alloc query, 600+450 balls, n=64, 2048 translations, r2=400")
    c1 = pkg.Correlator(A, B, g.n, g.box, g.origin)
    ref, got, nm = _both(pkg, c1, q, t, 400)
    e = np.abs(got - ref).max() / np.abs(ref).max()
    _say("  modes %d: max |noalloc - query| / max |query| = %.3g" % (nm, e))
    assert e <= TOL
    assert np.array_equal(got, ref)
    FA = oracle.o2_spectrum(A, np.eye(3), g.n, g.box)
    FB = oracle.o2_spectrum(B, oracle.quat_to_rot(q), g.n, g.box)
    orc = oracle.o2_query(FA, FB, g.box, t, 400)
    full = np.abs(oracle.o2_query(FA, FB, g.box, t[:64], 3 * (g.n // 2 - 1) ** 2)).max()
    eo = np.abs(got - orc).max() / full
    _say("  against the FP64 truncated sum: %.3g of the full-band peak" % eo)
    assert eo <= TOL
    # second call, smaller: another context (fewer balls, n = 32), 100
    # translations, |m|^2 <= 64; the scratch still holds the first call's data
    A2 = synth.mixture_balls(200, 1701)
    B2 = synth.mixture_balls(150, 2701)
    g2 = synth.grid_for(A2, B2, 32)
    q2 = synth.random_quaternions(1, 3701)[0]
    t2 = np.random.default_rng(8).uniform(-0.3, 0.3, (100, 3))
    _say("case: no-alloc query, second call, 200+150 balls, n=32, 100 translations, r2=64")
    c2 = pkg.Correlator(A2, B2, g2.n, g2.box, g2.origin)
    ref2, got2, nm2 = _both(pkg, c2, q2, t2, 64)
    e2 = np.abs(got2 - ref2).max() / np.abs(ref2).max()
    _say("  modes %d: max |noalloc - query| / max |query| = %.3g" % (nm2, e2))
    assert e2 <= TOL
    assert np.array_equal(got2, ref2)
    # and the first context again, after the second call
    ref3, got3, _ = _both(pkg, c1, q, t[:300], 100)
    assert np.array_equal(got3, ref3)
    c1.close()
    c2.close()


def test_noalloc_query_refuses_requests_beyond_its_scratch(pkg):
    A = synth.mixture_balls(600, 1702)
    B = synth.mixture_balls(4096, 2702)
    g = synth.grid_for(A, B, 128)
    q = synth.random_quaternions(1, 3702)[0]
    c = pkg.Correlator(A, B, g.n, g.box, g.origin)
    out = torch.empty(4, dtype=torch.float32, device="cuda")
    t = np.zeros((4, 3))
    _say("case: no-alloc query refusals (every mode at n=128; 2^16+ half-space modes)")
    lib = pkg.load_library()
    qq = np.ascontiguousarray(q, dtype=np.float64)
    tt = np.ascontiguousarray(t)
    nm = ctypes.c_int64()
    for r2 in (3 * 63 ** 2, 2000):
        rc = lib.corr_query_noalloc(c.ctx, qq.ctypes.data, tt.ctypes.data, 4, r2, out.data_ptr(), ctypes.byref(nm))
        assert rc == pkg.CORR_EUNSUPPORTED
        assert "corr_query_noalloc" in pkg.corr_last_error(c.ctx)
    # the context is still usable, and a request within the limits works
    s, _ = c.query(q, t, 100)
    with torch.cuda.device(c.device):
        pkg.corr_query_noalloc(c.ctx, q, t, 100, out.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), s.cpu().numpy())
    c.close()
