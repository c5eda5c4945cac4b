"""Failure paths of the C ABI, forced from the host so that every kernel still
exits normally: device allocations refused by the CORR_TEST_MAX_BYTES cap
(CORR_ENOMEM) and stage launches refused by CORR_TEST_FAIL_STAGE (CORR_EHIP).
After each failure the context must still give bitwise the results it gave
before (the header's promise that an error leaves the context usable)."""
import os
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


class _env:
    """Set one environment variable for a block, then remove it again."""

    def __init__(self, name, value):
        self.name, self.value = name, value

    def __enter__(self):
        os.environ[self.name] = self.value

    def __exit__(self, *exc):
        os.environ.pop(self.name, None)


def _case():
    A = synth.mixture_balls(500, 1301)
    B = synth.mixture_balls(400, 2301)
    return A, B, synth.random_quaternions(3, 3301), synth.grid_for(A, B, 32)


def _eval(c, q):
    s, pv, pi = c.eval(q)
    torch.cuda.synchronize()
    return s.cpu().numpy(), pv.cpu().numpy(), pi.cpu().numpy()


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_allocation_cap_refuses_create(pkg):
    A, B, q, g = _case()
    _say("case: create under a 1-byte allocation cap")
    with _env("CORR_TEST_MAX_BYTES", "1"):
        with pytest.raises(pkg.CorrError) as e:
            pkg.Correlator(A, B, g.n, g.box, g.origin)
    assert e.value.code == pkg.CORR_ENOMEM
    assert "CORR_TEST_MAX_BYTES" in str(e.value)


def test_allocation_cap_leaves_the_context_usable(pkg):
    A, B, q, g = _case()
    _say("case: offsets and workspace growth refused by the allocation cap")
    c = pkg.Correlator(A, B, g.n, g.box, g.origin, batch=2)
    ref = _eval(c, q)
    before = c.tuning()
    with _env("CORR_TEST_MAX_BYTES", "1"):
        with pytest.raises(pkg.CorrError) as e:
            c.set_offsets([0.01])
        assert e.value.code == pkg.CORR_ENOMEM
        with pytest.raises(pkg.CorrError) as e:
            c.set_tuning(**dict(before, slots=4))
        assert e.value.code == pkg.CORR_ENOMEM
    # the old workspace and tuning stay in force, and the results are unchanged
    assert c.tuning() == before
    assert _same(_eval(c, q), ref)
    # without the cap the same calls succeed
    c.set_offsets([0.01])
    c.set_offsets([])
    c.set_tuning(**dict(before, slots=4))
    assert _same(_eval(c, q), ref)
    c.close()


@pytest.mark.parametrize("stage", [0, 1, 2, 3, 5, 6, 7, 8])
def test_forced_launch_failure_in_eval(pkg, stage):
    A, B, q, g = _case()
    _say("case: launch of stage %d refused during corr_eval" % stage)
    c = pkg.Correlator(A, B, g.n, g.box, g.origin, batch=2)
    ref = _eval(c, q)
    with _env("CORR_TEST_FAIL_STAGE", str(stage)):
        with pytest.raises(pkg.CorrError) as e:
            c.eval(q)
    torch.cuda.synchronize()
    assert e.value.code == pkg.CORR_EHIP
    assert "CORR_TEST_FAIL_STAGE" in str(e.value)
    assert _same(_eval(c, q), ref)
    c.close()


def test_forced_launch_failure_in_prepare_a(pkg):
    A, B, q, g = _case()
    _say("case: launch of A's z pass refused during corr_prepare_a")
    c = pkg.Correlator(A, B, g.n, g.box, g.origin)
    ref = _eval(c, q)
    with _env("CORR_TEST_FAIL_STAGE", str(4)):
        with pytest.raises(pkg.CorrError) as e:
            c.prepare_a()
    assert e.value.code == pkg.CORR_EHIP
    # A's spectrum was left half done: recomputing it restores the results
    c.prepare_a()
    assert _same(_eval(c, q), ref)
    c.close()
