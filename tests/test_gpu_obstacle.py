"""GPU parity of the configuration-obstacle outputs and the offset slices.

corr_eval_slices scores B's rotations against A and against A's balls offset
by each delta of corr_set_offsets (Sec. 3.1, offset obstacles), and writes the
obstacle predicate score > threshold (Sec. 3.1 eq. eq_obs) as a bit mask with a
count per rotation.

Gates:
  - scores of each slice: max |s_gpu - s_o2| / max |s_o2| <= 1e-4 against the
    FP64 band-limited oracle of the offset balls;
  - mask and count: the predicate is a float decision, so it is checked bit for
    bit against the same comparison made on the CPU on the GPU's own float
    scores; against the FP64 oracle it must agree wherever the oracle's score
    is farther than the parity tolerance from the threshold.
"""
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


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_05075_amd as pkg
    pkg.load_library()


def _corr(A, B, g, **kw):
    from paper_1711_05075_amd import Correlator
    return Correlator(A, B, g.n, g.box, g.origin, **kw)


def _bits(words, n):
    """[..., n^3 / 32] int32 words -> [..., n, n, n] bool (bit b of word w: index 32 w + b)."""
    w = np.ascontiguousarray(words.cpu().numpy()).view(np.uint8)
    b = np.unpackbits(w.reshape(*w.shape[:-1], -1), axis=-1, bitorder="little")
    return b.reshape(*words.shape[:-1], n, n, n).astype(bool)


def _check_mask(out, thr, n):
    s = out["scores"].cpu().numpy()
    mask = _bits(out["obstacle"], n)
    want = s > np.float32(thr)
    assert np.array_equal(mask, want), "%d bits differ" % int(np.sum(mask != want))
    cnt = out["obstacle_count"].cpu().numpy()
    assert np.array_equal(cnt, want.reshape(*want.shape[:2], -1).sum(axis=-1))
    return mask


@pytest.mark.parametrize("n", [16, 64, 128])
def test_obstacle_mask_is_the_thresholded_float_scores(n):
    A = synth.mixture_balls(300, 1601)
    B = synth.mixture_balls(250, 2601)
    g = synth.grid_for(A, B, n)
    q = synth.random_quaternions(3, 3601)
    _say("case: obstacle mask, 300+250 balls, n=%d, 3 rotations" % n)
    c = _corr(A, B, g, batch=2)
    s_ref, pv_ref, pi_ref = c.eval(q)
    for thr in (0.0, 1e-3 * float(s_ref.abs().max().item())):
        out = c.eval_slices(q, obstacle=True, count=True, threshold=thr)
        torch.cuda.synchronize()
        # the same kernels as corr_eval: identical scores and peaks
        assert torch.equal(out["scores"][0], s_ref)
        assert torch.equal(out["peak_val"][0], pv_ref) and torch.equal(out["peak_idx"][0], pi_ref)
        mask = _check_mask(out, thr, n)
        _say("  threshold %.3g: obstacle fractions %s" % (thr, np.round(mask[0].reshape(3, -1).mean(axis=1), 4)))
        assert 0 < mask.sum() < mask.size
    c.close()


def test_obstacle_agrees_with_the_oracle_away_from_the_threshold():
    A = synth.mixture_balls(500, 1602)
    B = synth.mixture_balls(400, 2602)
    g = synth.grid_for(A, B, 64)
    q = synth.random_quaternions(2, 3602)
    _say("case: obstacle vs FP64 oracle, 500+400 balls, n=64")
    c = _corr(A, B, g)
    for r in range(len(q)):
        ref = oracle.o2_scores(A, B, q[r], g.n, g.box, g.origin)
        thr = 0.02 * np.abs(ref).max()
        out = c.eval_slices(q[r:r + 1], scores=False, peaks=False, obstacle=True, count=True, threshold=thr)
        torch.cuda.synchronize()
        mask = _bits(out["obstacle"], g.n)[0, 0]
        want = oracle.obstacle(ref, thr)
        clear = np.abs(ref - thr) > TOL * np.abs(ref).max()
        bad = np.sum((mask != want) & clear)
        _say("  rot %d: obstacle %d of %d, %d near the threshold, %d disagree away from it"
             % (r, int(want.sum()), want.size, int((~clear).sum()), int(bad)))
        assert bad == 0
        assert int(out["obstacle_count"][0, 0].item()) == int(mask.sum())
    c.close()


def test_obstacle_of_an_empty_shape_is_empty():
    A = synth.mixture_balls(100, 1603)
    B = np.zeros((0, 5))
    g = synth.grid_for(A, A, 32)
    c = _corr(A, B, g)
    out = c.eval_slices(synth.random_quaternions(2, 3603), obstacle=True, count=True, threshold=0.0)
    torch.cuda.synchronize()
    assert not out["scores"].any()
    assert not out["obstacle"].any()
    assert out["obstacle_count"].sum().item() == 0
    c.close()


def test_offset_slices_match_the_oracle():
    A = synth.mixture_balls(600, 1604)
    B = synth.mixture_balls(450, 2604)
    rmin = A[:, 3].min()
    offsets = [-0.5 * rmin, 0.0, 0.01, 0.03]
    g = synth.grid_for(A, B, 64, pad=2 * max(offsets))
    q = synth.random_quaternions(3, 3604)
    _say("case: offset slices %s, 600+450 balls, n=64, 3 rotations in batches of 2" % np.round(offsets, 4))
    c = _corr(A, B, g, batch=2)
    s_plain, _, _ = c.eval(q, peaks=False)
    thr = 0.01 * float(s_plain.abs().max().item())
    c.set_offsets(offsets)
    out = c.eval_slices(q, obstacle=True, count=True, threshold=thr)
    torch.cuda.synchronize()
    s = out["scores"].double().cpu().numpy()
    assert torch.equal(out["scores"][1], s_plain)  # offset 0 is the context's own score, bit for bit
    for k, d in enumerate(offsets):
        for r in range(len(q)):
            ref = oracle.o2_offset_scores(A, B, q[r], g.n, g.box, g.origin, d)
            e = np.abs(s[k, r] - ref).max() / np.abs(ref).max()
            _say("  offset %+.4f rot %d: e_rel vs FP64 = %.3g (peak %.4g)" % (d, r, e, ref.max()))
            assert e <= TOL
    _check_mask(out, thr, g.n)
    # growing the balls grows the obstacle
    cnt = out["obstacle_count"].cpu().numpy()
    assert np.all(np.diff(cnt, axis=0) > 0)
    c.close()


def test_offset_slice_outputs_without_scores_are_the_same():
    A = synth.mixture_balls(400, 1605)
    B = synth.mixture_balls(300, 2605)
    g = synth.grid_for(A, B, 32, pad=0.04)
    q = synth.random_quaternions(5, 3605)
    c = _corr(A, B, g, batch=3)
    c.set_offsets([0.02, -0.002])
    full = c.eval_slices(q, obstacle=True, count=True, threshold=1e-6)
    lean = c.eval_slices(q, scores=False, peaks=False, obstacle=True, count=True, threshold=1e-6)
    peaks = c.eval_slices(q, scores=False, peaks=True)
    torch.cuda.synchronize()
    assert torch.equal(full["obstacle"], lean["obstacle"])
    assert torch.equal(full["obstacle_count"], lean["obstacle_count"])
    assert torch.equal(full["peak_val"], peaks["peak_val"]) and torch.equal(full["peak_idx"], peaks["peak_idx"])
    flat = full["scores"].reshape(2, 5, -1)
    assert torch.equal(full["peak_val"], flat.max(dim=2).values)
    # clearing the offsets leaves one slice: the context's own score
    c.set_offsets([])
    one = c.eval_slices(q[:2], peaks=False)
    s, _, _ = c.eval(q[:2], peaks=False)
    torch.cuda.synchronize()
    assert one["scores"].shape[0] == 1 and torch.equal(one["scores"][0], s)
    c.close()


def test_set_offsets_errors_keep_the_previous_slices():
    import paper_1711_05075_amd as pkg
    A = synth.mixture_balls(200, 1606)
    B = synth.mixture_balls(150, 2606)
    g = synth.grid_for(A, B, 32, pad=0.02)
    c = _corr(A, B, g)
    c.set_offsets([0.0, 0.01])
    q = synth.random_quaternions(1, 3606)
    before = c.eval_slices(q, peaks=False)["scores"]
    rmin = A[:, 3].min()
    for bad, code in (([-rmin], pkg.CORR_EINVAL), ([np.nan], pkg.CORR_EINVAL),
                      ([0.0] * (pkg.CORR_MAX_SLICES + 1), pkg.CORR_EINVAL)):
        with pytest.raises(pkg.CorrError) as e:
            pkg.corr_set_offsets(c.ctx, bad)
        assert e.value.code == code
    after = c.eval_slices(q, peaks=False)["scores"]
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    with pytest.raises(pkg.CorrError) as e:
        pkg.corr_eval_slices(c.ctx, q, threshold=float("inf"))
    assert e.value.code == pkg.CORR_EINVAL
    c.close()
    sc = _corr(A, B, g, sc=(0.01, 1.0))
    with pytest.raises(pkg.CorrError) as e:
        pkg.corr_set_offsets(sc.ctx, [0.01])
    assert e.value.code == pkg.CORR_EUNSUPPORTED
    sc.close()


def test_offset_slices_full_size_single_rotation():
    # the single-rotation workload (4096 + 4096 balls, 128^3 translations) with
    # three offset slices; slice 2 checked against the FP64 oracle in full
    A, B, q, g0 = synth.single_rotation_case()
    offsets = [0.0, -0.002, 0.01]
    g = synth.grid_for(A, B, g0.n, pad=0.02)
    _say("case: offset slices %s, single rotation 4096+4096, n=128 (oracle takes a while)" % offsets)
    c = _corr(A, B, g)
    c.set_offsets(offsets)
    out = c.eval_slices(q, obstacle=True, count=True, threshold=0.0)
    torch.cuda.synchronize()
    thr = 0.01 * float(out["scores"][0].abs().max().item())
    _check_mask(out, 0.0, g.n)
    out = c.eval_slices(q, obstacle=True, count=True, threshold=thr)
    torch.cuda.synchronize()
    _check_mask(out, thr, g.n)
    ref = oracle.o2_offset_scores(A, B, q[0], g.n, g.box, g.origin, offsets[2])
    s = out["scores"][2, 0].double().cpu().numpy()
    e = np.abs(s - ref).max() / np.abs(ref).max()
    _say("  offset %+.3f: e_rel vs FP64 = %.3g; obstacle counts %s" % (offsets[2], e,
                                                                        out["obstacle_count"][:, 0].tolist()))
    assert e <= TOL
    c.close()
