"""Launch shapes, the autotuner and graph replay, through the C ABI.

No launch shape changes the arithmetic or its order, so every tuning must give
bitwise the same scores, peaks and obstacle bits as the default one; a graph
replay must give bitwise what the launch-by-launch evaluation gives, replay
after replay, with other device work and synchronisations between replays.
The default path itself is held to the FP64 oracle here once more (n = 32) and
in the parity tests.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_05075_amd as pkg
    pkg.load_library()


def _pair(n, na=600, nb=500, seed=0):
    A = synth.mixture_balls(na, 1000 + seed)
    B = synth.mixture_balls(nb, 2000 + seed)
    return A, B, synth.grid_for(A, B, n)


def _corr(A, B, g, **kw):
    from paper_1711_05075_amd import Correlator
    return Correlator(A, B, g.n, g.box, g.origin, **kw)


def _eval(c, q, out):
    import paper_1711_05075_amd as pkg
    s, pv, pi = out
    pkg.corr_eval(c.ctx, q, s.data_ptr(), pv.data_ptr(), pi.data_ptr())
    torch.cuda.synchronize()
    return s.clone(), pv.clone(), pi.clone()


def _outs(r, n):
    dev = torch.device("cuda:0")
    return (torch.empty((r, n, n, n), dtype=torch.float32, device=dev),
            torch.empty(r, dtype=torch.float32, device=dev), torch.empty(r, dtype=torch.int64, device=dev))


def _same(a, b, what):
    for x, y, name in zip(a, b, ("scores", "peak_val", "peak_idx")):
        assert torch.equal(x, y), "%s: %s differ" % (what, name)


@pytest.mark.parametrize("n", [32, 64, 128])
def test_every_launch_shape_gives_the_same_bits(n):
    import paper_1711_05075_amd as pkg
    A, B, g = _pair(n, seed=n)
    q = synth.random_quaternions(3, 3000 + n)
    _say("case: launch shapes, 600+500 balls, n=%d, 3 rotations" % n)
    c = _corr(A, B, g)
    out = _outs(3, n)
    ref = _eval(c, q, out)
    if n == 32:  # the default path against the FP64 oracle
        FA = oracle.o2_spectrum(A, np.eye(3), n, g.box)
        for r in range(3):
            FB = oracle.o2_spectrum(B, oracle.quat_to_rot(q[r]), n, g.box)
            s2 = oracle.o2_scores_from_spectra(FA, FB, g.box, g.origin)
            e = np.abs(ref[0][r].double().cpu().numpy() - s2).max() / np.abs(s2).max()
            _say("  rot %d: e_rel vs FP64 = %.3g" % (r, e))
            assert e <= 1e-4
    base = c.tuning()
    _say("  default tuning:", base)
    fields = ("cols_y", "cols_z", "cols_iy", "pairs_ix")
    for p, f in enumerate(fields):
        ch = pkg.corr_tuning_choices(c.ctx, p)
        assert ch[0] == base[f]
        for w in ch[1:]:
            c.set_tuning(**{f: w})
            _same(_eval(c, q, out), ref, "%s = %d" % (f, w))
            _say("  %s = %d: bitwise equal" % (f, w))
        c.set_tuning(**{f: base[f]})
    # the spreading pass's bins: y-groups of the sort keys
    bins = pkg.corr_tuning_choices(c.ctx, 4)
    assert bins[0] == base["bin_group"] and len(bins) >= 2
    for gsz in bins[1:]:
        c.set_tuning(bin_group=gsz)
        _same(_eval(c, q, out), ref, "bin_group = %d" % gsz)
        _say("  bin_group = %d: bitwise equal" % gsz)
    c.set_tuning(bin_group=base["bin_group"])
    # the spreading pass's tile height
    rows = pkg.corr_tuning_choices(c.ctx, 5)
    assert rows[0] == base["tile_rows"] and rows[1] == base["tile_rows"] // 2
    c.set_tuning(tile_rows=rows[1])
    _same(_eval(c, q, out), ref, "tile_rows = %d" % rows[1])
    _say("  tile_rows = %d: bitwise equal" % rows[1])
    c.set_tuning(tile_rows=rows[1], bin_group=bins[-1])
    _same(_eval(c, q, out), ref, "tile_rows = %d, bin_group = %d" % (rows[1], bins[-1]))
    c.set_tuning(tile_rows=base["tile_rows"], bin_group=base["bin_group"])
    cus = base["spread_wgs"] // 2
    for v in (1, cus):
        c.set_tuning(spread_wgs=v)
        _same(_eval(c, q, out), ref, "spread_wgs = %d" % v)
    c.set_tuning(spread_wgs=base["spread_wgs"])
    for sl in (1, 2):
        c.set_tuning(slots=sl)
        assert c.tuning()["slots"] == sl
        _same(_eval(c, q, out), ref, "slots = %d" % sl)
    _say("  spread_wgs and slots: bitwise equal")
    with pytest.raises(pkg.CorrError):
        c.set_tuning(cols_y=3)
    with pytest.raises(pkg.CorrError):
        c.set_tuning(spread_wgs=0)
    with pytest.raises(pkg.CorrError):
        c.set_tuning(slots=257)
    with pytest.raises(pkg.CorrError):
        c.set_tuning(bin_group=3)
    with pytest.raises(pkg.CorrError):
        c.set_tuning(tile_rows=3)
    c.close()


def test_autotune_keeps_a_valid_tuning_and_the_results():
    import paper_1711_05075_amd as pkg
    A, B, g = _pair(64, na=2000, nb=800, seed=7)
    q = synth.random_quaternions(8, 3007)
    _say("case: autotune, 2000+800 balls, n=64, 8 rotations")
    c = _corr(A, B, g)
    out = _outs(8, 64)
    ref = _eval(c, q, out)
    cus = c.tuning()["spread_wgs"] // 2  # the default is two per CU
    t = c.autotune(q, reps=1)
    _say("  kept:", t)
    assert t == c.tuning()
    for p, f in enumerate(("cols_y", "cols_z", "cols_iy", "pairs_ix", "bin_group", "tile_rows")):
        assert t[f] in pkg.corr_tuning_choices(c.ctx, p)
    assert 1 <= t["slots"] <= 256 and t["graph"] == 0
    _same(_eval(c, q, out), ref, "after autotune")
    # timing A's spectrum with each evaluation (the side stream joined inside)
    t = c.autotune(q, reps=1, with_a=True)
    _say("  kept with A's spectrum timed:", t)
    assert t["spread_wgs"] in (cus, cus + cus // 2, 2 * cus)
    _same(_eval(c, q, out), ref, "after autotune with A")
    # tuning in graph mode: every candidate is captured and replayed
    c.set_tuning(graph=1)
    t = c.autotune(q, reps=1)
    _say("  kept in graph mode:", t)
    assert t["graph"] == 1
    _same(_eval(c, q, out), ref, "after autotune in graph mode")
    _same(_eval(c, q, out), ref, "replay after autotune in graph mode")
    c.close()


def test_graph_replays_match_the_eager_evaluation():
    A, B, g = _pair(64, seed=11)
    q1 = synth.random_quaternions(5, 3011)
    q2 = synth.random_quaternions(5, 3012)
    _say("case: graph replay, 600+500 balls, n=64, 5 rotations in batches of 2")
    c = _corr(A, B, g, batch=2)
    out = _outs(5, 64)
    ref1 = _eval(c, q1, out)
    ref2 = _eval(c, q2, out)
    c.set_tuning(graph=1)
    import paper_1711_05075_amd as pkg
    pkg.corr_profile(c.ctx, True)
    pkg.corr_profile_read(c.ctx)
    for k in range(6):
        q, ref = (q1, ref1) if k % 2 == 0 else (q2, ref2)
        got = _eval(c, q, out)
        _same(got, ref, "replay %d" % k)
        # the program's own device work and a synchronisation between replays
        x = torch.randn(1 << 20, device="cuda:0")
        _ = float(x.sum())
        torch.cuda.synchronize()
    prof = pkg.corr_profile_read(c.ctx)
    _say("  6 replays bitwise equal; graph launches timed:", prof["graph"][1])
    assert prof["graph"][1] == 6 and prof["rotate"][1] == 0
    # new output buffers: captured again, same bits
    out2 = _outs(5, 64)
    _same(_eval(c, q1, out2), ref1, "new outputs")
    # fewer rotations, then back
    sub = _outs(2, 64)
    got = _eval(c, q2[:2], sub)
    for x, y in zip(got, ref2):
        assert torch.equal(x, y[:2])
    _same(_eval(c, q1, out), ref1, "back to five rotations")
    c.set_tuning(graph=0)
    _same(_eval(c, q2, out), ref2, "graph off")
    c.close()


def test_graph_replays_of_offset_slices():
    A, B, g = _pair(32, seed=13)
    g = synth.grid_for(A, B, 32, pad=0.02)
    q = synth.random_quaternions(3, 3013)
    _say("case: graph replay of slices, 600+500 balls, n=32, 3 rotations, 2 offsets")
    c = _corr(A, B, g)
    c.set_offsets([0.0, 0.005])
    kw = dict(scores=True, peaks=True, obstacle=True, count=True, threshold=1e-6)
    ref = c.eval_slices(q, **kw)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items()}
    c.set_tuning(graph=1)
    import paper_1711_05075_amd as pkg
    dev = torch.device("cuda:0")
    n = 32
    outs = {"scores": torch.empty((2, 3, n, n, n), dtype=torch.float32, device=dev),
            "peak_val": torch.empty((2, 3), dtype=torch.float32, device=dev),
            "peak_idx": torch.empty((2, 3), dtype=torch.int64, device=dev),
            "obstacle": torch.empty((2, 3, n ** 3 // 32), dtype=torch.int32, device=dev),
            "obstacle_count": torch.empty((2, 3), dtype=torch.int64, device=dev)}
    for k in range(3):
        pkg.corr_eval_slices(c.ctx, q, outs["scores"].data_ptr(), outs["peak_val"].data_ptr(),
                             outs["peak_idx"].data_ptr(), outs["obstacle"].data_ptr(),
                             outs["obstacle_count"].data_ptr(), 1e-6)
        torch.cuda.synchronize()
        for name in ref:
            assert torch.equal(outs[name], ref[name]), "replay %d: %s" % (k, name)
        for v in outs.values():
            v.zero_()
        torch.cuda.synchronize()
    _say("  3 replays bitwise equal (scores, peaks, obstacle bits and counts)")
    c.close()


def test_batch_graph_replays_match_the_eager_batch():
    from paper_1711_05075_amd import Batch
    pairs, quats = [], []
    for p, (n, na, nb) in enumerate(((32, 700, 300), (64, 1500, 900), (32, 400, 1200))):
        A = synth.mixture_balls(na, 1100 + p)
        B = synth.mixture_balls(nb, 2100 + p)
        g = synth.grid_for(A, B, n)
        pairs.append((A, B, n, g.box, g.origin))
        quats.append(synth.random_quaternions(2 + p, 3100 + p))
    _say("case: batch graph, 3 pairs (n = 32, 64, 32), 2..4 rotations")
    b = Batch(pairs, slots=2)
    ref = b.eval(quats, scores=True)
    torch.cuda.synchronize()
    ref_s = [x.clone() for x in ref[0]]
    ref_pv, ref_pi = ref[1].clone(), ref[2].clone()
    total = sum(len(q) * n ** 3 for q, n in zip(quats, b.ns))
    dev = torch.device("cuda:0")
    s = torch.empty(total, dtype=torch.float32, device=dev)
    pv = torch.empty(len(np.concatenate(quats)), dtype=torch.float32, device=dev)
    pi = torch.empty_like(pv, dtype=torch.int64)
    b.set_graph(True)
    for k in range(4):
        got = b.eval(quats, out=(s, pv, pi))
        torch.cuda.synchronize()
        for x, y in zip(got[0], ref_s):
            assert torch.equal(x, y), "replay %d: scores" % k
        assert torch.equal(got[1], ref_pv) and torch.equal(got[2], ref_pi), "replay %d: peaks" % k
        s.zero_()
        x = torch.randn(1 << 18, device=dev)
        _ = float(x.sum())
        torch.cuda.synchronize()
    _say("  4 replays bitwise equal")
    b.close()


def test_batch_autotune_keeps_every_bit():
    # the batch autotuner tries every spreading workgroup count, and for each
    # grid size in turn every width rank of every column pass, every bin-group
    # rank and every tile height; whatever it keeps, and every candidate it ran
    # (the outputs hold the last), the results stay bitwise
    from paper_1711_05075_amd import Batch
    pairs, quats = [], []
    for p, (n, na, nb) in enumerate(((32, 700, 300), (64, 1500, 900), (128, 400, 500), (32, 2500, 1200))):
        A = synth.mixture_balls(na, 1200 + p)
        B = synth.mixture_balls(nb, 2200 + p)
        g = synth.grid_for(A, B, n)
        pairs.append((A, B, n, g.box, g.origin))
        quats.append(synth.random_quaternions(3 + p, 3200 + p))
    _say("case: batch autotuner, 4 pairs (n = 32, 64, 128, 32), 3..6 rotations")
    b = Batch(pairs)
    ref = b.eval(quats, scores=True)
    torch.cuda.synchronize()
    ref_s = [x.clone() for x in ref[0]]
    ref_pv, ref_pi = ref[1].clone(), ref[2].clone()
    total = sum(len(q) * n ** 3 for q, n in zip(quats, b.ns))
    dev = torch.device("cuda:0")
    s = torch.empty(total, dtype=torch.float32, device=dev)
    pv = torch.empty(len(np.concatenate(quats)), dtype=torch.float32, device=dev)
    pi = torch.empty_like(pv, dtype=torch.int64)
    kept = b.autotune(quats, (s, pv, pi), reps=1)
    torch.cuda.synchronize()
    _say("  kept %s" % kept)
    assert 0 <= kept["rank_bin_group"] <= 2 and 0 <= kept["rank_tile_rows"] <= 1
    off = 0
    for x, q, n in zip(ref_s, quats, b.ns):
        assert torch.equal(s[off:off + len(q) * n ** 3].view(len(q), n, n, n), x)
        off += len(q) * n ** 3
    assert torch.equal(pv, ref_pv) and torch.equal(pi, ref_pi)
    # and a plain evaluation under the kept tuning
    got = b.eval(quats, scores=True)
    torch.cuda.synchronize()
    for x, y in zip(got[0], ref_s):
        assert torch.equal(x, y)
    b.close()


def test_side_stream_spectrum_of_a_is_joined_everywhere():
    # corr_prepare_a runs on a side stream; every later call must see its result
    import paper_1711_05075_amd as pkg
    A, B, g = _pair(64, na=1500, nb=700, seed=17)
    q = synth.random_quaternions(3, 3017)
    _say("case: A's spectrum on the side stream, 1500+700 balls, n=64")
    c = _corr(A, B, g)
    out = _outs(3, 64)
    ref = _eval(c, q, out)
    spec_a = c.spectrum(0).clone()
    t = np.array([[0.01, -0.02, 0.03], [0.0, 0.0, 0.0]])
    qry_ref, _ = c.query(q[0], t, 100)
    qry_ref = qry_ref.clone()
    pkg.corr_profile(c.ctx, True)
    for k in range(3):
        c.prepare_a()
        _same(_eval(c, q, out), ref, "eval after prepare_a %d" % k)
    prof = pkg.corr_profile_read(c.ctx)
    assert prof["spread_fft_x"][1] == 6  # three A passes and three B passes, all timed
    pkg.corr_profile(c.ctx, False)
    c.prepare_a()
    info = c.pass_info()
    assert info["knots"] == len(A) and info["rotations"] == 1 and info["live_tiles"] > 0
    c.prepare_a()
    assert torch.equal(c.spectrum(0), spec_a)
    c.prepare_a()
    got, _ = c.query(q[0], t, 100)
    torch.cuda.synchronize()
    assert torch.equal(got, qry_ref)
    c.prepare_a()
    c.set_tuning(graph=1)
    _same(_eval(c, q, out), ref, "graph after prepare_a")
    c.prepare_a()
    _same(_eval(c, q, out), ref, "graph replay after prepare_a")
    c.prepare_a()
    c.close()  # destroy with the side stream's work still queued
    _say("  evaluations, pass report, spectrum, query and graph replays after prepare_a: bitwise equal")
