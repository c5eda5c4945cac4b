"""Benchmark: rotation x translation scores per second on one MI355X.

Default workload: one rotation of two 4096-ball Gaussian-mixture shapes (radii
lognormal(ln 0.02, 0.3)) on a 128^3 translation grid, 2x oversampled spreading
grid, Kaiser-Bessel window of width 8.  One step = the whole pipeline for that
rotation including the fixed shape's spectrum (corr_prepare_a + corr_eval with
scores and peaks), inputs resident on the device.

Prints one JSON line with the throughput, the dominant kernel's roofline
(algorithmic bytes per launch / its mean event-timed duration) and the FP64
oracle timed on the host for one rotation of the same workload.  The line also
holds, under "batched", the 512-rotation workload (20000 + 2000 balls, 64^3)
timed launch by launch, as a hipGraph and autotuned (--no-batched skips it).
Other workloads: --batched, --uneven, --proposal, --query, --slices, --sc.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "traffic_spread_fftx_single_rotation_4096_n128.txt")


def stage_bytes(info, pa, pb):
    """Algorithmic HBM bytes of one launch of each stage for this workload.

    pa / pb are the occupancy reports of the A and B spreading passes
    (corr_pass_info): only live tiles are spread and written, and the later
    passes read only live z rows.  Each stage reads its inputs once and writes
    its outputs once: knot records (cell 4 B, window weights 12 w B, component
    weights 4 q B), complex64 spectra, float32 scores.  Stages that run once per
    shape (rotate, bin, spread, fft_y) are averaged over the A and B launches.
    """
    n, w = info["n"], info["kb_width"]
    h = n // 2
    spec = 8 * n * n * h

    def per_shape(p):
        q, k, ty, m = p["q"], p["knots"], p["tile_rows"], p["m"]
        rec = k * (4 + 12 * w + 4 * q)
        tile_out = p["live_tiles"] * ty * (m // 4) * 8 * q  # kept x modes of every line of a live tile
        rows_out = p["live_rows"] * n * h * 8 * q             # kept y modes of every live z row
        return {"rotate": k * (24 + 12 * w + 8), "bin": k * 4 + 2 * rec, "spread_fft_x": rec + tile_out,
                "fft_y": tile_out + rows_out, "rows_out": rows_out}

    a, b = per_shape(pa), per_shape(pb)
    out = {k: (a[k] + b[k]) / 2 for k in ("rotate", "bin", "spread_fft_x", "fft_y")}
    out["fft_z_spectrum"] = a["rows_out"] + spec
    out["fft_z_product"] = b["rows_out"] + 2 * spec
    out["ifft_y"] = 2 * spec
    out["ifft_x"] = spec + 4 * n ** 3
    return out


def measured_traffic():
    """HBM bytes per launch of the spreading kernel from the committed counter
    summary, if it was taken on the current kernel source; else None."""
    from paper_1711_05075_amd.rocprof_summary import kernel_source_digest
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    fields = {}
    for line in open(TRAFFIC_SUMMARY):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return float(fields["hbm_bytes_per_launch"])


def run_proposal(args, torch, pkg):
    """Rotation-proposal workflow: train the network on exhaustive peaks of
    seeded pairs, then compare its top-64 of 4096 candidates with exhaustive
    search, random-64 and a coarse n = 16 correlation."""
    dev = torch.device("cuda:0")
    n_train, n_unseen, rot_train, n_cand, top = args.proposal_pairs, max(1, args.proposal_pairs // 5), 1000, 4096, 64
    prop = pkg.Proposer(batch=1024, seed=11, device=dev)

    def volume(b):
        return float(np.sum(b[:, 4] * 4.0 * np.pi * b[:, 3] ** 3 / 3.0))

    def timed(f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    def visit(A, B, g, qtrain, qcand):
        """Exhaustive peaks (training and candidate rotations), times, coarse peaks."""
        c = pkg.Correlator(A, B, g.n, g.box, g.origin, batch=64, device=dev)
        c.eval(qcand[:top], scores=False)  # warm
        _, t64 = timed(lambda: c.eval(qcand[:top], scores=False))
        ytr = c.eval(qtrain, scores=False)[1].double().cpu().numpy() if len(qtrain) else np.zeros(0)
        (_, pv, _), t_exh = timed(lambda: c.eval(qcand, scores=False))
        peaks = pv.double().cpu().numpy()
        c.close()
        cc = pkg.Correlator(A, B, 16, g.box, g.origin, batch=64, device=dev)
        cc.eval(qcand[:top], scores=False)
        (_, pc, _), t_coarse = timed(lambda: cc.eval(qcand, scores=False))
        coarse = pc.double().cpu().numpy()
        cc.close()
        return ytr, peaks, coarse, t64, t_exh, t_coarse

    t_start = time.perf_counter()
    seen = synth.proposal_pairs(n_train, 5000)
    unseen = synth.proposal_pairs(n_unseen, 9000)
    X_parts, y_parts, records = [], [], []
    for p, (A, B, g) in enumerate(seen + unseen):
        is_seen = p < n_train
        # training rotations: an evenly spread set (super-Fibonacci spiral, turned per
        # pair); candidates: fresh uniform random rotations
        qtrain = synth.super_fibonacci_quaternions(rot_train, 6000 + p) if is_seen else np.zeros((0, 4))
        qcand = synth.random_quaternions(n_cand, 7000 + p, canonical=True)
        ytr, peaks, coarse, t64, t_exh, t_coarse = visit(A, B, g, qtrain, qcand)
        vv = volume(A) * volume(B)
        da, db = prop.descriptor(A), prop.descriptor(B)
        if is_seen:
            # targets standardised per pair: the ranking is within a pair, so the
            # network should spend its capacity on how the peak varies with rotation;
            # then exp(beta z), standardised again: a monotone map (the ranking is
            # unchanged) that stretches the top of the range, where the ranking matters
            t = ytr / vv
            z = (t - t.mean()) / max(t.std(), 1e-12)
            if args.proposal_beta > 0:
                e = np.exp(args.proposal_beta * z)
                z = (e - e.mean()) / max(e.std(), 1e-12)
            X_parts.append(prop.features(qtrain, da, db))
            y_parts.append(torch.tensor(z, dtype=torch.float32, device=dev))
        records.append(dict(seen=is_seen, qcand=qcand, da=da, db=db, peaks=peaks, coarse=coarse, t64=t64,
                            t_exh=t_exh, t_coarse=t_coarse))
        print("pair %d/%d n_a %d n_b %d: exhaustive %.1f ms" % (p + 1, len(seen) + len(unseen), len(A), len(B),
                                                                  t_exh * 1e3), file=sys.stderr, flush=True)
    t_data = time.perf_counter() - t_start
    X = torch.cat(X_parts)
    y = torch.cat(y_parts)
    schedule = [(int(e), float(lr)) for e, lr in (part.split(":") for part in args.proposal_schedule.split(","))]

    def train_all():
        out = []
        for ep, lr in schedule:  # Adam's state carries over between the phases
            out += list(prop.train(X, y, ep, lr))
        return out

    losses, t_train = timed(train_all)

    def hits(order_idx, peaks):
        best = peaks.max()
        got = peaks[order_idx].max()
        return (got >= (1 - 1e-4) * best, int(np.argmax(peaks)) in set(order_idx.tolist()), got >= 0.99 * best)

    rng = np.random.default_rng(12)
    res = {k: {"mlp": [], "random": [], "coarse": [], "mlp_with_fallback": []} for k in ("seen", "unseen")}
    t_mlp_all, speed_mlp, speed_coarse = [], [], []
    # fallback: the network has only learnt the rotational landscapes of the
    # training pairs, so a pair whose descriptors match none of them is searched
    # exhaustively instead
    train_desc = np.stack([np.concatenate([r["da"].cpu().numpy(), r["db"].cpu().numpy()])
                           for r in records if r["seen"]])
    t_fb_all, t_exh_all = [], []
    for r in records:
        Xc = prop.features(r["qcand"], r["da"], r["db"])
        idx, t_mlp = timed(lambda: prop.rank(Xc, top).cpu().numpy())
        t_mlp_all.append(t_mlp)
        key = "seen" if r["seen"] else "unseen"
        res[key]["mlp"].append(hits(idx, r["peaks"]))
        res[key]["random"].append(hits(rng.choice(n_cand, top, replace=False), r["peaks"]))
        res[key]["coarse"].append(hits(np.argsort(-r["coarse"], kind="stable")[:top], r["peaks"]))
        d = np.concatenate([r["da"].cpu().numpy(), r["db"].cpu().numpy()])
        known = float(np.abs(train_desc - d).sum(axis=1).min()) < 1e-6
        if known:
            res[key]["mlp_with_fallback"].append(hits(idx, r["peaks"]))
            t_fb_all.append(t_mlp + r["t64"])
        else:
            res[key]["mlp_with_fallback"].append((True, True, True))
            t_fb_all.append(t_mlp + r["t_exh"])
        t_exh_all.append(r["t_exh"])
        speed_mlp.append(r["t_exh"] / (t_mlp + r["t64"]))
        speed_coarse.append(r["t_exh"] / (r["t_coarse"] + r["t64"]))
    # matrix-core use of the network: one forward pass over the 4096 candidates
    Xc = prop.features(records[0]["qcand"], records[0]["da"], records[0]["db"])
    prop.predict(Xc)
    _, t_pred = timed(lambda: prop.predict(Xc))
    flops = 2.0 * (160 * 256 + 256 * 256 + 256 * 256 + 256) * n_cand

    def summary(lst):
        a = np.array(lst, dtype=float)
        return {"recall": float(a[:, 0].mean()), "strict": float(a[:, 1].mean()), "within_1pct": float(a[:, 2].mean()),
                "pairs": len(lst)}

    out = {
        "metric": "proposal recall: best of top-64 of 4096 candidate rotations within 1e-4 of the exhaustive peak",
        "value": summary(res["seen"]["mlp"])["recall"], "unit": "fraction of pairs", "higher_is_better": True,
        "n_gpus": 1, "data": "synthetic",
        "config": {"workload": "rotation proposal: mixture pairs, 500-5000 balls (log-uniform), n = 64 grids, "
                               "%d training pairs x %d rotations, %d candidates, top %d, coarse proxy n = 16"
                               % (n_train, rot_train, n_cand, top),
                   "train_samples": int(X.shape[0]), "schedule_epochs_lr": schedule,
                   "target_beta": args.proposal_beta, "unseen_pairs": n_unseen},
        "seen": {k: summary(v) for k, v in res["seen"].items()},
        "unseen": {k: summary(v) for k, v in res["unseen"].items()},
        "speedup_vs_exhaustive": {"mlp_median": float(np.median(speed_mlp)),
                                  "coarse_median": float(np.median(speed_coarse)),
                                  "mlp_with_fallback_all_pairs": float(np.sum(t_exh_all) / np.sum(t_fb_all))},
        "all_pairs_mlp_with_fallback": summary(res["seen"]["mlp_with_fallback"] + res["unseen"]["mlp_with_fallback"]),
        "times_ms": {"exhaustive_4096_median": 1e3 * float(np.median([r["t_exh"] for r in records])),
                     "full_64_median": 1e3 * float(np.median([r["t64"] for r in records])),
                     "mlp_rank_4096_median": 1e3 * float(np.median(t_mlp_all)),
                     "coarse_4096_median": 1e3 * float(np.median([r["t_coarse"] for r in records])),
                     "train_total": 1e3 * t_train, "data_generation_total": 1e3 * t_data},
        "train_loss_by_epoch": [round(float(v), 4) for v in losses[::5]] + [round(float(losses[-1]), 4)],
        "mlp_forward": {"flops": flops, "ms": 1e3 * t_pred, "tflops": flops / t_pred / 1e12,
                        "mfma_frac_of_bf16_peak": flops / t_pred / 2.5e15},
    }
    prop.close()
    print(json.dumps(out), flush=True)


def run_query(args, torch, pkg):
    """Single-configuration queries on the single-rotation workload: time per
    call and error against the full band and the plain lens sum, by mode radius."""
    import oracle
    dev = torch.device("cuda:0")
    A, B, q, g = synth.single_rotation_case()
    c = pkg.Correlator(A, B, g.n, g.box, g.origin, device=dev)
    R = oracle.quat_to_rot(q[0])
    # near-contact translations: pair offsets of random ball pairs, jittered
    rng = np.random.default_rng(21)
    ia, ib = rng.integers(0, len(A), 64), rng.integers(0, len(B), 64)
    t = A[ia, :3] - B[ib, :3] @ R.T + rng.normal(0, 0.02, (64, 3))
    s1 = oracle.o1_points(A, B, R, t)
    full = 3 * (g.n // 2 - 1) ** 2
    s_full, _ = c.query(q[0], t, full)
    s_full = s_full.double().cpu().numpy()
    t_many = rng.uniform(-0.5, 0.5, (1024, 3))
    rows = []
    for r2 in (4, 25, 100, 400, 1600, full):
        sq, nm = c.query(q[0], t, r2)
        sq = sq.double().cpu().numpy()
        times = {}
        for name, tt in (("1", t[:1]), ("1024", t_many)):
            out = torch.empty(len(tt), dtype=torch.float32, device=dev)
            for _ in range(args.warmup):
                pkg.corr_query(c.ctx, q[0], tt, r2, out.data_ptr())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                pkg.corr_query(c.ctx, q[0], tt, r2, out.data_ptr())
            torch.cuda.synchronize()
            times[name] = (time.perf_counter() - t0) * 1e6 / args.steps
        rows.append({"mode_radius2": r2, "modes": nm, "us_per_call_1_translation": times["1"],
                     "us_per_call_1024_translations": times["1024"],
                     "err_vs_full_band": float(np.abs(sq - s_full).max() / np.abs(s_full).max()),
                     "err_vs_plain_lens_sum": float(np.abs(sq - s1).max() / np.abs(s1).max())})
        print("mode radius^2 %d: %d modes, %.1f us" % (r2, nm, times["1"]), file=sys.stderr, flush=True)
    c.close()
    print(json.dumps({"metric": "single-configuration query time (Parseval sum over the modes |m|^2 <= r2)",
                      "unit": "us per call", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": "single rotation, 4096+4096 mixture balls, n = 128 spectrum of A; "
                                             "64 near-contact translations for the errors"},
                      "rows": rows}), flush=True)


def run_slices(args, torch, pkg):
    """Offset slices and obstacle masks: time per pass for 1, 4 and 8 slices of
    A's balls offset by delta in [0, 0.02], writing every slice's scores and
    peaks, or only its obstacle bits and count; B is spread once per rotation."""
    dev = torch.device("cuda:0")
    rows = []
    for name, case in (("single rotation, 4096+4096 mixture balls, n = 128", synth.single_rotation_case),
                       ("512 rotations, 20000+2000 mixture balls, n = 64", synth.batched_rotations_case)):
        A, B, q, g = case()
        g = synth.grid_for(A, B, g.n, pad=0.04)
        c = pkg.Correlator(A, B, g.n, g.box, g.origin, device=dev)
        n, R = g.n, len(q)

        def timed(f):
            for _ in range(args.warmup):
                f()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                f()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3 / args.steps

        s = torch.empty((R, n, n, n), dtype=torch.float32, device=dev)
        pv = torch.empty(R, dtype=torch.float32, device=dev)
        pi = torch.empty(R, dtype=torch.int64, device=dev)
        t_plain = timed(lambda: pkg.corr_eval(c.ctx, q, s.data_ptr(), pv.data_ptr(), pi.data_ptr()))
        thr = 0.01 * float(pv.max().item())
        del s
        row = {"workload": name, "rotations": R, "ms_corr_eval": t_plain, "threshold": thr, "slices": []}
        for K in (1, 4, 8):
            c.set_offsets(np.linspace(0.0, 0.02, K))
            sc = torch.empty((K, R, n, n, n), dtype=torch.float32, device=dev)
            pvk = torch.empty((K, R), dtype=torch.float32, device=dev)
            pik = torch.empty((K, R), dtype=torch.int64, device=dev)
            mk = torch.empty((K, R, n ** 3 // 32), dtype=torch.int32, device=dev)
            ck = torch.empty((K, R), dtype=torch.int64, device=dev)
            t_sc = timed(lambda: pkg.corr_eval_slices(c.ctx, q, sc.data_ptr(), pvk.data_ptr(), pik.data_ptr()))
            del sc
            t_ob = timed(lambda: pkg.corr_eval_slices(c.ctx, q, None, None, None, mk.data_ptr(), ck.data_ptr(), thr))
            row["slices"].append({"slices": K, "ms_scores_and_peaks": t_sc, "ms_obstacle_bits_only": t_ob,
                                  "slice_rot_trans_per_s_obstacle": K * R * n ** 3 / (t_ob * 1e-3),
                                  "obstacle_fraction": float(ck.sum().item()) / (K * R * n ** 3)})
            print("%s: %d slices: %.3f ms with scores, %.3f ms obstacle only" % (name, K, t_sc, t_ob),
                  file=sys.stderr, flush=True)
        s1, s8 = row["slices"][0], row["slices"][-1]
        row["ms_per_extra_slice_scores"] = (s8["ms_scores_and_peaks"] - s1["ms_scores_and_peaks"]) / 7
        row["ms_per_extra_slice_obstacle"] = (s8["ms_obstacle_bits_only"] - s1["ms_obstacle_bits_only"]) / 7
        rows.append(row)
        c.close()
    print(json.dumps({"metric": "offset slices: time per pass (B spread once, product and inverse per slice)",
                      "unit": "ms", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                      "steps": args.steps, "warmup": args.warmup, "dtype": "f32",
                      "config": {"workload": "offsets linspace(0, 0.02, K) on A's balls; box padded by 0.04; "
                                             "obstacle threshold 1 % of the unoffset peak"},
                      "rows": rows}), flush=True)


def _timed(torch, f, warmup, steps):
    for _ in range(warmup):
        f()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def _o2_rel(A, B, q, g, s_gpu):
    """max |s_gpu - s_o2| / max |s_o2| against the FP64 band-limited oracle."""
    import oracle
    FA = oracle.o2_spectrum(A, np.eye(3), g.n, g.box)
    FB = oracle.o2_spectrum(B, oracle.quat_to_rot(q), g.n, g.box)
    ref = oracle.o2_scores_from_spectra(FA, FB, g.box, g.origin)
    return float(np.abs(s_gpu - ref).max() / np.abs(ref).max())


def measure_batched(args, torch, pkg, sample=(0, 255, 511)):
    """Batched rotations: 20000 + 2000 mixture balls, 512 rotations, n = 64, all
    in one corr_eval call.  Timed launch by launch with the default launch
    shapes, as one replayed hipGraph, and as a graph after the autotuner; the
    error against the FP64 oracle is taken on sampled rotations."""
    dev = torch.device("cuda:0")
    A, B, q, g = synth.batched_rotations_case()
    R, n = len(q), g.n
    c = pkg.Correlator(A, B, n, g.box, g.origin, device=dev)
    s = torch.empty((R, n, n, n), dtype=torch.float32, device=dev)
    pv = torch.empty(R, dtype=torch.float32, device=dev)
    pi = torch.empty(R, dtype=torch.int64, device=dev)

    def step():
        pkg.corr_eval(c.ctx, q, s.data_ptr(), pv.data_ptr(), pi.data_ptr())

    rows = {}
    rows["default"] = (_timed(torch, step, args.warmup, args.steps), c.tuning())
    c.set_tuning(graph=1)
    rows["graph"] = (_timed(torch, step, args.warmup, args.steps), c.tuning())
    t0 = time.perf_counter()
    pkg.corr_autotune(c.ctx, q, s.data_ptr(), pv.data_ptr(), pi.data_ptr(), reps=2)
    tune_s = time.perf_counter() - t0
    rows["autotuned graph"] = (_timed(torch, step, args.warmup, args.steps), c.tuning())
    for k, (ms, t) in rows.items():
        print("batched 512 rotations, %s: %.3f ms  %s" % (k, ms, t), file=sys.stderr, flush=True)
    best = min(rows, key=lambda k: rows[k][0])
    ms = rows[best][0]
    step()
    torch.cuda.synchronize()
    errs = [_o2_rel(A, B, q[r], g, s[r].double().cpu().numpy()) for r in sample]
    out = {"metric": "rotations*translations scored/s at <=1e-4 rel err vs FP64", "value": R * n ** 3 / (ms * 1e-3),
           "unit": "rot*trans/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "512 rotations, 20000+2000 mixture balls, 64^3 translations, sigma 2, KB width 8, "
                                  "one corr_eval call (scores and peaks)", "n": n, "box": g.box,
                      "q_a": int(c.info["q_a"]), "q_b": int(c.info["q_b"])},
           "modes": {k: {"ms": v[0], "tuning": v[1]} for k, v in rows.items()}, "best_mode": best,
           "autotune_seconds": tune_s,
           "e_rel_vs_fp64_sampled": {str(r): e for r, e in zip(sample, errs)}}
    c.close()
    return out


def run_batched(args, torch, pkg):
    print(json.dumps(measure_batched(args, torch, pkg)), flush=True)


def run_uneven(args, torch, pkg):
    """Uneven batch: 64 pairs, ball counts log-uniform in [500, 50000], grids of
    32^3, 64^3 or 128^3, 32 rotations each, in one corr_batch_eval call (one
    hipGraph launch when replayed); the error against the FP64 oracle of
    rotation 0 of every pair."""
    dev = torch.device("cuda:0")
    cases = synth.uneven_batch_case()
    b = pkg.Batch([(A, B, g.n, g.box, g.origin) for A, B, q, g in cases], device=dev)
    quats = [q for A, B, q, g in cases]
    ns = [g.n for A, B, q, g in cases]
    total_rt = sum(len(q) * n ** 3 for q, n in zip(quats, ns))
    s = torch.empty(total_rt, dtype=torch.float32, device=dev)
    nrot = sum(len(q) for q in quats)
    pv = torch.empty(nrot, dtype=torch.float32, device=dev)
    pi = torch.empty(nrot, dtype=torch.int64, device=dev)

    def step():
        b.eval(quats, out=(s, pv, pi))

    slots = {}
    for p, n in enumerate(ns):
        slots.setdefault(str(n), set()).add(int(b.info(p)["batch"]))
    print("rotations per pass by grid size: %s" % {k: sorted(v) for k, v in slots.items()}, file=sys.stderr,
          flush=True)
    rows = {"default": _timed(torch, step, args.warmup, args.steps)}
    b.set_graph(True)
    rows["graph"] = _timed(torch, step, args.warmup, args.steps)
    for k, ms in rows.items():
        print("uneven batch, %s: %.3f ms" % (k, ms), file=sys.stderr, flush=True)
    best = min(rows, key=rows.get)
    ms = rows[best]
    step()
    torch.cuda.synchronize()
    per_pair = []
    t0 = time.perf_counter()
    off = 0
    for p, (A, B, q, g) in enumerate([] if args.no_cpu_baseline else cases):
        n3 = g.n ** 3
        e = _o2_rel(A, B, q[0], g, s[off:off + n3].view(g.n, g.n, g.n).double().cpu().numpy())
        per_pair.append({"pair": p, "n": g.n, "n_a": len(A), "n_b": len(B), "e_rel_rot0": e})
        off += len(q) * n3
        if p % 8 == 7:
            print("oracle: %d pairs checked, worst e_rel %.3g" % (p + 1, max(r["e_rel_rot0"] for r in per_pair)),
                  file=sys.stderr, flush=True)
    out = {"metric": "rotations*translations scored/s at <=1e-4 rel err vs FP64", "value": total_rt / (ms * 1e-3),
           "unit": "rot*trans/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "uneven batch: 64 pairs, ball counts log-uniform in [500, 50000], grids 32/64/128, "
                                  "32 rotations each, one corr_batch_eval call (scores and peaks)",
                      "pairs_per_n": {str(n): ns.count(n) for n in (32, 64, 128)}, "correlations": nrot},
           "modes_ms": rows, "best_mode": best,
           "rotations_per_pass_by_n": {k: sorted(v) for k, v in slots.items()},
           "e_rel_vs_fp64_worst": max((r["e_rel_rot0"] for r in per_pair), default=None),
           "oracle_seconds": time.perf_counter() - t0,
           "per_pair": per_pair}
    b.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default launch shapes instead of autotuning them first")
    ap.add_argument("--tuning", type=str, default=None, metavar="K=V,...",
                    help="fixed launch shapes (corr_tuning fields), e.g. spread_wgs=384,cols_y=16; skips the autotuner")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 512-rotation batched workload that the default run also reports")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (reference for hardware byte counters)")
    ap.add_argument("--proposal", action="store_true",
                    help="run the rotation-proposal workflow instead (recall and speed-up vs exhaustive search)")
    ap.add_argument("--proposal-pairs", type=int, default=100)
    ap.add_argument("--proposal-schedule", type=str, default="250:1e-3,100:3e-4,50:1e-4",
                    help="training phases EPOCHS:LR,... (Adam state carries over)")
    ap.add_argument("--proposal-beta", type=float, default=0.0,
                    help="target map exp(beta z) of the per-pair standardised peaks (0: none)")
    ap.add_argument("--query", action="store_true",
                    help="time single-configuration queries (Sec. 4.1) instead, by number of modes")
    ap.add_argument("--slices", action="store_true",
                    help="time offset slices and obstacle masks (corr_eval_slices) instead")
    ap.add_argument("--batched", action="store_true",
                    help="time 512 rotations of a 20000 + 2000 ball pair at n = 64 (eager, graph, autotuned) instead")
    ap.add_argument("--uneven", action="store_true",
                    help="time the 64-pair uneven batch (eager, graph) and check every pair against the oracle instead")
    ap.add_argument("--sc", type=str, default=None, metavar="R0,LAMBDA",
                    help="score shape complementarity (skin offset R0, penalty LAMBDA) instead of the overlap")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1711_05075_amd as pkg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        # a plain copy kernel of known size: reads and writes `nbytes` per launch
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.warmup + args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": args.warmup + args.steps}), flush=True)
        return
    if args.proposal:
        run_proposal(args, torch, pkg)
        return
    if args.query:
        run_query(args, torch, pkg)
        return
    if args.slices:
        run_slices(args, torch, pkg)
        return
    if args.batched:
        run_batched(args, torch, pkg)
        return
    if args.uneven:
        run_uneven(args, torch, pkg)
        return
    A, B, q, g = synth.single_rotation_case()
    sc = tuple(float(v) for v in args.sc.split(",")) if args.sc else None
    if sc:
        g = synth.grid_for(A, B, g.n, pad=2 * sc[0])
    c = pkg.Correlator(A, B, g.n, g.box, g.origin, device=dev, sc=sc)
    n = g.n
    scores = torch.empty((1, n, n, n), dtype=torch.float32, device=dev)
    pv = torch.empty(1, dtype=torch.float32, device=dev)
    pi = torch.empty(1, dtype=torch.int64, device=dev)

    def step():
        pkg.corr_prepare_a(c.ctx)
        pkg.corr_eval(c.ctx, q, scores.data_ptr(), pv.data_ptr(), pi.data_ptr())

    # launch shapes: fixed by --tuning, or chosen by the library's autotuner for
    # this very step (A's spectrum + one rotation), or the defaults
    tune_s = None
    if args.tuning:
        c.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))})
        tuning_source = "fixed (--tuning)"
    elif args.no_autotune:
        tuning_source = "defaults"
    else:
        t0 = time.perf_counter()
        pkg.corr_autotune(c.ctx, q, scores.data_ptr(), pv.data_ptr(), pi.data_ptr(), reps=10, with_a=True)
        tune_s = time.perf_counter() - t0
        tuning_source = "autotuned on corr_prepare_a + corr_eval"

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    pkg.corr_profile(c.ctx, True)
    pkg.corr_profile_read(c.ctx)  # clear
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pkg.corr_profile_read(c.ctx)
    pkg.corr_profile(c.ctx, False)

    # throughput without the profiling events (second timed pass, same work)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ms_step = (t3 - t2) * 1e3 / args.steps
    rot_trans = n ** 3  # one rotation per step
    value = rot_trans / (ms_step * 1e-3)

    info = c.info
    pkg.corr_prepare_a(c.ctx)
    pass_a = c.pass_info()
    pkg.corr_eval(c.ctx, q, scores.data_ptr(), pv.data_ptr(), pi.data_ptr())
    pass_b = c.pass_info()
    nbytes = stage_bytes(info, pass_a, pass_b)
    dom = max((k for k in prof if prof[k][1] > 0), key=lambda k: prof[k][0])
    dom_ms = prof[dom][0] / prof[dom][1]
    dom_bytes = nbytes.get(dom)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9 if dom_bytes else None
    # the committed counters were taken on the default (overlap) workload
    traffic = measured_traffic() if dom == "spread_fft_x" and not sc else None

    out = {
        "metric": ("shape-complementarity " if sc else "") + "rotations*translations scored/s at <=1e-4 rel err vs FP64",
        "value": value,
        "unit": "rot*trans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single rotation, 4096+4096 mixture balls, 128^3 translations, sigma 2, KB width 8"
                               + (", complementarity r0 = %g, lambda = %g" % sc if sc else ""),
                   "n_a": int(info["n_a"]), "n_b": int(info["n_b"]), "n": n, "box": g.box,
                   "q_a": int(info["q_a"]), "q_b": int(info["q_b"])},
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in prof.items() if v[1]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                     "alg_bytes_per_launch": dom_bytes, "mean_launch_ms": dom_ms},
        "tuning": c.tuning(), "tuning_source": tuning_source, "autotune_seconds": tune_s,
        "occupancy": {"a": {k: pass_a[k] for k in ("tiles", "live_tiles", "live_rows")},
                      "b": {k: pass_b[k] for k in ("tiles", "live_tiles", "live_rows")}},
    }

    if not args.no_cpu_baseline:
        import oracle
        s_gpu = scores[0].double().cpu().numpy()
        threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
        t4 = time.perf_counter()
        if sc:
            FA = oracle.o2_sc_spectrum(A, np.eye(3), n, g.box, *sc)
            FB = oracle.o2_sc_spectrum(B, oracle.quat_to_rot(q[0]), n, g.box, *sc)
        else:
            FA = oracle.o2_spectrum(A, np.eye(3), n, g.box)
            FB = oracle.o2_spectrum(B, oracle.quat_to_rot(q[0]), n, g.box)
        ref = oracle.o2_scores_from_spectra(FA, FB, g.box, g.origin)
        t5 = time.perf_counter()
        out["cpu_baseline"] = {"value": rot_trans / (t5 - t4), "unit": "rot*trans/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "FP64 band-limited oracle (direct NDFT of both shapes + FP64 inverse FFT), "
                                         "one rotation of the same workload, full 128^3 grid"}
        out["e_rel_vs_fp64"] = float(np.abs(s_gpu - ref).max() / np.abs(ref).max())
    c.close()
    if not args.no_batched and not sc:
        # the batched-rotations workload as well, so that one run reports both
        b = measure_batched(args, torch, pkg, sample=(0,))
        out["batched"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "config", "best_mode", "modes",
                                            "autotune_seconds", "e_rel_vs_fp64_sampled")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
