"""Benchmark: rotation x translation scores per second on one MI355X.

Default workload: one rotation of two 4096-ball Gaussian-mixture shapes (radii
lognormal(ln 0.02, 0.3)) on a 128^3 translation grid, 2x oversampled spreading
grid, Kaiser-Bessel window of width 8.  One step = the whole pipeline for that
rotation including the fixed shape's spectrum (corr_prepare_a + corr_eval with
scores and peaks), inputs resident on the device.

Prints one JSON line with the throughput, the dominant kernel's roofline
(algorithmic bytes per launch / its mean event-timed duration) and the FP64
oracle timed on the host for one rotation of the same workload.
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


KERNEL_SOURCE = os.path.join(ROOT, "paper_1711_05075_amd", "csrc", "corr_kernels.hip")
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
    import hashlib
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    fields = {}
    for line in open(TRAFFIC_SUMMARY):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != src:
        return None
    return float(fields["hbm_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (reference for hardware byte counters)")
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
    A, B, q, g = synth.single_rotation_case()
    c = pkg.Correlator(A, B, g.n, g.box, g.origin, device=dev)
    n = g.n
    scores = torch.empty((1, n, n, n), dtype=torch.float32, device=dev)
    pv = torch.empty(1, dtype=torch.float32, device=dev)
    pi = torch.empty(1, dtype=torch.int64, device=dev)

    def step():
        pkg.corr_prepare_a(c.ctx)
        pkg.corr_eval(c.ctx, q, scores.data_ptr(), pv.data_ptr(), pi.data_ptr())

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
    traffic = measured_traffic() if dom == "spread_fft_x" else None

    out = {
        "metric": "rotations*translations scored/s at <=1e-4 rel err vs FP64",
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
        "config": {"workload": "single rotation, 4096+4096 mixture balls, 128^3 translations, sigma 2, KB width 8",
                   "n_a": int(info["n_a"]), "n_b": int(info["n_b"]), "n": n, "box": g.box,
                   "q_a": int(info["q_a"]), "q_b": int(info["q_b"])},
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in prof.items() if v[1]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                     "alg_bytes_per_launch": dom_bytes, "mean_launch_ms": dom_ms},
        "occupancy": {"a": {k: pass_a[k] for k in ("tiles", "live_tiles", "live_rows")},
                      "b": {k: pass_b[k] for k in ("tiles", "live_tiles", "live_rows")}},
    }

    if not args.no_cpu_baseline:
        import oracle
        s_gpu = scores[0].double().cpu().numpy()
        threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
        t4 = time.perf_counter()
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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
