"""Short text summaries of rocprofv3 output.

  python -m paper_1711_05075_amd.rocprof_summary stats <kernel_stats.csv> <out.txt> "<title>" "<command>"
      [<kernel_trace.csv> <kernel regex> <K>]
      per-kernel call counts and durations from a --kernel-trace --stats run;
      with a kernel trace, also the mean duration of every dispatch of the
      kernels matching the regex (all their instantiations together) and of
      the last K of them, the launches a program timed itself at its end;

  python -m paper_1711_05075_amd.rocprof_summary traffic <kernel regex> <fetch.csv> <write.csv>
      <copy_fetch.csv> <copy_write.csv> <copy bytes> <out.txt> "<commands>"
      HBM bytes per launch of one kernel from FETCH_SIZE and WRITE_SIZE counter
      runs (KiB per dispatch), each scaled by what the same counter reads for a
      plain copy kernel that reads and writes <copy bytes> per launch; records
      the SHA-256 of the kernel source the counters were taken on.
"""
import csv
import hashlib
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCE = os.path.join(ROOT, "paper_1711_05075_amd", "csrc", "corr_kernels.hip")


def kernel_source_digest(text=None):
    """SHA-256 of the source the spreading kernel is compiled from: the kernel
    file up to the end of k_spread_fftx (the column FFT engine, the sort and
    spreading code), so that later kernels in the file do not void counters
    taken on it."""
    if text is None:
        text = open(KERNEL_SOURCE).read()
    end = text.index("// Index of kept output mode")
    return hashlib.sha256(text[:end].encode()).hexdigest()


def _short(name):
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    return re.sub(r"^void ", "", name).split("(")[0].split("::")[-1]


def family(trace, regex, last):
    """Mean duration (us) of all dispatches of the kernels matching regex in a
    kernel-trace CSV, and of the last `last` of them by start time."""
    d = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
               for r in csv.DictReader(open(trace)) if re.search(regex, r["Kernel_Name"]))
    if len(d) < last:
        raise SystemExit("only %d dispatches of /%s/ in %s" % (len(d), regex, trace))
    tail = d[len(d) - last:]
    return len(d), sum(x for _, x in d) / len(d) / 1e3, sum(x for _, x in tail) / last / 1e3


def stats(src, dst, title, cmd, trace=None, regex=None, last=None):
    rows = list(csv.DictReader(open(src)))
    lines = ["# " + title, "#", "# command (one MI355X, repository root):", "#   " + cmd,
             "# durations in microseconds, from rocprofv3 --kernel-trace --stats", "",
             "%-26s %6s %12s %10s %7s" % ("kernel", "calls", "total_us", "avg_us", "pct")]
    for r in rows:
        lines.append("%-26s %6s %12.1f %10.1f %7.2f" % (_short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e3,
                                                         float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    if trace:
        last = int(last)
        n, avg, tail = family(trace, regex, last)
        lines += ["", "# kernels matching /%s/, every instantiation together (kernel trace):" % regex,
                  "family_dispatches: %d" % n, "family_avg_us: %.1f" % avg,
                  "family_last_%d_avg_us: %.1f" % (last, tail)]
    open(dst, "w").write("\n".join(lines) + "\n")


def _counter(path, regex, counter):
    """Mean counter value (KiB) per dispatch of the kernels matching regex."""
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter and re.search(regex, r["Kernel_Name"]):
            vals[r["Dispatch_Id"]] = vals.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    if not vals:
        raise SystemExit("no %s rows for /%s/ in %s" % (counter, regex, path))
    return sum(vals.values()) / len(vals), len(vals)


def traffic(regex, fetch, write, cfetch, cwrite, copy_bytes, dst, cmds):
    copy_bytes = float(copy_bytes)
    f_kib, nf = _counter(fetch, regex, "FETCH_SIZE")
    w_kib, nw = _counter(write, regex, "WRITE_SIZE")
    cf_kib, _ = _counter(cfetch, "copyBuffer", "FETCH_SIZE")
    cw_kib, _ = _counter(cwrite, "copyBuffer", "WRITE_SIZE")
    kf, kw = copy_bytes / (cf_kib * 1024), copy_bytes / (cw_kib * 1024)
    total = kf * f_kib * 1024 + kw * w_kib * 1024
    sha = kernel_source_digest()
    lines = ["# HBM traffic per launch of kernels matching /%s/" % regex, "#",
             "# commands (one MI355X, repository root; one counter per run):"]
    lines += ["#   " + c for c in cmds.split(";;")]
    lines += ["#",
              "# kernel_source_sha256 covers corr_kernels.hip up to the end of k_spread_fftx.",
              "# FETCH_SIZE and WRITE_SIZE are KiB per dispatch; each is scaled by what it",
              "# reads for a plain copy of %d bytes per launch." % copy_bytes, "",
              "dispatches_fetch: %d" % nf, "dispatches_write: %d" % nw,
              "fetch_kib_per_launch: %.1f" % f_kib, "write_kib_per_launch: %.1f" % w_kib,
              "copy_fetch_kib: %.1f" % cf_kib, "copy_write_kib: %.1f" % cw_kib,
              "fetch_scale: %.4f" % kf, "write_scale: %.4f" % kw,
              "hbm_bytes_per_launch: %.0f" % total,
              "kernel_source_sha256: %s" % sha]
    open(dst, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:9])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:10])
    else:
        raise SystemExit(__doc__)
